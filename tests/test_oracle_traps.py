"""Deep traps in the oracle (CPU only): a trap is a site whose barrier is
raised (the origin-barrier reading of per-site barriers), as the paper's
conclusion suggests for the charge trapping of scarce defects.

Pinned here: with no ion-ion coupling and no bias, a lone ion on a trap site
with free neighbours attempts one hop per half-step (its left bond in one
parity, its right bond in the other), each with the same probability
p = min(nu0 dt exp(-Ea_trap / kT), 1), and cannot come back within the step it
left in.  So the number of whole steps it stays is geometric: it is still there
after k steps with probability (1 - p)^(2k), exactly.  The test checks the
survival fraction over many independent rails against this law (4 standard
errors at every k), in both precisions, and that the traps generator places
exactly round(fraction x sites) traps of the given depth."""
import math

import numpy as np
import pytest

import oracle
from workloads import FP32, FP64, Physics, constant, sparse_traps


def test_sparse_traps_generator():
    ea = sparse_traps((40, 50), 0.3, 0.01, 0.25, seed=3, dtype=np.float64)
    assert ea.shape == (2000,)
    assert int(np.isclose(ea, 0.55).sum()) == 20 and int(np.isclose(ea, 0.3).sum()) == 1980
    again = sparse_traps((40, 50), 0.3, 0.01, 0.25, seed=3, dtype=np.float64)
    assert np.array_equal(ea, again)
    base = np.linspace(0.2, 0.3, 2000)
    ea2 = sparse_traps((40, 50), 0.0, 0.01, 0.25, seed=3, dtype=np.float64, field=base)
    assert np.allclose(ea2 - base, np.where(np.isclose(ea, 0.55), 0.25, 0.0))


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_lone_ion_dwell_time_in_a_trap(precision):
    R, L, trap = 6000, 24, 11
    ph = Physics(precision=precision, ea_ev=0.05, coulomb_kappa_v=0.0, seed=21)
    ea_trap = 0.12
    ea = np.full((R, L), 0.05)
    ea[:, trap] = ea_trap
    p_or = oracle.OracleParams(ph, [R], [L], ea.reshape(-1))
    occ = np.zeros((R, L), dtype=np.int8)
    occ[:, trap] = 1
    occ = occ.reshape(-1)
    p = min(ph.nu0_hz * ph.dt_s * math.exp(-ea_trap / ph.kT_ev), 1.0)
    stayed = np.ones(R, dtype=bool)
    for k in range(1, 13):
        oracle.run(p_or, [constant(0.0)], occ, k - 1, 1, want_dec=False)
        stayed &= occ.reshape(R, L)[:, trap] == 1
        expect = (1.0 - p) ** (2 * k)
        se = math.sqrt(expect * (1 - expect) / R)
        assert abs(stayed.mean() - expect) < 4 * se + 1e-12, (k, stayed.mean(), expect, se)
    assert 0.2 < stayed.mean() < 0.8      # the law is tested where it has power
