"""Open electrodes and deep traps on the GPU against the oracle (needs an
MI355X).

* Open electrodes (kmc_set_electrodes): every rail end is one more bond to a
  reservoir; the trajectories, per-step net counts (interior hops and
  transfers) and deciles follow the oracle in lockstep (binary64 and
  binary32, both parities of the rail length, one device open and one closed,
  per-site barriers, wider windows).  The ion number changes.
* Deep traps (a few sites with raised barriers, the paper's suggestion for the
  charge trapping of scarce defects): lockstep with the oracle in the wave
  kernel (the automatic strategy), and the dwell time of lone ions on traps
  against its exact law (1 - p)^(2k) (see the oracle's pins)."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import BF16X2, FP32, FP64, Physics, constant, gaussian_barriers, sparse_traps, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _open_case(ph, rails, sites, filling, protocols, el_per_device, steps, chunk, ea=None):
    from paper_2511_09413_amd import Simulator
    sim = Simulator(ph, rails, sites, ea=ea)
    for d, el in enumerate(el_per_device):
        if el is not None:
            sim.set_electrodes(*el, device=d)
    assert sim.launch_mode == "half_step"
    p_or = oracle.OracleParams(ph, rails, sites, ea)
    occ0 = oracle.fill(p_or, filling)
    sim.load_occupancy(occ0)
    sim.set_protocols(protocols)
    st = lockstep(sim, p_or, protocols, occ0, steps, chunk, electrodes=el_per_device)
    assert st["resyncs"] == 0 and st["gpu_log"] == st["oracle_log"]
    occ = sim.read_occupancy()
    return sim, st, occ0, occ


@pytest.mark.parametrize("case", ["fp64_even", "fp32_two_devices", "fp64_barriers_wide"])
def test_open_electrodes_follow_oracle(case):
    if case == "fp64_even":
        ph = Physics(precision=FP64, seed=3, ea_ev=0.15)
        rails, sites = [16], [40]
        el = [(0.12, 0.08, 0.12, -0.08)]
        sim, st, occ0, occ = _open_case(ph, rails, sites, [0.3], [constant(1.0)], el, 300, 100)
    elif case == "fp32_two_devices":
        ph = Physics(precision=FP32, seed=4, ea_ev=0.14)
        rails, sites = [10, 7], [33, 50]
        el = [(0.1, 0.1, 0.15, 0.0), None]
        sim, st, occ0, occ = _open_case(ph, rails, sites, [0.2, 0.4], [triangle(1.5, 200e-12), constant(-0.6)], el,
                                        300, 60)
        # the closed device keeps its ion count rail by rail
        n0 = rails[0] * sites[0]
        o0, o1 = occ0[n0:].reshape(7, 50), occ[n0:].reshape(7, 50)
        assert np.array_equal(o0.sum(axis=1), o1.sum(axis=1))
    else:
        ph = Physics(precision=FP64, seed=5, ea_ev=0.14, rail_range=2, cutoff_sites=40, screening_sites=2.0,
                     coulomb_kappa_v=0.04)
        rails, sites = [9], [61]
        ea = gaussian_barriers((9, 61), 0.14, 0.01, seed=7, dtype=np.float64)
        el = [(0.09, 0.05, 0.11, 0.02)]
        sim, st, occ0, occ = _open_case(ph, rails, sites, [0.35], [constant(0.7)], el, 200, 50, ea=ea)
    assert int(occ.sum()) != int(occ0.sum())          # the ion number is free
    assert st["hops"] > 50
    print(f"{case}: ions {int(occ0.sum())} -> {int(occ.sum())}, |net| sum {st['hops']}, "
          f"near-threshold draws {st['oracle_log']}")
    sim.close()


def test_closing_electrodes_restores_the_default_strategy():
    from paper_2511_09413_amd import KMC_EUNSUPPORTED, KmcError, Simulator
    from workloads import c1_plain_fp64
    wl = c1_plain_fp64()
    sim = Simulator(wl.physics, wl.rails, wl.sites)
    auto = sim.launch_mode
    sim.set_electrodes(0.1, 0.0, 0.1, 0.0)
    assert sim.launch_mode == "half_step"
    occ = sim.snapshot()
    with pytest.raises(KmcError) as err:
        sim.score_replay(occ, 0, np.ones((4, 1)))
    assert err.value.status == KMC_EUNSUPPORTED
    sim.set_electrodes(0.1, 0.0, 0.1, 0.0, open=False)
    assert sim.launch_mode == auto
    sim.close()
    dense = Simulator(Physics(precision=BF16X2, screening_sites=0.0, cutoff_sites=63, rail_range=4), [8], [64])
    with pytest.raises(KmcError) as err:
        dense.set_electrodes(0.1, 0.0, 0.1, 0.0)
    assert err.value.status == KMC_EUNSUPPORTED
    dense.close()


def test_deep_traps_follow_oracle_in_the_wave_kernel():
    """128 x 1024 rails, binary32, barriers N(0.15, 0.01) eV with 0.5 % of the
    sites 0.25 eV deeper; the automatic (wave) strategy against the oracle."""
    from paper_2511_09413_amd import Simulator
    R, L = 128, 1024
    base = gaussian_barriers((R, L), 0.15, 0.01, seed=8, dtype=np.float64)
    ea = sparse_traps((R, L), 0.0, 0.005, 0.25, seed=9, dtype=np.float32, field=base)
    ph = Physics(precision=FP32, seed=12, ea_ev=0.15)
    sim = Simulator(ph, [R], [L], ea=ea)
    assert sim.launch_mode == "wave"
    p_or = oracle.OracleParams(ph, [R], [L], ea)
    occ0 = oracle.fill(p_or, [0.3])
    sim.load_occupancy(occ0)
    sim.set_protocols([constant(0.8)])
    st = lockstep(sim, p_or, [constant(0.8)], occ0, 400, 200)
    assert st["resyncs"] == 0 and st["hops"] > 200
    print(f"traps 128x1024: |net| sum {st['hops']}, near-threshold draws {st['oracle_log']}")
    sim.close()


def test_trap_dwell_time_law_on_gpu():
    """Lone ions on trap sites (no ion-ion coupling, no bias): the fraction
    still on their trap after k steps against (1 - p)^(2k) within 4 standard
    errors, p = nu0 dt exp(-Ea_trap / kT)."""
    from paper_2511_09413_amd import Simulator
    R, L, trap = 20000, 24, 11
    ph = Physics(precision=FP64, ea_ev=0.05, coulomb_kappa_v=0.0, seed=23)
    ea_trap = 0.12
    ea = np.full((R, L), 0.05)
    ea[:, trap] = ea_trap
    occ = np.zeros((R, L), dtype=np.int8)
    occ[:, trap] = 1
    sim = Simulator(ph, [R], [L], ea=ea.reshape(-1))
    sim.load_occupancy(occ.reshape(-1))
    p = min(ph.nu0_hz * ph.dt_s * math.exp(-ea_trap / ph.kT_ev), 1.0)
    stayed = np.ones(R, dtype=bool)
    for k in range(1, 25):
        sim.run_steps(1)
        stayed &= sim.read_occupancy().reshape(R, L)[:, trap] == 1
        expect = (1.0 - p) ** (2 * k)
        se = math.sqrt(expect * (1 - expect) / R)
        assert abs(stayed.mean() - expect) < 4 * se, (k, stayed.mean(), expect, se)
    print(f"dwell: survival after 24 steps {stayed.mean():.4f} against {(1 - p) ** 48:.4f}")
    sim.close()
