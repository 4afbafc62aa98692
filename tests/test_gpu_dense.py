"""Dense long-range potential on MFMA (KMC_BF16X2) against the binary64 oracle
(needs an MI355X).

Error bound of phi.  Each kernel value is represented as hi + lo with
|K - hi - lo| <= 2^-16 |K|; the occupancy weights (0, 1, 2) are exact.  The
FP32 accumulation of n = 2 (m + 1) Lp products (both halves) rounds at most n
times, each by at most 2^-24 of the running sum, which never exceeds
sum_j occ_j |K| = phi_abs.  So
    |phi_gpu - phi_64| <= (2^-16 + n 2^-24) phi_abs,
with phi_abs = phi_64 for kappa > 0 (all K > 0).  The decisions then use
dE = e_app + phi(t) - K(1,0) - phi(o) in binary32: trajectories equal the
binary64 oracle's except where |u - p| is below the resulting error of p,
far inside the logged 1e-6 window; the lockstep harness resynchronises only
there."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import BF16X2, FP64, Physics, c4_dense, constant, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _bound(m, L):
    lp = (L + 127) // 128 * 128
    return 2.0 ** -16 + 2 * (m + 1) * lp * 2.0 ** -24


@pytest.mark.parametrize("rails,L,m,cut,lam", [
    ([150, 7], 96, 4, 95, 0.0),      # two devices, a partial 128-rail tile, small device wraps
    ([40], 512, 4, 511, 0.0),        # the dense configuration's rail length
    ([33], 200, 1, 16, 4.0),         # screened, cutoff shorter than the rail
    ([5], 1000, 2, 999, 0.0),        # rail range covering the whole (small) ring
])
def test_dense_potential_matches_oracle(rails, L, m, cut, lam):
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=BF16X2, seed=4, coulomb_kappa_v=0.025, screening_sites=lam, cutoff_sites=cut,
                 rail_range=m)
    sites = [L] * len(rails)
    sim = Simulator(ph, rails, sites)
    sim.fill_random([0.3] * len(rails))
    occ = sim.read_occupancy()
    phi = sim.dense_potential().cpu().numpy().astype(np.float64)
    ref = oracle.dense_potential(oracle.OracleParams(ph.replace(precision=FP64), rails, sites), occ)
    err = np.abs(phi - ref)
    assert np.all(err <= _bound(m, L) * ref + 1e-30), (err.max(), (err / ref).max())
    assert (err / ref).max() < 1e-4


@pytest.mark.parametrize("R,L,m,protocol", [(16, 64, 4, constant(0.8)), (24, 128, 4, triangle(1.0, 150e-12))])
def test_dense_trajectory_follows_fp64_oracle(R, L, m, protocol):
    """Unscreened 1/r over the whole rail and +-m rails, validation barrier:
    step-by-step equality with the binary64 oracle, resynchronised only in
    chunks where both logged a near-threshold draw."""
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=BF16X2, seed=8, ea_ev=0.15, screening_sites=0.0, cutoff_sites=L - 1, rail_range=m)
    ph64 = ph.replace(precision=FP64)
    sim = Simulator(ph, [R, R], [L, L])
    p_or = oracle.OracleParams(ph64, [R, R], [L, L])
    occ0 = oracle.fill(p_or, [0.3, 0.2])
    sim.load_occupancy(occ0)
    sim.set_protocols([protocol, constant(-0.5)])
    st = lockstep(sim, p_or, [protocol, constant(-0.5)], occ0, 200, 25, max_resync=3)
    assert st["hops"] > 100
    assert st["resyncs"] <= 3


def test_c4_full_size_sampled():
    """64 replicas x 1024 rails x 512 sites after a few steps: the potential on
    sampled rails against the binary64 oracle.  The potential of a rail only
    involves the rails within +-4, so the oracle evaluates a 17-rail strip
    centred on it (wrap distance 8 > 4: the same neighbours as in the ring)."""
    from paper_2511_09413_amd import Simulator
    wl = c4_dense(n_steps=4)
    R, L = wl.rails[0], wl.sites[0]
    sim = Simulator(wl.physics, wl.rails, wl.sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    sim.run_steps(4)
    occ = sim.read_occupancy().reshape(len(wl.rails), R, L)
    phi = sim.dense_potential().cpu().numpy().astype(np.float64).reshape(len(wl.rails), R, L)
    p_strip = oracle.OracleParams(wl.physics.replace(precision=FP64), [17], [L])
    for d, r in ((0, 0), (0, 513), (37, 1023), (63, 200)):
        strip = occ[d, [(r + k) % R for k in range(-8, 9)]]
        ref = oracle.dense_potential(p_strip, strip).reshape(17, L)[8]
        err = np.abs(phi[d, r] - ref)
        assert np.all(err <= _bound(4, L) * ref), (d, r, err.max())
