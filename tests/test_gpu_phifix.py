"""Long-range potential kept hop by hop in fixed point (KMC_PHI_FIXED) against
the binary64 oracle (needs an MI355X).

What is exact and what is bounded.  Every kernel value is rounded once to a
multiple of 2^-F V (F <= 52, chosen by the library so that no sum can exceed
2^61 units), and the potential is the exact integer sum of those values over
the ions of the window.  Integer sums do not depend on their order, so the
potential kept up to date by thousands of hops equals the one computed from
scratch bit for bit (checked after every run below).  Against the binary64
potential of the oracle the difference is at most the n rounded terms,
    |2^-F phi_fix - phi_64| <= n 2^-(F+1) + 2^-50 phi_64
(the second term covers the oracle's own binary64 summation).  A decision
uses dE_coul = 2^-F (phi(t) - K(1,0) - phi(o)), exact in the fixed-point units
and rounded once, then binary64 energies and probabilities as the oracle's
binary64 path; p differs from the oracle's by about (beta/2) n 2^-(F+1) p,
below 1e-12 p here, so a decision can differ only for a draw within that of
p, which lies inside the logged 1e-6 window.  The trajectories are therefore
compared in lockstep with the oracle's binary64 path, as the other binary64
paths are."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import FP64, PHI_FIXED, Physics, Workload, c4_dense, constant, step_then_relax, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _terms(p_or, rails, sites, m, cut):
    """Largest number of terms of one site's potential."""
    n = 0
    for R, L in zip(rails, sites):
        n = max(n, min(R, 2 * m + 1) * (2 * min(cut, L - 1) + 1))
    return n


def _check_potential(sim, ph, rails, sites):
    phi, F = sim.fixed_potential()
    fresh, F2 = sim.fixed_potential(recompute=True)
    assert F == F2 and 16 <= F <= 52
    phi = phi.cpu().numpy()
    assert np.array_equal(phi, fresh.cpu().numpy())       # hop by hop == from scratch, bit for bit
    occ = sim.read_occupancy()
    p64 = oracle.OracleParams(ph.replace(precision=FP64), rails, sites)
    ref = oracle.dense_potential(p64, occ)
    n = _terms(p64, rails, sites, ph.rail_range, ph.cutoff_sites)
    err = np.abs(np.ldexp(phi.astype(np.float64), -F) - ref)
    bound = n * 2.0 ** -(F + 1) + 2.0 ** -50 * np.abs(ref)
    assert np.all(err <= bound), (err.max(), n, F)
    return err.max(), F


@pytest.mark.parametrize("rails,sites,m,cut,lam", [
    ([40], [512], 4, 511, 0.0),            # the dense configuration's rail length and rail range
    ([12, 5], [128, 96], 4, 127, 0.0),     # two devices of different lengths, a ring shorter than 2m + 1
    ([33], [200], 1, 16, 4.0),             # screened, cutoff shorter than the rail
    ([7], [2048], 2, 40, 2.0),             # the longest rail of the path
])
def test_fixed_potential_matches_oracle(rails, sites, m, cut, lam):
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=PHI_FIXED, seed=4, coulomb_kappa_v=0.025, screening_sites=lam, cutoff_sites=cut,
                 rail_range=m)
    sim = Simulator(ph, rails, sites)
    sim.fill_random([0.3] * len(rails))
    e, F = _check_potential(sim, ph, rails, sites)
    print(f"fixed phi {rails}x{sites} m={m} cut={cut}: F={F}, max |error| {e:.3e} V")


def _lockstep_case(ph, rails, sites, filling, protocols, steps, chunk, ea=None):
    from paper_2511_09413_amd import Simulator
    sim = Simulator(ph, rails, sites, ea=ea)
    assert sim.launch_mode == "half_step"
    p_or = oracle.OracleParams(ph.replace(precision=FP64), rails, sites, ea)
    occ0 = oracle.fill(p_or, filling)
    sim.load_occupancy(occ0)
    sim.set_protocols(protocols)
    st = lockstep(sim, p_or, protocols, occ0, steps, chunk)
    assert st["resyncs"] == 0 and st["gpu_log"] == st["oracle_log"]
    _check_potential(sim, ph, rails, sites)
    return st


@pytest.mark.parametrize("case", ["dense", "two_devices", "screened_barriers", "small_ring"])
def test_trajectories_follow_fp64_oracle(case):
    if case == "dense":
        ph = Physics(precision=PHI_FIXED, seed=7, ea_ev=0.15, screening_sites=0.0, cutoff_sites=255, rail_range=4)
        st = _lockstep_case(ph, [24], [256], [0.3], [step_then_relax(1.0, 100e-12)], 200, 50)
    elif case == "two_devices":
        ph = Physics(precision=PHI_FIXED, seed=8, ea_ev=0.15, screening_sites=0.0, cutoff_sites=159, rail_range=4)
        st = _lockstep_case(ph, [10, 6], [160, 96], [0.3, 0.2], [triangle(1.5, 200e-12), constant(-0.7)], 200, 40)
    elif case == "screened_barriers":
        ph = Physics(precision=PHI_FIXED, seed=9, ea_ev=0.15, screening_sites=4.0, cutoff_sites=16, rail_range=1)
        g = np.random.default_rng(12)
        ea = 0.15 + 0.03 * g.standard_normal(20 * 300)
        st = _lockstep_case(ph, [20], [300], [0.3], [constant(0.8)], 150, 50, ea=ea)
    else:
        ph = Physics(precision=PHI_FIXED, seed=10, ea_ev=0.12, screening_sites=3.0, cutoff_sites=30, rail_range=2,
                     coulomb_kappa_v=0.04)
        st = _lockstep_case(ph, [3], [64], [0.4], [triangle(1.0, 100e-12)], 200, 100)
    assert st["hops"] > 100
    print(f"{case}: {st['hops']} hops in lockstep, near-threshold draws {st['oracle_log']}")


def test_hop_list_overflow_recomputes():
    """A barrier of 0 eV makes nearly every candidate hop, more than the hop
    list holds (4096 per half-step), so every half-step falls back to the
    from-scratch potential; the trajectory still follows the oracle."""
    ph = Physics(precision=PHI_FIXED, seed=11, ea_ev=0.0, screening_sites=0.0, cutoff_sites=191, rail_range=4)
    rails, sites = [256], [192]
    # sites that changed in the first step: at most twice the hops of its two
    # half-steps, so more than 4 x 4096 changed sites means a half-step of
    # more than 4096 hops
    p_or = oracle.OracleParams(ph.replace(precision=FP64), rails, sites)
    occ = oracle.fill(p_or, [0.45])
    before = occ.copy()
    oracle.run(p_or, [constant(0.3)], occ, 0, 1)
    assert int((occ != before).sum()) > 4 * 4096
    _lockstep_case(ph, rails, sites, [0.45], [constant(0.3)], 10, 5)


def test_dense_shape_sampled():
    """The dense configuration's shape (64 replicas x 1024 x 512, unscreened
    over the whole rail, +-4 rails) at a lower barrier (thousands of hops
    per step): after 12 steps the potential kept hop by hop equals the one
    computed from scratch, and replica 0 agrees with the oracle on rails
    within its light cone (the oracle updates 300 consecutive rails of that
    replica, the others frozen; a frozen rail's error reaches 4 rails further
    per half-step, so the middle 108 rails are exact after 24 half-steps)."""
    from paper_2511_09413_amd import Simulator
    wl = c4_dense()
    ph = wl.physics.replace(precision=PHI_FIXED, ea_ev=0.15)
    sim = Simulator(ph, wl.rails, wl.sites)
    sim.fill_random(wl.filling)
    occ0 = sim.read_occupancy()
    sim.set_protocols(wl.protocols)
    net, _ = sim.run_steps(12, tallies=True)
    assert int(np.abs(net.cpu().numpy()).sum()) > 1000
    phi, F = sim.fixed_potential()
    fresh, _ = sim.fixed_potential(recompute=True)
    assert np.array_equal(phi.cpu().numpy(), fresh.cpu().numpy())
    R, L = wl.rails[0], wl.sites[0]
    occ = sim.read_occupancy().reshape(len(wl.rails), R, L)
    p1 = oracle.OracleParams(ph.replace(precision=FP64), [R], [L])
    oracle.set_threads(8)
    try:
        for lo in (0, 600):
            part = occ0.reshape(len(wl.rails), R, L)[0].copy().reshape(-1)
            oracle.run(p1, wl.protocols[:1], part, 0, 12, rail_lo=lo, rail_hi=lo + 300, want_dec=False)
            ref = part.reshape(R, L)
            assert np.array_equal(occ[0, lo + 96:lo + 204], ref[lo + 96:lo + 204]), lo
    finally:
        oracle.set_threads(1)
