"""Dense long-range potential on MFMA (KMC_BF16X2) against the binary64 oracle
(needs an MI355X).

Error bound of phi.  Each kernel value is represented as hi + lo with
|K - hi - lo| <= 2^-16 |K|; the occupancy weights (0, 1, 2) are exact.  The
FP32 accumulation of n = 2 (m + 1) Lp products (both halves) rounds at most n
times, each by at most 2^-24 of the running sum, which never exceeds
sum_j occ_j |K| = phi_abs.  So
    |phi_gpu - phi_64| <= (2^-16 + n 2^-24) phi_abs,
with phi_abs = phi_64 for kappa > 0 (all K > 0).  The decisions then use
dE = e_app + phi(t) - K(1,0) - phi(o) in binary32: a decision can differ from
the binary64 oracle's only where |u - p| is below the resulting error of p
(in the worst case (beta/2) |dE error| p, about 1e-3 p at the validation
barrier), so ensembles are compared within their statistical error."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from workloads import BF16X2, FP64, Physics, c4_dense, step_then_relax

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
    print(f"phi error {rails}x{L} m={m}: max rel {(err / ref).max():.3e}, mean rel {(err / ref).mean():.3e}, "
          f"max abs {err.max():.3e} V (bound {_bound(m, L):.3e} rel)")


def test_dense_ensemble_matches_fp64_oracle():
    """64 replicas of 16 x 64, unscreened 1/r over the whole rail and +-4
    rails, validation barrier (0.15 eV), a 1 V pulse then relaxation: the
    BF16X2 path against the binary64 oracle from the same initial states and
    seeds.  The two ensembles' mean currents (pulse and relaxation windows)
    and first-decile relaxation curves agree within 3 sigma of the ensemble
    error (the potential's rounding moves a decision only where u lies within
    about 1e-3 of p relative; most replicas keep the oracle's trajectory)."""
    from paper_2511_09413_amd import Simulator
    D, R, L, n, n_on = 64, 16, 64, 300, 150
    ph = Physics(precision=BF16X2, seed=8, ea_ev=0.15, screening_sites=0.0, cutoff_sites=L - 1, rail_range=4)
    ph64 = ph.replace(precision=FP64)
    proto = step_then_relax(1.0, n_on * ph.dt_s)
    sim = Simulator(ph, [R] * D, [L] * D)
    p_or = oracle.OracleParams(ph64, [R] * D, [L] * D)
    occ0 = oracle.fill(p_or, [0.3] * D)
    sim.load_occupancy(occ0)
    sim.set_protocols([proto] * D)
    net_g, dec_g = sim.run_steps(n, tallies=True)
    net_g, dec_g = net_g.cpu().numpy(), dec_g.cpu().numpy()
    occ_g = sim.read_occupancy()
    occ_o = occ0.copy()
    out = oracle.run(p_or, [proto] * D, occ_o, 0, n)
    ions = out["dec"][0].sum(axis=1).astype(np.float64)
    assert np.array_equal(dec_g[0].sum(axis=1), out["dec"][0].sum(axis=1))

    def check(xg, xo, what):
        gap = abs(xg.mean() - xo.mean())
        sig = np.sqrt(xg.var(ddof=1) / D + xo.var(ddof=1) / D)
        assert gap <= 3.0 * sig + 1e-15, (what, xg.mean(), xo.mean(), sig)

    for w in (slice(0, n_on), slice(n_on, n)):
        check(net_g[w].mean(axis=0), out["net"][w].mean(axis=0).astype(np.float64), f"current {w}")
    f_g = dec_g[:, :, 0] / ions
    f_o = out["dec"][:, :, 0] / ions
    for k in (50, 100, 149, 200, 250, n - 1):
        check(f_g[k], f_o[k], f"first-decile fraction at step {k}")
    same = (occ_g.reshape(D, -1) == occ_o.reshape(D, -1)).all(axis=1)
    print(f"dense ensemble: {int(same.sum())} of {D} replicas end in the oracle's state; "
          f"hops {int(np.abs(out['net']).sum())}")
    assert np.abs(out["net"]).sum() > 1000
    assert same.sum() >= D // 2


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
        # the Coulomb part of dE of a bond, phi(s + 1) - phi(s) up to K(1, 0): its error
        dv = np.abs(np.diff(phi[d, r]) - np.diff(ref))
        print(f"c4 rail ({d}, {r}): phi max rel err {(err / ref).max():.3e} mean {(err / ref).mean():.3e}; "
              f"bond dV err max {dv.max():.3e} V mean {dv.mean():.3e} V")
