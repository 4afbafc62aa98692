"""Score-function replay on the GPU (kmc_score_replay) against the oracle's
replay on the same seeds, and the autograd bridge (needs an MI355X).

Tolerance.  Both sides take the same decisions (the replay decides as the
forward does) and sum the terms W g (y - p)/(1 - p) in binary64, in different
orders.  The score terms take the Coulomb part of dE in binary64 rounded once
to the path precision: the GPU as +-(phi(s + 1) - phi(s)) - K(1, 0), summed
in one pass over the bond's window whenever a hop changed it, the oracle
(coul64) as the window sum.  The two binary64 values differ by at most
(n + 8) eps64 B, with n the window's terms and B = A + |dE| + |dE_coul| +
2 K(1, 0), A the window's sum of |K(t - j)| + |K(o - j)| over occupied
sites.  After the rounding to the path
precision (eps) the Coulomb parts are equal or one unit apart, so dE differs
by at most eps B, the exponent's argument by (beta/2) eps B plus the two
roundings of its evaluation (2 eps |arg|), and the exponential by a few units
(device vs glibc).  In binary32 the replay kernels take a term's exponential
as 2^(arg log2 e) on the hardware's base-2 exponential: the product's
rounding adds |arg| eps/2 to p's relative error, so the argument's part is
bounded by 3 eps |arg|.  A relative change dp/p = x moves a term by
|W g| p/(1 - p)^2 x (and the kappa term also through dE_coul itself), so
    |grad_gpu - grad_oracle| <= 4 eps sens + 3 eps sens_arg
                                + (eps + (n + 8) eps64) sens_b + 1e-9 mag
with sens = sum |W g| p/(1-p)^2, sens_arg the same weighted by |arg|,
sens_b the dE-scale sum of the oracle (orc_run_opts) and mag = sum |term|;
the last part covers the binary64 summation order."""
import math

import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from workloads import FP32, FP64, Physics, c5_gradient, constant, small_case, step_then_relax, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

EPS = {FP64: 2.0 ** -52, FP32: 2.0 ** -23}


def _tolerance(ref, ph):
    eps = EPS[ph.precision]
    n_terms = (2 * ph.rail_range + 1) * (2 * ph.cutoff_sites + 2)
    c_b = eps + (n_terms + 8) * EPS[FP64]
    return 4 * eps * ref["sens"] + 3 * eps * ref["sens_arg"] + c_b * ref["sens_b"] + 1e-9 * ref["mag"]


def _forward_and_replay(ph, rails, sites, filling, protocols, n_steps, weights_seed, ea=None, mode="auto",
                        tile_sites=0):
    import torch
    from paper_2511_09413_amd import Simulator
    sim = Simulator(ph, rails, sites, ea=ea, mode=mode, tile_sites=tile_sites)
    sim.fill_random(filling)
    sim.set_protocols(protocols)
    occ0 = sim.snapshot()
    occ0_h = occ0.cpu().numpy()
    net_g, _ = sim.run_steps(n_steps, tallies=True)
    D = len(rails)
    W = np.random.default_rng(weights_seed).normal(size=(n_steps, D))
    grad = sim.score_replay(occ0, 0, torch.from_numpy(W)).cpu().numpy()
    p_or = oracle.OracleParams(ph, rails, sites, ea)
    fwd = oracle.run(p_or, protocols, occ0_h.copy(), 0, n_steps, want_dec=False)
    ref = oracle.score_replay(p_or, protocols, occ0_h, 0, W, coul64=True)
    return sim, grad, ref, net_g.cpu().numpy(), fwd


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("mode,tile", [("half_step", 0), ("persistent", 0), ("half_step", 512), ("wave", 0)])
def test_replay_matches_oracle_ragged(precision, mode, tile):
    """Two devices of different shapes, validation barrier (many hops), a bias
    sweep: the GPU replay's four sums per device equal the oracle's."""
    ph = Physics(precision=precision, seed=77, ea_ev=0.15)
    rails, sites = [24, 5], [128, 77]
    protos = [triangle(1.0, 300e-12), constant(-0.4)]
    sim, grad, ref, net_g, fwd = _forward_and_replay(ph, rails, sites, [0.3, 0.45], protos, 300, 5, mode=mode,
                                                     tile_sites=tile)
    assert np.array_equal(net_g, fwd["net"])      # forward trajectory identical to the oracle's
    assert np.abs(fwd["net"]).sum() > 100
    tol = _tolerance(ref, ph)
    assert np.all(np.abs(grad - ref["grad"]) <= tol), (grad, ref["grad"], tol)
    assert np.all(ref["mag"] > 0)


def test_replay_with_barrier_field_and_wide_interaction():
    """Per-site barriers (origin-site barrier), +-2 rails, unscreened, cutoff 40."""
    R, L = 16, 96
    ph = Physics(precision=FP64, seed=5, ea_ev=0.15, screening_sites=0.0, cutoff_sites=40, rail_range=2)
    ea = np.random.default_rng(3).normal(0.15, 0.02, size=R * L)
    sim, grad, ref, net_g, fwd = _forward_and_replay(ph, [R], [L], [0.3], [constant(0.6)], 120, 9, ea=ea)
    assert np.array_equal(net_g, fwd["net"])
    assert np.all(np.abs(grad - ref["grad"]) <= _tolerance(ref, ph))


def test_replay_many_hops_per_half_step():
    """A barrier low enough that about half the candidates hop: each half-step
    accepts more hops than the list holds (4096 for this lattice), so the
    potential is recomputed from the new state after every half-step."""
    ph = Physics(precision=FP64, seed=21, ea_ev=0.02)
    R, L = 64, 1024
    sim, grad, ref, net_g, fwd = _forward_and_replay(ph, [R], [L], [0.3], [triangle(0.5, 40e-12)], 8, 4)
    assert np.array_equal(net_g, fwd["net"])
    assert ref["hops"][0] > 8 * 2 * 4096
    assert np.all(np.abs(grad - ref["grad"]) <= _tolerance(ref, ph)), (grad, ref["grad"], _tolerance(ref, ph))


@pytest.mark.parametrize("rails,sites,m,cut,precision", [
    ([1, 2, 3], [40, 33, 57], 2, 16, FP64),   # rings shorter than the rail range: duplicate offsets
    ([4, 2], [19, 64], 1, 0, FP32),           # cutoff 0: no Coulomb term, K(1, 0) = 0
    ([6], [24], 2, 30, FP32),                 # window longer than the rail
    ([3], [400], 1, 200, FP64),               # recomputation from global memory (cutoff above 128)
    ([2], [1400], 0, 600, FP32),              # start-up without LDS tiles (cutoff above 512)
])
def test_replay_edge_geometries(rails, sites, m, cut, precision):
    """Replay of small rings, cutoff 0 and windows longer than the rail, with a
    barrier low enough that the potential differences see many updates."""
    ph = Physics(precision=precision, seed=31, ea_ev=0.08, rail_range=m, cutoff_sites=cut)
    protos = [triangle(1.0, 80e-12), constant(0.5), step_then_relax(-1.0, 30e-12)][:len(rails)]
    sim, grad, ref, net_g, fwd = _forward_and_replay(ph, rails, sites, [0.4] * len(rails), protos, 80, 6)
    assert np.array_equal(net_g, fwd["net"])
    assert np.all(ref["hops"] > 20)
    tol = _tolerance(ref, ph)
    assert np.all(np.abs(grad - ref["grad"]) <= tol), (grad, ref["grad"], tol)


@pytest.mark.parametrize("seed", range(4))
def test_replay_random_geometries(seed):
    """Seeded random lattices: rail counts 1..12, sites 2..300, rail ranges
    0..3, cutoffs 0..40, screened and unscreened, both precisions, barriers
    0.08..0.15 eV; 60 steps replayed against the oracle's replay."""
    g = np.random.default_rng(3000 + seed)
    n_dev = int(g.integers(1, 4))
    m = int(g.integers(0, 4))
    rails = [int(g.integers(1, 13)) for _ in range(n_dev)]
    sites = [int(g.integers(2, 301)) for _ in range(n_dev)]
    cut = int(g.integers(0, 41))
    lam = float(g.choice([0.0, 2.0, 4.0]))
    precision = FP64 if seed % 2 == 0 else FP32
    ph = Physics(precision=precision, seed=seed + 70, ea_ev=float(g.uniform(0.08, 0.15)), rail_range=m,
                 cutoff_sites=cut, screening_sites=lam)
    protos = [triangle(1.0, 80e-12), constant(0.5), step_then_relax(-1.0, 30e-12)][:n_dev]
    fill = [float(g.uniform(0.1, 0.5)) for _ in range(n_dev)]
    sim, grad, ref, net_g, fwd = _forward_and_replay(ph, rails, sites, fill, protos, 60, 11 + seed)
    assert np.array_equal(net_g, fwd["net"])
    tol = _tolerance(ref, ph)
    assert np.all(np.abs(grad - ref["grad"]) <= tol), (grad, ref["grad"], tol)


def test_replay_leaves_the_context_alone():
    """Replaying does not change the state, the step counter or the tallies:
    continuing afterwards gives the same trajectory as a context that never
    replayed."""
    import torch
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=FP32, seed=3, ea_ev=0.15)
    a = Simulator(ph, [12], [64])
    b = Simulator(ph, [12], [64])
    for s in (a, b):
        s.fill_random([0.3])
        s.set_protocols([constant(0.5)])
    occ0 = a.snapshot()
    a.run_steps(40)
    b.run_steps(40)
    a.score_replay(occ0, 0, torch.ones((40, 1), dtype=torch.float64))
    assert a.step == b.step == 40
    na, _ = a.run_steps(60, tallies=True)
    nb, _ = b.run_steps(60, tallies=True)
    assert torch.equal(na, nb)
    assert np.array_equal(a.read_occupancy(), b.read_occupancy())
    assert np.array_equal(a.read_current()[1], b.read_current()[1])


def test_replay_rejects_kappa_zero():
    import torch
    from paper_2511_09413_amd import KmcError, Simulator
    sim = Simulator(Physics(precision=FP32, coulomb_kappa_v=0.0), [4], [32])
    with pytest.raises(KmcError):
        sim.score_replay(sim.snapshot(), 0, torch.ones((2, 1), dtype=torch.float64))


def test_autograd_backward_equals_oracle_estimator():
    """decile_observable's backward = the same estimator computed on the CPU:
    oracle forward for f, leave-one-out baseline, reverse cumulative weights,
    oracle replay, summed over replicas."""
    import torch
    from paper_2511_09413_amd.autograd import THETA, ObservableSpec, decile_observable
    ph = Physics(precision=FP64, seed=12, ea_ev=0.15)
    D, R, L, n = 6, 8, 40, 80
    protos = [step_then_relax(1.0, 40e-12)] * D
    spec = ObservableSpec(ph, [R] * D, [L] * D, [0.3] * D, protos, n, decile=0)
    theta = torch.tensor([getattr(ph, k) for k in THETA], dtype=torch.float64, requires_grad=True)
    w = torch.linspace(0.5, 1.5, n, dtype=torch.float64)
    f = decile_observable(theta, spec)
    (f * w.to(f.device)[:, None]).sum().backward()
    g_gpu = theta.grad.numpy()

    p_or = oracle.OracleParams(ph, [R] * D, [L] * D)
    occ0 = oracle.fill(p_or, [0.3] * D)
    out = oracle.run(p_or, protos, occ0.copy(), 0, n)
    ions = out["dec"][0].sum(axis=1).astype(np.float64)
    fo = out["dec"][:, :, 0] / ions
    assert np.allclose(f.detach().cpu().numpy(), fo, rtol=0, atol=0)
    base = (fo.sum(axis=1, keepdims=True) - fo) / (D - 1)
    W = np.cumsum((w.numpy()[:, None] * (fo - base))[::-1], axis=0)[::-1]
    ref = oracle.score_replay(p_or, protos, occ0, 0, W, coul64=True)
    tol = _tolerance(ref, ph).sum(axis=0)
    assert np.all(np.abs(g_gpu - ref["grad"].sum(axis=0)) <= tol), (g_gpu, ref["grad"].sum(axis=0), tol)


def test_c5_full_size_sampled():
    """512 replicas x 256 x 512 (FP32), the gradient workload's shape: replay
    256 steps on the GPU; for two sampled replicas (the first and the last)
    the oracle computes the same replica alone (the replicas before it shrunk
    to 1 x 2 sites with zero weight, so the replica index of the random stream
    is unchanged)."""
    import torch
    from paper_2511_09413_amd import Simulator
    n = 256
    wl = c5_gradient(n_steps=n)
    ph = wl.physics.replace(ea_ev=0.2)
    D = len(wl.rails)
    sim = Simulator(ph, wl.rails, wl.sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    occ0 = sim.snapshot()
    sim.run_steps(n)
    W = np.random.default_rng(1).normal(size=(n, D))
    grad = sim.score_replay(occ0, 0, torch.from_numpy(W)).cpu().numpy()
    occ0_h = occ0.cpu().numpy().reshape(D, -1)
    for d in (0, D - 1):
        rails = [1] * d + [wl.rails[d]]
        sites = [2] * d + [wl.sites[d]]
        p_or = oracle.OracleParams(ph, rails, sites)
        occ = np.concatenate([np.zeros(2 * d, dtype=np.int8), occ0_h[d]])
        Wd = np.zeros((n, d + 1))
        Wd[:, d] = W[:, d]
        ref = oracle.score_replay(p_or, [wl.protocols[d]] * (d + 1), occ, 0, Wd, coul64=True)
        assert ref["hops"][d] > 100
        tol = _tolerance(ref, ph)[d]
        assert np.all(np.abs(grad[d] - ref["grad"][d]) <= tol), (d, grad[d], ref["grad"][d], tol)
