"""Gradients of the mean-current and relaxation-time observables on the GPU
(needs an MI355X).

* The autograd bridges (current_observable, relaxation_time over the replica
  mean of decile_observable) against the same estimator computed on the CPU:
  oracle forward, oracle decay fit and implicit-function weights, leave-one-out
  baseline, reverse cumulative weights, oracle replay.  The two sides take the
  same decisions; the replay sums differ by the tolerance derived in
  test_gpu_score.py, and the weights by the fits' agreement (1e-8 relative,
  pinned on the CPU), which adds 1e-7 of the terms' magnitude.
* The binary32 GPU replay against the oracle's binary64 replay (no binary64
  Coulomb option): the trajectories coincide (no decision lies within the
  binary32 error of its threshold; checked), and the binary32 roundings of
  the terms are what the tolerance of test_gpu_score.py bounds with the
  binary32 unit roundoff.
* Common-random-number central finite differences of the GPU simulation
  against the GPU score estimator, within 3 sigma of their combined standard
  error, on a validation variant: 4096 replicas of 2 x 16 sites at a barrier
  of 0.08 eV (about 30 hops per replica in 40 steps, so that a relative step
  of 1e-3 in every parameter flips some decisions; at 0.15 eV a step in the
  Coulomb coupling flips none, and the differences then read exactly 0 with
  a standard error of 0).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import relaxation as rx
from parity_util import gpu_available
from test_gpu_score import _tolerance
from workloads import FP32, FP64, Physics, step_then_relax, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

E_CHARGE = 1.602176634e-19


def _spec(ph, D, R, L, n, proto, decile=0):
    from paper_2511_09413_amd.autograd import ObservableSpec
    return ObservableSpec(ph, [R] * D, [L] * D, [0.3] * D, [proto] * D, n, decile=decile)


def _oracle_estimate(ph, D, R, L, n, proto, grad_f, grad_cur):
    """The score estimator on the CPU for upstream gradients grad_f, grad_cur
    [n, D] of the decile-0 fraction and the current.  Returns (grad [4], the
    oracle replay record, f, cur)."""
    p_or = oracle.OracleParams(ph, [R] * D, [L] * D)
    occ0 = oracle.fill(p_or, [0.3] * D)
    out = oracle.run(p_or, [proto] * D, occ0.copy(), 0, n)
    ions = out["dec"][0].sum(axis=1).astype(np.float64)
    f = out["dec"][:, :, 0] / ions
    cur = out["net"].astype(np.float64) * (E_CHARGE / ph.dt_s) / L

    def loo(x):
        return x - (x.sum(axis=1, keepdims=True) - x) / (D - 1)

    contrib = grad_f * loo(f) + grad_cur * loo(cur)
    W = np.cumsum(contrib[::-1], axis=0)[::-1]
    ref = oracle.score_replay(p_or, [proto] * D, occ0, 0, W)
    return ref["grad"].sum(axis=0), ref, f, cur


def _theta(ph):
    import torch
    from paper_2511_09413_amd.autograd import THETA
    return torch.tensor([getattr(ph, k) for k in THETA], dtype=torch.float64, requires_grad=True)


def test_relaxation_time_gradient_equals_oracle_estimator():
    """tau of the replica-mean first-decile curve after a 1 V pulse: GPU
    autograd (score replay) against the CPU estimator with the oracle's fit."""
    from paper_2511_09413_amd.autograd import decile_observable, relaxation_time, step_times
    ph = Physics(precision=FP64, seed=41, ea_ev=0.06)
    D, R, L, n, n_on = 24, 8, 64, 240, 80
    proto = step_then_relax(1.0, n_on * ph.dt_s)
    spec = _spec(ph, D, R, L, n, proto)
    theta = _theta(ph)
    f = decile_observable(theta, spec)
    t = step_times(spec)
    win = slice(n_on, n)
    t0 = n_on * ph.dt_s
    tau = relaxation_time(f.mean(dim=1)[win], t[win], t0)
    tau.backward()
    g_gpu = theta.grad.numpy()

    f_np = f.detach().cpu().numpy()
    m = f_np.mean(axis=1)[win]
    params, _ = rx.fit_decay(t[win], m, t0)
    assert abs(float(tau.detach()) - params[2]) <= 1e-8 * params[2]
    w = rx.tau_weights(t[win], m, t0, params)
    grad_f = np.zeros((n, D))
    grad_f[win] = w[:, None] / D
    est, ref, f_or, _ = _oracle_estimate(ph, D, R, L, n, proto, grad_f, np.zeros((n, D)))
    assert np.array_equal(f_np, f_or)
    tol = _tolerance(ref, ph).sum(axis=0) + 1e-7 * ref["mag"].sum(axis=0)
    assert np.all(np.abs(g_gpu - est) <= tol), (g_gpu, est, tol)
    assert np.all(ref["mag"].sum(axis=0) > 0)


def test_mean_current_gradient_equals_oracle_estimator():
    """Mean electrode current over a triangle sweep: GPU autograd against the
    CPU estimator."""
    from paper_2511_09413_amd.autograd import mean_current
    ph = Physics(precision=FP32, seed=43, ea_ev=0.1)
    D, R, L, n = 16, 8, 48, 150
    proto = triangle(1.5, n * ph.dt_s)
    spec = _spec(ph, D, R, L, n, proto)
    theta = _theta(ph)
    ic = mean_current(theta, spec, window=slice(30, n))
    ic.backward()
    g_gpu = theta.grad.numpy()
    grad_cur = np.zeros((n, D))
    grad_cur[30:] = 1.0 / ((n - 30) * D)
    est, ref, _, cur = _oracle_estimate(ph, D, R, L, n, proto, np.zeros((n, D)), grad_cur)
    assert abs(float(ic.detach()) - cur[30:].mean()) <= 1e-12 * max(abs(cur[30:]).max(), 1e-30)
    assert np.abs(cur).sum() > 0
    tol = _tolerance(ref, ph).sum(axis=0) + 1e-7 * ref["mag"].sum(axis=0)
    assert np.all(np.abs(g_gpu - est) <= tol), (g_gpu, est, tol)


def test_fp32_replay_against_fp64_oracle_replay():
    """The binary32 GPU replay against the oracle's plain binary64 replay of
    the same decisions (no binary64-Coulomb option)."""
    import torch
    from paper_2511_09413_amd import Simulator
    ph32 = Physics(precision=FP32, seed=45, ea_ev=0.12)
    ph64 = ph32.replace(precision=FP64)
    rails, sites, n = [20, 7], [96, 61], 200
    protos = [triangle(1.0, n * 1e-12), step_then_relax(-0.8, 80e-12)]
    sim = Simulator(ph32, rails, sites)
    sim.fill_random([0.3, 0.4])
    sim.set_protocols(protos)
    occ0 = sim.snapshot()
    net_g, _ = sim.run_steps(n, tallies=True)
    W = np.random.default_rng(8).normal(size=(n, 2))
    grad = sim.score_replay(occ0, 0, torch.from_numpy(W)).cpu().numpy()
    p64 = oracle.OracleParams(ph64, rails, sites)
    occ0_h = occ0.cpu().numpy()
    fwd = oracle.run(p64, protos, occ0_h.copy(), 0, n, want_dec=False)
    assert np.array_equal(net_g.cpu().numpy(), fwd["net"]), "binary32 and binary64 decisions differ"
    assert np.abs(fwd["net"]).sum() > 100
    ref = oracle.score_replay(p64, protos, occ0_h, 0, W)
    eps32 = 2.0 ** -23
    n_terms = (2 * ph32.rail_range + 1) * (2 * ph32.cutoff_sites + 2)
    # the bound of test_gpu_score.py (binary32 exponential as 2^(arg log2 e))
    tol = (4 * eps32 * ref["sens"] + 3 * eps32 * ref["sens_arg"] + (eps32 + (n_terms + 8) * 2.0 ** -52) * ref["sens_b"]
           + 1e-9 * ref["mag"])
    assert np.all(np.abs(grad - ref["grad"]) <= tol), (grad, ref["grad"], tol)
    # the binary32 terms do differ from binary64 ones (the comparison is not vacuous)
    assert np.any(np.abs(grad - ref["grad"]) > 0)


@pytest.mark.parametrize("observable", ["decile", "current"])
def test_crn_finite_differences_agree_with_score_estimator(observable):
    """F = sum_n w_n x_n per replica (x the decile-0 fraction or the current)
    under a pulse then relaxation; CRN central differences (h = 1e-3, same
    seeds) of the GPU simulation against the GPU score estimator, per theta
    within 3 sigma of the combined standard error, at least three of the four
    resolved beyond 3 sigma of zero by the score estimator."""
    import torch
    from paper_2511_09413_amd.autograd import (THETA, crn_fd, decile_observable, current_observable,
                                               gpu_objective)
    ph = Physics(precision=FP32, seed=47, ea_ev=0.08)
    D, R, L, n = 4096, 2, 16, 40
    proto = step_then_relax(1.0, 20 * ph.dt_s)
    spec = _spec(ph, D, R, L, n, proto)
    w = np.linspace(0.2, 1.0, n)
    theta = _theta(ph)
    fn = decile_observable if observable == "decile" else current_observable
    x = fn(theta, spec)
    wt = torch.from_numpy(w).to(x.device)
    (x * wt[:, None]).sum().backward()
    est_mean = theta.grad.numpy() / D
    # per-replica estimates for the standard error: replay with the same weights
    from paper_2511_09413_amd.autograd import _observable, _simulator, _loo_deviation
    sim = _simulator(spec, [getattr(ph, k) for k in THETA])
    f, cur, occ0, step0 = _observable(sim, spec)
    xx = f if observable == "decile" else cur
    contrib = wt[:, None] * _loo_deviation(xx)
    Wm = torch.flip(torch.cumsum(torch.flip(contrib, [0]), 0), [0])
    per = sim.score_replay(occ0, step0, Wm).cpu().numpy()      # [D, 4]
    sim.close()
    assert np.allclose(per.mean(axis=0), est_mean, rtol=1e-12, atol=0)
    se_s = per.std(axis=0, ddof=1) / math.sqrt(D)
    th = np.array([getattr(ph, k) for k in THETA])
    fd_mean, fd_per = crn_fd(gpu_objective(spec, w, observable), th, h=1e-3)
    se_fd = fd_per.std(axis=1, ddof=1) / math.sqrt(D)
    assert np.all(se_fd > 0), "a parameter step flipped no decision: the differences carry no information"
    gap = np.abs(est_mean - fd_mean)
    bound = 3.0 * np.sqrt(se_s ** 2 + se_fd ** 2)
    assert np.all(gap <= bound), (est_mean, fd_mean, se_s, se_fd)
    assert np.sum(np.abs(est_mean) > 3.0 * se_s) >= 3, (est_mean, se_s)
