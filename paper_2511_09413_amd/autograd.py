"""Gradients of simulated observables with respect to the physical parameters.

Two estimators of d E[F] / d theta, theta = (Ea, nu0, kappa, alpha):

* the score-function (likelihood-ratio) estimator, exposed as
  torch.autograd.Function: the forward pass runs the hop steps on the GPU and
  returns the per-step observables of every replica (the fraction of its ions
  in one decile, and its electrode current); the backward pass replays the
  same steps with kmc_score_replay, which sums (d log p / d theta)
  (y - p)/(1 - p) over every hop decision, weighted by the future deviation of
  the observables from a leave-one-out replica baseline;
* central finite differences with common random numbers (crn_fd): the same
  seeds at theta (1 +- h).

Derived observables compose in torch: the mean current over a window is a
mean of the current rows, and the relaxation time (relaxation_time) is the
decay time of a least-squares exponential through the replica-mean decile
curve, whose backward pass applies the fit's implicit-function weights
d tau / d m_n (kmc_fit_decay), so that d tau / d theta = sum_n w_n
d E[f_n] / d theta flows into the replay.

Every hop is a Bernoulli decision with the Arrhenius probability of the rate
law (main text Eq. hop_rate, barrier shifted by half the energy change as in
Eq. 2); the relaxation time is that of the single-exponential decay of the
first-decile fraction after the bias is removed (main text section 4; SI S5).
The gradient machinery is this library's, not the paper's.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

ELEMENTARY_CHARGE = 1.602176634e-19

THETA = ("ea_ev", "nu0_hz", "coulomb_kappa_v", "field_coupling")


@dataclass
class ObservableSpec:
    """What to simulate: physics (its four theta fields are replaced by the
    theta tensor), geometry, filling, one protocol (t_s, v_volt) per device and
    the number of steps.  The observable is the fraction of each device's ions
    in decile `decile` after each step.  `ea` is an optional per-site barrier
    field; theta[0] then shifts it by theta[0] - physics.ea_ev."""
    physics: object
    rails: Sequence[int]
    sites: Sequence[int]
    filling: Sequence[float]
    protocols: Sequence
    n_steps: int
    decile: int = 0
    ea: Optional[np.ndarray] = None
    device: str = "cuda:0"
    mode: str = "auto"
    keep: dict = field(default_factory=dict)


def _simulator(spec: ObservableSpec, theta_values: Sequence[float]):
    from . import Simulator
    ph = spec.physics.replace(**{k: float(v) for k, v in zip(THETA, theta_values)})
    ea = None
    if spec.ea is not None:
        ea = np.asarray(spec.ea, dtype=np.float64) + (float(theta_values[0]) - spec.physics.ea_ev)
    sim = Simulator(ph, spec.rails, spec.sites, ea=ea, device=spec.device, mode=spec.mode)
    sim.fill_random(spec.filling)
    sim.set_protocols(spec.protocols)
    return sim


def _observable(sim, spec: ObservableSpec):
    """Run spec.n_steps; returns (f [n_steps, D] decile fraction, I [n_steps, D]
    electrode current in A, start state, start step)."""
    torch = sim.torch
    occ0 = sim.snapshot()
    step0 = sim.step
    _record(sim, spec.n_steps)
    net, dec = sim.run_steps(spec.n_steps, tallies=True)
    ions = dec[0].sum(dim=1).to(torch.float64).clamp_min(1.0)
    f = dec[:, :, spec.decile].to(torch.float64) / ions
    sites = torch.as_tensor([float(x) for x in spec.sites], dtype=torch.float64, device=f.device)
    cur = net.to(torch.float64) * (ELEMENTARY_CHARGE / spec.physics.dt_s) / sites
    return f, cur, occ0, step0


RECORD_CAP = 1024                # accepted hops per half-step kept by the recording
RECORD_MAX_BYTES = 1 << 30       # larger recordings are not made (the replay then draws again)


def _record(sim, n_steps: int) -> None:
    """Record the forward's hops for the replay where the context supports
    it and the buffer stays moderate; otherwise the replay draws the decisions
    again (same result)."""
    from . import KMC_EUNSUPPORTED, KmcError
    if 32 * n_steps * RECORD_CAP > RECORD_MAX_BYTES:
        return
    try:
        sim.record_hops(n_steps, RECORD_CAP)
    except KmcError as err:
        if err.status != KMC_EUNSUPPORTED:
            raise


def _loo_deviation(x):
    """x minus the leave-one-out replica mean (0 baseline for one replica)."""
    D = x.shape[1]
    if D < 2:
        return x
    return x - (x.sum(dim=1, keepdim=True) - x) / (D - 1)


def _torch_function():
    import torch

    class KmcObservables(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, spec):
            th = theta.detach().to("cpu", torch.float64).tolist()
            sim = _simulator(spec, th)
            f, cur, occ0, step0 = _observable(sim, spec)
            ctx.sim, ctx.occ0, ctx.step0 = sim, occ0, step0
            ctx.f, ctx.cur = f, cur
            ctx.theta_meta = (theta.dtype, theta.device)
            return f.clone(), cur.clone()

        @staticmethod
        def backward(ctx, grad_f, grad_cur):
            contrib = torch.zeros_like(ctx.f)
            if grad_f is not None:
                contrib += grad_f.to(contrib.device, torch.float64) * _loo_deviation(ctx.f)
            if grad_cur is not None:
                contrib += grad_cur.to(contrib.device, torch.float64) * _loo_deviation(ctx.cur)
            W = torch.flip(torch.cumsum(torch.flip(contrib, [0]), 0), [0])  # sum over n' >= n
            grad = ctx.sim.score_replay(ctx.occ0, ctx.step0, W)
            dtype, device = ctx.theta_meta
            ctx.sim.close()
            return grad.sum(dim=0).to(device, dtype), None

    class RelaxationTime(torch.autograd.Function):
        @staticmethod
        def forward(ctx, m, t_s, t0, start):
            from . import fit_decay
            params, w = fit_decay(np.asarray(t_s, dtype=np.float64),
                                  m.detach().to("cpu", torch.float64).numpy(), float(t0), start=start)
            ctx.w = torch.as_tensor(w, dtype=m.dtype, device=m.device)
            return torch.as_tensor(params[2], dtype=m.dtype, device=m.device)

        @staticmethod
        def backward(ctx, grad_tau):
            return grad_tau * ctx.w, None, None, None

    return KmcObservables, RelaxationTime


_FN = None


def _functions():
    global _FN
    if _FN is None:
        _FN = _torch_function()
    return _FN


def observables(theta, spec: ObservableSpec):
    """(f, I): f[n, d] the fraction of replica d's ions in decile spec.decile
    after step n, I[n, d] its electrode current in step n (A; e net / (L dt),
    Ramo-Shockley for blocking electrodes).  Both differentiable in theta
    through the score-function estimator; one replay serves both."""
    return _functions()[0].apply(theta, spec)


def decile_observable(theta, spec: ObservableSpec):
    """f[n, d] (differentiable in theta through the score-function estimator)."""
    return observables(theta, spec)[0]


def current_observable(theta, spec: ObservableSpec):
    """I[n, d] electrode current per step and replica (differentiable in theta)."""
    return observables(theta, spec)[1]


def mean_current(theta, spec: ObservableSpec, window: Optional[slice] = None):
    """Replica- and window-mean electrode current (A), differentiable in theta."""
    cur = current_observable(theta, spec)
    return (cur if window is None else cur[window]).mean()


def relaxation_time(m, t_s, t0: float, start=None):
    """tau of the least-squares C + A exp(-(t - t0)/tau) through the curve m
    (a 1-D tensor, e.g. the replica mean of decile_observable over the
    relaxation window) sampled at t_s; differentiable in m through the fit's
    implicit-function weights."""
    return _functions()[1].apply(m, t_s, t0, start)


def step_times(spec: ObservableSpec, first_step: int = 0):
    """Simulated time (s) after each of the spec's steps: (k + 1) dt."""
    return (np.arange(spec.n_steps, dtype=np.float64) + 1.0 + first_step) * spec.physics.dt_s


def crn_fd(simulate: Callable[[Sequence[float]], np.ndarray], theta: Sequence[float], h: float = 1e-3):
    """Central differences with common random numbers: simulate(theta) must
    return the per-replica value of F with fixed seeds; returns
    (mean [4], per-replica estimates [4, replicas]) of
    (F(theta_i (1 + h)) - F(theta_i (1 - h))) / (2 h theta_i)."""
    theta = np.asarray(theta, dtype=np.float64)
    rows = []
    for i in range(len(theta)):
        up, dn = theta.copy(), theta.copy()
        up[i] *= 1.0 + h
        dn[i] *= 1.0 - h
        rows.append((np.asarray(simulate(up)) - np.asarray(simulate(dn))) / (2.0 * h * theta[i]))
    per = np.array(rows)
    return per.mean(axis=1), per


def gpu_objective(spec: ObservableSpec, weights: np.ndarray,
                  observable: str = "decile") -> Callable[[Sequence[float]], np.ndarray]:
    """simulate(theta) -> per-replica F = sum_n weights[n] x[n, d] on the GPU,
    x the decile fraction (observable="decile") or the electrode current in A
    (observable="current")."""
    w = np.asarray(weights, dtype=np.float64)
    if observable not in ("decile", "current"):
        raise ValueError("observable must be 'decile' or 'current'")

    def simulate(theta):
        sim = _simulator(spec, theta)
        f, cur, _, _ = _observable(sim, spec)
        x = f if observable == "decile" else cur
        out = (x.cpu().numpy() * w[:, None]).sum(axis=0)
        sim.close()
        return out

    return simulate
