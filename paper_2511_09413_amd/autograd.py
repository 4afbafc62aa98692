"""Gradients of simulated observables with respect to the physical parameters.

Two estimators of d E[F] / d theta, theta = (Ea, nu0, kappa, alpha):

* the score-function (likelihood-ratio) estimator, exposed as a
  torch.autograd.Function: the forward pass runs the hop steps on the GPU and
  returns the decile-population observable; the backward pass replays the
  same steps with kmc_score_replay, which sums (d log p / d theta) (y - p)/(1 - p)
  over every hop decision, weighted by the future deviation of the observable
  from a leave-one-out replica baseline;
* central finite differences with common random numbers (crn_fd): the same
  seeds at theta (1 +- h).

Every hop is a Bernoulli decision with the Arrhenius probability of the rate
law (main text Eq. hop_rate, barrier shifted by half the energy change as in
Eq. 2); the gradient machinery is this library's, not the paper's.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np

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
    """Run spec.n_steps; returns (f [n_steps, D] float64, start state, start step)."""
    torch = sim.torch
    occ0 = sim.snapshot()
    step0 = sim.step
    _, dec = sim.run_steps(spec.n_steps, tallies=True)
    ions = dec[0].sum(dim=1).to(torch.float64).clamp_min(1.0)
    f = dec[:, :, spec.decile].to(torch.float64) / ions
    return f, occ0, step0


def _torch_function():
    import torch

    class DecileObservable(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, spec):
            th = theta.detach().to("cpu", torch.float64).tolist()
            sim = _simulator(spec, th)
            f, occ0, step0 = _observable(sim, spec)
            ctx.sim, ctx.occ0, ctx.step0 = sim, occ0, step0
            ctx.f = f
            ctx.theta_meta = (theta.dtype, theta.device)
            return f.clone()

        @staticmethod
        def backward(ctx, grad_f):
            f = ctx.f
            D = f.shape[1]
            if D > 1:
                base = (f.sum(dim=1, keepdim=True) - f) / (D - 1)  # leave-one-out replica mean
            else:
                base = torch.zeros_like(f)
            contrib = grad_f.to(f.device, torch.float64) * (f - base)
            W = torch.flip(torch.cumsum(torch.flip(contrib, [0]), 0), [0])  # sum over n' >= n
            grad = ctx.sim.score_replay(ctx.occ0, ctx.step0, W)
            dtype, device = ctx.theta_meta
            ctx.sim.close()
            return grad.sum(dim=0).to(device, dtype), None

    return DecileObservable


_FN = None


def decile_observable(theta, spec: ObservableSpec):
    """f[n, d] (differentiable in theta through the score-function estimator)."""
    global _FN
    if _FN is None:
        _FN = _torch_function()
    return _FN.apply(theta, spec)


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


def gpu_objective(spec: ObservableSpec, weights: np.ndarray) -> Callable[[Sequence[float]], np.ndarray]:
    """simulate(theta) -> per-replica F = sum_n weights[n] f[n, d] on the GPU."""
    w = np.asarray(weights, dtype=np.float64)

    def simulate(theta):
        sim = _simulator(spec, theta)
        f, _, _ = _observable(sim, spec)
        out = (f.cpu().numpy() * w[:, None]).sum(axis=0)
        sim.close()
        return out

    return simulate
