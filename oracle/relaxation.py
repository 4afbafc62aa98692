"""Relaxation time of the decay observable, and its sensitivity to the data.

TEST INFRASTRUCTURE ONLY: imported by tests/ (the product library has its own
fit behind the C ABI and never imports this module).

What is computed.  After the polarising bias is removed, the fraction of ions
in the first decile decays exponentially towards an asymptote that every run
shares, a single diffusion-controlled relaxation (main text section 4,
"relaxation decay"; SI S5 "Current relaxation and influence of relaxation
time").  The relaxation time tau of an ensemble-mean curve m_n sampled at
times t_n of the relaxation window is therefore the tau of the least-squares
single exponential

    g(t) = C + A exp(-(t - t0) / tau),
    (C, A, tau) = argmin  S = sum_n (m_n - g(t_n))^2 ,

found by Gauss-Newton iteration in binary64: with residuals r_n = m_n - g(t_n)
and the Jacobian J_nk = dg(t_n)/d beta_k of beta = (C, A, tau), each step
solves the normal equations (J^T J) delta = J^T r and takes beta + delta,
halving delta while S does not decrease.  Times are measured in units of the
window length from t0 inside the fit (the same minimum, a better-conditioned
J^T J).

The data weights w_n = d tau / d m_n follow from the implicit-function theorem
on the stationarity condition G(beta, m) = J(beta)^T r(beta, m) = 0:
dG/dm_n = J_n and dG/dbeta = -(J^T J - sum_n r_n H_n) with H_n the Hessian of
g(t_n) in beta, so

    d beta / d m_n = (J^T J - sum_n r_n H_n)^(-1) J_n ,

and w_n is its tau component.  A gradient of tau with respect to a model
parameter theta is then sum_n w_n d m_n / d theta (the score-function
estimator of d E[sum_n w_n f_n] / d theta, with the weights held fixed).
"""
from __future__ import annotations

import numpy as np


def decay_model(t, t0, C, A, tau):
    """g(t) = C + A exp(-(t - t0)/tau)."""
    t = np.asarray(t, dtype=np.float64)
    return C + A * np.exp(-(t - t0) / tau)


def decay_jacobian(t, t0, C, A, tau):
    """[n][3]: dg/dC = 1, dg/dA = e, dg/dtau = A (t - t0) e / tau^2, with
    e = exp(-(t - t0)/tau)."""
    t = np.asarray(t, dtype=np.float64)
    x = t - t0
    e = np.exp(-x / tau)
    return np.stack([np.ones_like(x), e, A * x * e / tau ** 2], axis=1)


def decay_hessian(t, t0, C, A, tau):
    """[n][3][3]: second derivatives of g(t_n) in (C, A, tau).  g is linear in
    C and A, so only d2g/dA dtau = x e / tau^2 and
    d2g/dtau^2 = A e (x^2 / tau^4 - 2 x / tau^3) are nonzero (x = t - t0)."""
    t = np.asarray(t, dtype=np.float64)
    x = t - t0
    e = np.exp(-x / tau)
    H = np.zeros((len(x), 3, 3))
    H[:, 1, 2] = H[:, 2, 1] = x * e / tau ** 2
    H[:, 2, 2] = A * e * (x ** 2 / tau ** 4 - 2.0 * x / tau ** 3)
    return H


def initial_guess(t, m, t0):
    """A starting point: C from the last tenth of the window, A = m(first) - C,
    tau from the first time |m - C| falls below |A|/e (else a third of the
    window)."""
    t = np.asarray(t, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    tail = max(1, len(m) // 10)
    C = float(np.mean(m[-tail:]))
    A = float(m[0] - C)
    below = np.nonzero(np.abs(m - C) < abs(A) / np.e)[0]
    tau = float(t[below[0]] - t0) if len(below) and t[below[0]] > t0 else float(t[-1] - t0) / 3.0
    if not tau > 0:
        tau = float(t[-1] - t[0]) / 3.0
    return C, A, tau


def _scaled(t, t0):
    """Times as x = (t - t0)/T with T the window's largest |t - t0|: the fit
    runs in (C, A, tau/T), which is the same least-squares problem with a
    well-conditioned Jacobian (in seconds, dg/dtau is ~1e17 times dg/dC)."""
    t = np.asarray(t, dtype=np.float64)
    T = float(np.max(np.abs(t - t0)))
    if not T > 0:
        raise ValueError("the window needs a time other than t0")
    return (t - t0) / T, T


def fit_decay(t, m, t0, start=None, max_iter=200):
    """Gauss-Newton least-squares fit of C + A exp(-(t - t0)/tau) to (t, m).
    Far from the minimum a step is halved until the residual sum decreases;
    once the relative step is below 1e-6 the full Gauss-Newton steps are
    taken until they stop shrinking (the residual sum is then flat to
    rounding, so it can no longer guide the step).  Returns (C, A, tau) and
    the number of iterations."""
    m = np.asarray(m, dtype=np.float64)
    x, T = _scaled(t, t0)
    C, A, tau = start if start is not None else initial_guess(t, m, t0)
    beta = np.array([C, A, tau / T], dtype=np.float64)

    def ssr(b):
        return float(np.sum((m - decay_model(x, 0.0, *b)) ** 2))

    s = ssr(beta)
    prev = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        J = decay_jacobian(x, 0.0, *beta)
        r = m - decay_model(x, 0.0, *beta)
        delta = np.linalg.solve(J.T @ J, J.T @ r)
        rel = float(np.max(np.abs(delta) / np.maximum(np.abs(beta), 1e-300)))
        if rel < 1e-6:
            if rel >= prev:
                break                 # the steps stopped shrinking: converged to rounding
            beta = beta + delta
            prev = rel
            if rel < 1e-15:
                break
            continue
        lam = 1.0
        while True:
            trial = beta + lam * delta
            if trial[2] > 0:
                s_trial = ssr(trial)
                if s_trial <= s:
                    break
            lam *= 0.5
            if lam < 1e-12:
                raise RuntimeError("decay fit: no descent step")
        beta, s = trial, s_trial
    return (beta[0], beta[1], beta[2] * T), it


def tau_weights(t, m, t0, params):
    """w_n = d tau / d m_n at the fitted params (C, A, tau), from the
    implicit-function theorem on J^T r = 0 (solved in the scaled time of
    fit_decay, then tau = T tau_scaled)."""
    m = np.asarray(m, dtype=np.float64)
    x, T = _scaled(t, t0)
    b = (params[0], params[1], params[2] / T)
    J = decay_jacobian(x, 0.0, *b)
    H = decay_hessian(x, 0.0, *b)
    r = m - decay_model(x, 0.0, *b)
    M = J.T @ J - np.einsum("n,nij->ij", r, H)
    dbeta = np.linalg.solve(M, J.T)          # [3][n]: d beta / d m_n
    return T * dbeta[2]
