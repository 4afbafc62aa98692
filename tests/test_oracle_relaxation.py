"""Pins of the oracle's relaxation-time fit (CPU only).

The fit (oracle/relaxation.py) takes the single-exponential decay of the
first-decile fraction that the paper reports after the bias is removed (main
text section 4, relaxation decay; SI S5) and returns tau by Gauss-Newton least
squares, plus the implicit-function weights w_n = d tau / d m_n.  Pinned here
against:
  * exact recovery of (C, A, tau) from noise-free exponentials, rising and
    falling, with the window starting before, at or after t0;
  * the derivative formulas (Jacobian, Hessian) against central differences
    of the model itself;
  * w_n against central differences of the whole fit (refits of perturbed
    data), on noisy data where the residual term of the implicit derivative
    matters (dropping it fails this test);
  * exact invariances: a constant added to the data, or the data scaled,
    leave tau unchanged, so sum_n w_n = 0 and sum_n w_n m_n = 0;
  * the least-squares optimum itself: no small step in any direction lowers
    the residual sum.
"""
import numpy as np
import pytest

from oracle import relaxation as rx


@pytest.mark.parametrize("C,A,tau,t0,window", [
    (0.21, 0.35, 3.0e-9, 10e-9, (10e-9, 40e-9)),
    (0.10, -0.05, 1.0e-9, 0.0, (0.0, 8e-9)),       # rising towards the asymptote
    (0.33, 0.02, 7.5e-9, 5e-9, (6e-9, 60e-9)),     # window starts after t0
    (1.5, 2.0, 40.0, 0.0, (-5.0, 200.0)),          # seconds, window before t0
])
def test_exact_recovery(C, A, tau, t0, window):
    t = np.linspace(window[0], window[1], 400)
    m = rx.decay_model(t, t0, C, A, tau)
    (c, a, ta), it = rx.fit_decay(t, m, t0)
    assert abs(ta - tau) <= 1e-9 * tau, (ta, tau, it)
    assert abs(c - C) <= 1e-9 * (abs(C) + abs(A))
    assert abs(a - A) <= 1e-9 * abs(A)


def test_derivatives_against_model_differences():
    t = np.linspace(0.0, 5.0, 50)
    t0, beta = 0.3, np.array([0.2, 0.7, 1.3])
    J = rx.decay_jacobian(t, t0, *beta)
    H = rx.decay_hessian(t, t0, *beta)
    for k in range(3):
        h = 1e-6 * max(abs(beta[k]), 1.0)
        up, dn = beta.copy(), beta.copy()
        up[k] += h
        dn[k] -= h
        fd = (rx.decay_model(t, t0, *up) - rx.decay_model(t, t0, *dn)) / (2 * h)
        assert np.allclose(J[:, k], fd, rtol=1e-7, atol=1e-9)
        fdJ = (rx.decay_jacobian(t, t0, *up) - rx.decay_jacobian(t, t0, *dn)) / (2 * h)
        assert np.allclose(H[:, :, k], fdJ, rtol=1e-6, atol=1e-8)


def _noisy(seed, n=300, C=0.25, A=0.4, tau=4e-9, t0=2e-9, sigma=0.03):
    g = np.random.default_rng(seed)
    t = np.linspace(t0, t0 + 25e-9, n)
    return t, t0, rx.decay_model(t, t0, C, A, tau) + g.normal(0.0, sigma, n)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_weights_against_refit_differences(seed):
    t, t0, m = _noisy(seed)
    params, _ = rx.fit_decay(t, m, t0)
    w = rx.tau_weights(t, m, t0, params)
    idx = np.random.default_rng(seed).choice(len(t), 12, replace=False)
    eps = 1e-5
    for i in idx:
        up, dn = m.copy(), m.copy()
        up[i] += eps
        dn[i] -= eps
        tp = rx.fit_decay(t, up, t0, start=params)[0][2]
        tm = rx.fit_decay(t, dn, t0, start=params)[0][2]
        fd = (tp - tm) / (2 * eps)
        assert abs(fd - w[i]) <= 1e-7 * np.abs(w).max(), (i, fd, w[i])


def test_residual_term_is_needed():
    """On noisy data the Gauss-Newton-only weights ((J^T J)^-1 J^T) differ from
    the refit differences by far more than the tolerance above."""
    t, t0, m = _noisy(7, sigma=0.08)
    params, _ = rx.fit_decay(t, m, t0)
    w = rx.tau_weights(t, m, t0, params)
    J = rx.decay_jacobian(t, t0, *params)
    w_gn = np.linalg.solve(J.T @ J, J.T)[2]
    assert np.abs(w - w_gn).max() > 1e-3 * np.abs(w).max()


@pytest.mark.parametrize("seed", [4, 5])
def test_weight_invariances(seed):
    t, t0, m = _noisy(seed)
    params, _ = rx.fit_decay(t, m, t0)
    w = rx.tau_weights(t, m, t0, params)
    scale = np.abs(w).sum()
    assert abs(w.sum()) <= 1e-9 * scale                 # m + c: C absorbs the shift
    assert abs((w * m).sum()) <= 1e-9 * scale * np.abs(m).max()   # s m: C, A scale
    # and the fit itself: tau unchanged under shift and scale of the data
    tau = params[2]
    assert abs(rx.fit_decay(t, m + 0.7, t0)[0][2] - tau) <= 1e-9 * tau
    assert abs(rx.fit_decay(t, 3.0 * m, t0)[0][2] - tau) <= 1e-9 * tau


def test_fit_is_a_least_squares_minimum():
    t, t0, m = _noisy(9)
    params, _ = rx.fit_decay(t, m, t0)
    beta = np.array(params)
    s0 = np.sum((m - rx.decay_model(t, t0, *beta)) ** 2)
    g = np.random.default_rng(0)
    for _ in range(50):
        d = g.normal(size=3) * np.abs(beta) * 1e-4
        assert np.sum((m - rx.decay_model(t, t0, *(beta + d))) ** 2) >= s0 * (1 - 1e-12)
