"""The oracle's score-function replay against exact derivatives of the chain
(CPU only).

For an observable F = sum_n w_n f(x_n) of a tiny device, E[F] is computed
exactly from the enumerated chain (oracle/exact_chain.py) and differentiated by
central differences in each parameter theta = (Ea, nu0, kappa, alpha).  The
likelihood-ratio estimator

    grad = mean over replicas of  sum_c s_c W(n_c),
    W(n) = sum_{n' >= n} w_n' (f(x_n') - E[f(x_n')]),
    s_c  = (d log p_c / d theta) (y_c - p_c) / (1 - p_c),

is unbiased for dE[F]/dtheta (the score of each decision has zero mean given
the past), so its replica mean must agree with the exact derivative within its
standard error."""
import math

import numpy as np
import pytest

import oracle
from oracle.exact_chain import Lattice
from workloads import FP32, FP64, Physics, constant, triangle

THETA = ("ea_ev", "nu0_hz", "coulomb_kappa_v", "field_coupling")


def _physics(**kw):
    base = dict(precision=FP64, ea_ev=0.06, coulomb_kappa_v=0.04, screening_sites=4.0,
                cutoff_sites=16, rail_range=1, seed=21)
    base.update(kw)
    return Physics(**base)


def _exact_mean_f(ph, R, L, ions, occ0, volts):
    lat = Lattice(R, L, ions, ph)
    P0 = np.zeros(len(lat.states))
    P0[lat.state_of(occ0)] = 1.0
    f = np.array([float(x[:, 0].sum()) for x in lat.states])  # ions on site 0
    ev = lat.evolve(P0, volts)
    return ev["P"] @ f


def _exact_gradient(ph, R, L, ions, occ0, volts, w, rel=1e-4):
    out = []
    for name in THETA:
        th = getattr(ph, name)
        h = rel * th
        fp = _exact_mean_f(ph.replace(**{name: th + h}), R, L, ions, occ0, volts) @ w
        fm = _exact_mean_f(ph.replace(**{name: th - h}), R, L, ions, occ0, volts) @ w
        out.append((fp - fm) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("R,L,ions,protocol,precision,ea", [
    (2, 4, [2, 1], constant(0.35), FP64, 0.03),
    (1, 6, [3], triangle(0.9, 8e-12), FP64, 0.06),
    (2, 4, [1, 2], constant(-0.5), FP32, 0.03),
])
def test_score_estimator_matches_exact_derivative(R, L, ions, protocol, precision, ea):
    ph = _physics(precision=precision, ea_ev=ea)
    lat = Lattice(R, L, ions, ph)
    occ0 = lat.states[len(lat.states) // 3]
    n_steps, D = 5, 20000
    volts = [oracle.protocol_voltage(protocol[0], protocol[1], n * ph.dt_s) for n in range(n_steps)]
    w = np.array([0.2, 0.5, 1.0, -0.3, 0.8])
    mean_f = _exact_mean_f(ph, R, L, ions, occ0, volts)
    exact = _exact_gradient(ph, R, L, ions, occ0, volts, w)

    p = oracle.OracleParams(ph, [R] * D, [L] * D)
    occ = np.tile(occ0.reshape(-1), D)
    fwd = oracle.run(p, [protocol] * D, occ.copy(), 0, n_steps)
    f = fwd["dec"][:, :, 0].astype(np.float64)               # [n][d]: ions on site 0 (L < 10)
    assert L < 10
    contrib = w[:, None] * (f - mean_f[:, None])
    W = np.cumsum(contrib[::-1], axis=0)[::-1]               # sum over n' >= n
    rep = oracle.score_replay(p, [protocol] * D, occ, 0, W)
    assert np.array_equal(rep["occ"], fwd["occ"])            # the replay follows the same trajectory
    est = rep["grad"].mean(axis=0)
    se = rep["grad"].std(axis=0) / math.sqrt(D)
    for q in range(4):
        assert abs(est[q] - exact[q]) < 4.5 * se[q], (THETA[q], est[q], exact[q], se[q])
    # the comparison has power: the derivatives are resolved well beyond noise
    assert (np.abs(exact) > 3 * se).sum() >= 3, (exact, se)


def test_score_is_zero_when_probability_saturates():
    """p clamped at 1 has no parameter dependence: every term vanishes."""
    ph = _physics(ea_ev=-0.5)
    p = oracle.OracleParams(ph, [2], [6])
    occ = np.array([1, 0, 1, 0, 0, 1, 0, 1, 1, 0, 0, 0], dtype=np.int8)
    rep = oracle.score_replay(p, [constant(0.2)], occ, 0, np.ones((4, 1)))
    assert np.all(rep["grad"] == 0.0) and np.all(rep["mag"] == 0.0)


def test_score_needs_kappa():
    ph = _physics(coulomb_kappa_v=0.0)
    p = oracle.OracleParams(ph, [1], [4])
    with pytest.raises(ValueError):
        oracle.score_replay(p, [constant(0.0)], np.array([1, 0, 0, 1], dtype=np.int8), 0, np.ones((2, 1)))


def test_crn_fd_harness_matches_exact_derivative():
    """The common-random-numbers finite-difference harness of the package,
    driven by the oracle as simulator, agrees with the exact derivative."""
    from paper_2511_09413_amd.autograd import crn_fd
    R, L, ions = 1, 6, [3]
    protocol = triangle(0.9, 8e-12)
    ph = _physics(ea_ev=0.06)
    lat = Lattice(R, L, ions, ph)
    occ0 = lat.states[len(lat.states) // 3]
    n_steps, D = 5, 20000
    volts = [oracle.protocol_voltage(protocol[0], protocol[1], n * ph.dt_s) for n in range(n_steps)]
    w = np.array([0.2, 0.5, 1.0, -0.3, 0.8])
    exact = _exact_gradient(ph, R, L, ions, occ0, volts, w)

    def simulate(theta):
        phx = ph.replace(**dict(zip(THETA, theta)))
        p = oracle.OracleParams(phx, [R] * D, [L] * D)
        out = oracle.run(p, [protocol] * D, np.tile(occ0.reshape(-1), D), 0, n_steps)
        return (out["dec"][:, :, 0] * w[:, None]).sum(axis=0)

    theta = [getattr(ph, k) for k in THETA]
    mean, per = crn_fd(simulate, theta, h=1e-2)
    se = per.std(axis=1) / math.sqrt(D)
    for q in range(4):
        assert abs(mean[q] - exact[q]) < 4.5 * se[q] + 1e-3 * abs(exact[q]), (THETA[q], mean[q], exact[q], se[q])


def test_coul64_option_and_tolerance_scales():
    """The coul64 option gives the score terms the binary64 Coulomb sum rounded
    once to binary32.  The binary64 path is unchanged by it; the binary32 path
    keeps its decisions (final state, accepted hops) and its gradient moves by
    no more than a change of each Coulomb part by the binary32 sum's error
    bound ((n + 1) eps A, n window terms) plus one rounding, with the resulting
    roundings of the exponent's argument, allow: 2 eps sens_arg + (n + 3) eps
    sens_b.  The accepted-hop count has the parity and at least the size of the
    net hop count."""
    protos = [triangle(1.0, 60e-12), constant(-0.4)]
    for precision in (FP64, FP32):
        ph = _physics(precision=precision, ea_ev=0.15, seed=5)
        p = oracle.OracleParams(ph, [6, 3], [40, 23])
        occ = oracle.fill(p, [0.3, 0.45])
        W = np.random.default_rng(2).normal(size=(40, 2))
        a = oracle.score_replay(p, protos, occ, 0, W)
        b = oracle.score_replay(p, protos, occ, 0, W, coul64=True)
        assert np.array_equal(a["occ"], b["occ"]) and np.array_equal(a["hops"], b["hops"])
        fwd = oracle.run(p, protos, occ.copy(), 0, 40, want_dec=False)
        net = fwd["net"].sum(axis=0)
        assert np.all(a["hops"] >= np.abs(net)) and np.all((a["hops"] - net) % 2 == 0)
        assert np.all(b["sens_b"] > 0) and np.all(b["sens_arg"] > b["sens"])
        if precision == FP64:
            assert np.array_equal(a["grad"], b["grad"])
        else:
            eps, n = 2.0 ** -23, (2 * ph.rail_range + 1) * (2 * ph.cutoff_sites + 2)
            diff = np.abs(a["grad"] - b["grad"])
            assert np.any(diff > 0)
            assert np.all(diff <= 2 * eps * b["sens_arg"] + (n + 3) * eps * b["sens_b"])
