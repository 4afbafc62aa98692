"""The oracle's whole step against exact enumeration of the Markov chain on tiny
lattices, and the enumerator against theory (CPU only)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.exact_chain import Lattice
from workloads import FP64, Physics, constant, triangle


def _physics(**kw):
    base = dict(precision=FP64, ea_ev=0.06, coulomb_kappa_v=0.04, screening_sites=4.0,
                cutoff_sites=16, rail_range=1, seed=11)
    base.update(kw)
    return Physics(**base)


@pytest.mark.parametrize("R,L,ions", [(1, 8, [3]), (2, 4, [2, 1]), (3, 3, [1, 2, 1])])
def test_half_steps_are_stochastic_and_boltzmann_stationary(R, L, ions):
    """Each half-step matrix is column-stochastic; with no ion-ion coupling and a
    static bias the Boltzmann measure at fixed ion number per rail is stationary
    under each half-step (detailed balance, main text section 3), including with
    a per-site barrier field (site energy -Ea)."""
    rng = np.random.default_rng(R * 10 + L)
    ea = rng.uniform(0.05, 0.1, size=R * L)
    ph = _physics(coulomb_kappa_v=0.0)
    lat = Lattice(R, L, ions, ph, ea_site=ea)
    for V in (0.0, 0.15):  # small enough that no probability saturates at 1
        pi = lat.boltzmann(V)
        for h in (0, 1):
            T, _ = lat.half_step_matrix(h, V)
            assert np.allclose(T.sum(axis=0), 1.0, atol=1e-14)
            assert np.abs(T @ pi - pi).max() < 1e-14


def _oracle_histogram(lat, ph, R, L, occ0, protocol, steps, D):
    p = oracle.OracleParams(ph, [R] * D, [L] * D)
    occ = np.tile(occ0.reshape(-1), D)
    out = oracle.run(p, [protocol] * D, occ, 0, steps, want_dec=False)
    idx = np.array([lat.state_of(x) for x in occ.reshape(D, R, L)])
    return np.bincount(idx, minlength=len(lat.states)), out["net"]


@pytest.mark.parametrize("R,L,ions,protocol", [
    (1, 8, [3], constant(0.35)),
    (2, 4, [2, 1], triangle(0.8, 6e-12)),
    (3, 3, [1, 2, 1], constant(-0.5)),
])
def test_oracle_matches_exact_chain(R, L, ions, protocol):
    """D independent replicas (one Philox stream each) of a tiny device: the
    histogram of final states passes a chi-square test against the exact
    distribution P_n = T1 T0 ... P_0, and the per-step mean net hop count agrees
    within 4 standard errors."""
    ph = _physics()
    lat = Lattice(R, L, ions, ph)
    rng = np.random.default_rng(5)
    occ0 = lat.states[rng.integers(len(lat.states))]
    steps, D = 4, 30000
    volts = [oracle.protocol_voltage(protocol[0], protocol[1], n * ph.dt_s) for n in range(steps)]
    P0 = np.zeros(len(lat.states))
    P0[lat.state_of(occ0)] = 1.0
    ex = lat.evolve(P0, volts)
    hist, net = _oracle_histogram(lat, ph, R, L, occ0, protocol, steps, D)
    expect = ex["P"][-1] * D
    keep = expect > 5
    obs = np.append(hist[keep], hist[~keep].sum())
    exp_ = np.append(expect[keep], expect[~keep].sum())
    if exp_[-1] == 0:
        obs, exp_ = obs[:-1], exp_[:-1]
    chi2 = ((obs - exp_) ** 2 / exp_).sum()
    pval = stats.chi2.sf(chi2, len(obs) - 1)
    assert pval > 1e-4, (chi2, len(obs), pval)
    for n in range(steps):
        m, se = net[:, :].mean(axis=1)[n], net[n].std() / math.sqrt(D)
        assert abs(m - ex["net"][n]) < 4 * se + 1e-12, (n, m, ex["net"][n], se)


def test_oracle_matches_exact_chain_with_barrier_field():
    """Same check with a per-site barrier field (origin-site barrier)."""
    R, L, ions = 2, 4, [1, 2]
    rng = np.random.default_rng(9)
    ea = rng.uniform(0.03, 0.1, size=R * L)
    ph = _physics()
    lat = Lattice(R, L, ions, ph, ea_site=ea)
    occ0 = lat.states[3]
    steps, D = 3, 30000
    P0 = np.zeros(len(lat.states))
    P0[lat.state_of(occ0)] = 1.0
    ex = lat.evolve(P0, [0.25] * steps)
    p = oracle.OracleParams(ph, [R] * D, [L] * D, ea_site=np.tile(ea, D))
    occ = np.tile(occ0.reshape(-1), D)
    oracle.run(p, [constant(0.25)] * D, occ, 0, steps, want_dec=False)
    idx = np.array([lat.state_of(x) for x in occ.reshape(D, R, L)])
    hist = np.bincount(idx, minlength=len(lat.states))
    expect = ex["P"][-1] * D
    keep = expect > 5
    chi2 = ((hist[keep] - expect[keep]) ** 2 / expect[keep]).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
