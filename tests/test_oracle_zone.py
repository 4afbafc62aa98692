"""Pins of the oracle's paper-literal zone model (SI S2.1; CPU only).

Pinned here:
  * the zone index against the paper's definition z = ceil(X / (L_x / Z)),
    evaluated in exact rational arithmetic for every column;
  * the table against Eqs. S2-S4: P_right / P_left = B = exp(-dE / kT) and
    P_left + P_right = P0, with dE = q dV_net d_hop / t_dev (Eq. S1);
  * the space-charge reading: no correction for equal zone populations, a
    correction linear in the factor, mirror antisymmetry (reflect the rail
    and the bias: left and right swap), and the sign (a pile of ions repels);
  * the two uniforms per ion and step: the words of the pinned Philox4x32-10
    at the stated counter, distinct across ions and steps;
  * conservation and exclusion over long runs, and the tallies against a
    recount;
  * the whole one-step and two-step distributions of single small rails
    against exact enumeration of every trial outcome (chi-square), with and
    without the space-charge term;
  * closed forms for one free ion far from the walls: mean displacement per
    step P_left - P_right and mean squared displacement P_left + P_right -
    2 P_left P_right.
Whole trajectories of the zone model are "parity unpinned": the paper prints
no numbers for them (its figures are placeholders)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.exact_zone import step_distribution

KT300 = 8.617333262e-5 * 300.0


@pytest.mark.parametrize("L,Z", [(200, 10), (15, 10), (37, 10), (7, 3), (10, 10), (1000, 7)])
def test_zone_index_is_the_papers_definition(L, Z):
    for x in range(1, L + 1):
        width = Fraction(L, Z)
        expect = math.ceil(Fraction(x) / width)
        assert oracle.zone_index(x, L, Z) == expect, (x, L, Z)
    # every zone is used and zones are monotone
    zs = [oracle.zone_index(x, L, Z) for x in range(1, L + 1)]
    assert zs[0] >= 1 and zs[-1] == Z and all(b >= a for a, b in zip(zs, zs[1:]))


@pytest.mark.parametrize("V", [0.0, 0.7, -2.5, 5.0])
def test_table_follows_eqs_s1_to_s4(V):
    p = oracle.ZoneParams(rails=100, ions=60, sites=200, p0=0.4, v_factor=2e-4)
    counts = np.array([900, 700, 600, 500, 550, 580, 600, 620, 480, 470])
    pl, pr, dv = oracle.zone_table(p, V, counts)
    dE = dv * p.s.hop_over_thickness
    assert np.allclose(pr / pl, np.exp(-dE / KT300), rtol=1e-13, atol=0)
    assert np.allclose(pl + pr, 0.4, rtol=1e-14, atol=0)
    assert np.all(pl > 0) and np.all(pr > 0)


def test_space_charge_reading():
    p = oracle.ZoneParams(rails=10, ions=30, sites=100, p0=0.5, v_factor=1e-3)
    even = np.full(10, 30)
    _, _, dv = oracle.zone_table(p, 1.3, even)
    assert np.allclose(dv, 1.3, rtol=0, atol=1e-15)           # equal populations: no correction
    counts = np.array([80, 40, 30, 25, 20, 20, 25, 20, 20, 20])
    _, _, dv1 = oracle.zone_table(p, 1.3, counts)
    p2 = oracle.ZoneParams(rails=10, ions=30, sites=100, p0=0.5, v_factor=2e-3)
    _, _, dv2 = oracle.zone_table(p2, 1.3, counts)
    assert np.allclose(dv2 - 1.3, 2.0 * (dv1 - 1.3), rtol=1e-12, atol=1e-15)   # linear in the factor
    # a pile at the grounded electrode pushes ions away from it (drop below V)
    assert np.all(dv1 < 1.3)
    # mirror: reflect the populations and the bias, left and right swap
    pl, pr, _ = oracle.zone_table(p, 1.3, counts)
    ml, mr, _ = oracle.zone_table(p, -1.3, counts[::-1])
    assert np.allclose(pl, mr[::-1], rtol=1e-13) and np.allclose(pr, ml[::-1], rtol=1e-13)


def test_uniforms_are_philox_words():
    seed = 0x1234_5678_9ABC
    seen = set()
    for rail in (0, 3):
        for ion in range(6):
            for n in (0, 1, 77):
                wr, wl = oracle.zone_words(seed, rail, ion, n)
                blk = oracle.philox([ion >> 1, rail, n, 2 << 1], [seed & 0xFFFFFFFF, seed >> 32])
                assert (wr, wl) == (blk[2 * (ion & 1)], blk[2 * (ion & 1) + 1])
                seen.update([(wr,), (wl,)])
    assert len(seen) == 2 * 2 * 6 * 3


def _random_X(g, rails, ions, sites):
    return np.array([np.sort(g.choice(sites, ions, replace=False)) + 1 for _ in range(rails)], dtype=np.int32)


def test_conservation_exclusion_and_tallies():
    g = np.random.default_rng(4)
    rails, ions, L = 16, 12, 30
    p = oracle.ZoneParams(rails, ions, L, p0=0.6, v_factor=3e-3, seed=11)
    X = _random_X(g, rails, ions, L)
    prot = ([0.0, 20e-3, 40e-3], [4.0, -4.0, 0.0])
    moved = 0
    for k in range(8):
        before = X.copy()
        out = oracle.zone_run(p, prot, X, 25 * k, 25)
        assert np.all(np.diff(X, axis=1) >= 1) and X.min() >= 1 and X.max() <= L
        assert X.shape == (rails, ions)
        zones = np.zeros(10, dtype=np.int64)
        for x in X.reshape(-1):
            zones[oracle.zone_index(int(x), L, 10) - 1] += 1
        assert np.array_equal(out["zones"][-1], zones)
        assert out["zones"].sum(axis=1).tolist() == [rails * ions] * 25
        # each left move lowers the column sum by 1, each right move raises it
        assert int(before.sum()) - int(X.sum()) == int(out["net"].sum())
        moved += int(np.abs(out["net"]).sum())
    assert moved > 100


def _chi2(counts, probs, n):
    keys = [k for k in probs if probs[k] * n >= 5]
    rest_p = 1.0 - sum(probs[k] for k in keys)
    obs = [counts.get(k, 0) for k in keys]
    exp_ = [probs[k] * n for k in keys]
    other = n - sum(obs)
    if rest_p * n >= 5:
        obs.append(other)
        exp_.append(rest_p * n)
    else:
        assert other <= max(10, 10 * rest_p * n), (other, rest_p * n)
    chi = sum((o - e) ** 2 / e for o, e in zip(obs, exp_))
    return chi, len(obs) - 1


@pytest.mark.parametrize("X0,V,vf,steps", [
    ((2, 4, 5), 0.8, 0.0, 1),
    ((1, 3, 6), -0.5, 0.0, 2),
    ((2, 4, 5), 0.3, 0.02, 1),     # space charge on: the zone populations change the table
    ((3, 5), 0.0, 0.05, 2),
])
def test_distribution_matches_exact_enumeration(X0, V, vf, steps):
    """Independent single-rail runs (one seed each) against the exact
    distribution after `steps` steps (chi-square at 1e-4)."""
    L, n_runs = 6, 12000
    base = oracle.ZoneParams(1, len(X0), L, zones=3, p0=0.7, kT=0.05, v_factor=vf, hop_over_thickness=0.5)
    dist = {tuple(X0): 1.0}
    for _ in range(steps):
        nxt = {}
        for x, q in dist.items():
            for y, r in step_distribution(base, x, V).items():
                nxt[y] = nxt.get(y, 0.0) + q * r
        dist = nxt
    assert abs(sum(dist.values()) - 1.0) < 1e-12
    counts = {}
    for seed in range(n_runs):
        p = oracle.ZoneParams(1, len(X0), L, zones=3, p0=0.7, kT=0.05, v_factor=vf, hop_over_thickness=0.5,
                              seed=seed * 7919 + 1)
        X = np.array([X0], dtype=np.int32)
        oracle.zone_run(p, ([0.0], [V]), X, 0, steps)
        key = tuple(int(v) for v in X[0])
        counts[key] = counts.get(key, 0) + 1
    for k in counts:
        assert k in dist, k     # no state outside the exact support (exclusion, walls, conflicts)
    chi, dof = _chi2(counts, dist, n_runs)
    from scipy.stats import chi2
    assert chi2.sf(chi, dof) > 1e-4, (chi, dof, counts, dist)


def test_free_ion_closed_forms():
    """One ion per rail far from the walls, no space charge (every zone has the
    same probabilities): per step the displacement is +1 with probability
    P_r (1 - P_l) and -1 with P_l (1 - P_r), independently from step to step,
    so its mean is P_r - P_l and its mean square P_l + P_r - 2 P_l P_r."""
    rails, L, steps = 20000, 400, 12
    p = oracle.ZoneParams(rails, 1, L, zones=10, p0=0.6, v_factor=0.0, seed=3)
    V = 1.5
    pl, pr, _ = oracle.zone_table(p, V, np.ones(10))
    assert np.allclose(pl, pl[0]) and np.allclose(pr, pr[0])
    X = np.full((rails, 1), 200, dtype=np.int32)
    oracle.zone_run(p, ([0.0], [V]), X, 0, steps)
    d = X[:, 0] - 200.0
    mean1 = pr[0] - pl[0]
    var1 = pl[0] + pr[0] - 2 * pl[0] * pr[0] - mean1 ** 2
    m_exp, v_exp = steps * mean1, steps * var1
    assert abs(d.mean() - m_exp) < 4.5 * math.sqrt(v_exp / rails)
    # sample variance of a sum of i.i.d. three-point steps: its standard error
    # is below 1.5 v sqrt(2 / n) for these probabilities
    assert abs(d.var() - v_exp) < 4.5 * 1.5 * v_exp * math.sqrt(2.0 / rails)
