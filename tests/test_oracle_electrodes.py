"""Pins of the oracle's open electrodes (CPU only).

With open electrodes each rail's two ends exchange ions with reservoirs: the
grounded one behind site 0 and the biased one behind site L-1, each a virtual
site (-1 and L) whose ion has the reservoir energy mu plus its bias energy and
no Coulomb interaction; a transfer is one more bond of the checkerboard with
the electrode's barrier and the rate law of any hop.  Pinned here:
  * the transfer's energy change against E(after) - E(before) of the whole
    lattice energy, corrected by the reservoir ion's energy, computed by the
    independent enumerator (several geometries, both sides, both
    directions, both precisions' definitions);
  * the transfer words: Philox4x32-10 at the stated counter (stream 3),
    distinct from every hop and placement word;
  * equilibrium: with no ion-ion coupling and both reservoirs at the same
    energy, the grand-canonical measure exp(-beta (E - mu* N)) is exactly
    stationary under each half-step (detailed balance of every bond);
  * the whole chain: replica histograms of the oracle against the exact
    distribution P_n = T1 T0 ... P_0 over every configuration (chi-square),
    and the mean net transfer count per step (within 4 standard errors);
  * closed electrodes (None for a device) leave the trajectory bit for bit
    the same as without the option."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.exact_chain import Lattice
from workloads import FP32, FP64, Physics, constant, triangle


def _physics(**kw):
    base = dict(precision=FP64, ea_ev=0.06, coulomb_kappa_v=0.04, screening_sites=4.0,
                cutoff_sites=16, rail_range=1, seed=11)
    base.update(kw)
    return Physics(**base)


@pytest.mark.parametrize("R,L,m,cut", [(1, 6, 1, 16), (3, 5, 1, 2), (2, 7, 2, 6), (4, 4, 1, 1)])
def test_transfer_energy_is_energy_difference(R, L, m, cut):
    ph = _physics(rail_range=m, cutoff_sites=cut, coulomb_kappa_v=0.05)
    el = (0.05, 0.02, 0.07, -0.03)
    lat = Lattice(R, L, None, ph, electrodes=el)
    p = oracle.OracleParams(ph, [R], [L])
    g = np.random.default_rng(R * 100 + L)
    for trial in range(20):
        x = (g.random((R, L)) < 0.5).astype(np.int8)
        V = float(g.uniform(-2, 2))
        r = int(g.integers(R))
        for side in (0, 1):
            site = 0 if side == 0 else L - 1
            inject = x[r, site] == 0
            mu = el[1] if side == 0 else el[3]
            got = oracle.electrode_delta_energy(p, R, L, x, r, side, inject, V, mu)
            _, ref = lat.transfer_probability(x, r, side, V)
            assert abs(got - ref) <= 1e-12 * (1 + abs(ref)), (trial, side, got, ref)


def test_transfer_energy_binary32_is_rounded_binary64():
    """The binary32 definition differs from binary64 only by rounding."""
    ph64 = _physics(coulomb_kappa_v=0.05)
    p64 = oracle.OracleParams(ph64, [2], [9])
    p32 = oracle.OracleParams(ph64.replace(precision=FP32), [2], [9])
    g = np.random.default_rng(3)
    for _ in range(30):
        x = (g.random((2, 9)) < 0.4).astype(np.int8)
        V = float(g.uniform(-1, 1))
        for side in (0, 1):
            inject = bool(g.integers(2))
            a = oracle.electrode_delta_energy(p64, 2, 9, x, 1, side, inject, V, 0.03)
            b = oracle.electrode_delta_energy(p32, 2, 9, x, 1, side, inject, V, 0.03)
            assert b == float(np.float32(b))
            assert abs(a - b) <= 1e-6 * (1 + abs(a))


def test_transfer_words():
    seed = 0xDEADBEEF12345
    key = [seed & 0xFFFFFFFF, seed >> 32]
    words = set()
    for d in (0, 3):
        for r in (0, 7):
            for n in (0, 5):
                for h in (0, 1):
                    blk = oracle.philox([0, r, n, (d << 4) | (3 << 1) | h], key)
                    for side in (0, 1):
                        w = oracle.electrode_word(seed, d, n, r, h, side)
                        assert w == blk[side]
                        words.add(w)
    assert len(words) == 2 * 2 * 2 * 2 * 2
    # no overlap with the hop and placement counters: their fourth counter
    # words are 16 d + h and 16 d + 2, the transfers' 16 d + 6 + h
    hop = {oracle.hop_word(seed, d, n, r, s) for d in (0, 3) for r in (0, 7) for n in (0, 5) for s in range(16)}
    assert not (hop & words)


@pytest.mark.parametrize("R,L,V", [(1, 5, 0.0), (1, 4, 0.3), (2, 3, -0.4)])
def test_grand_canonical_measure_is_stationary(R, L, V):
    """No ion-ion coupling, a uniform barrier, both reservoirs at the same
    energy (mu_bias chosen so that mu + q V_app(virtual site) is equal): each
    half-step's matrix is column-stochastic and leaves exp(-beta (E - mu* N))
    unchanged.  The barriers keep every probability below 1 (a clamped
    probability breaks detailed balance)."""
    ph = _physics(coulomb_kappa_v=0.0, ea_ev=0.12)
    mu_g = 0.02
    mu_b = mu_g + ph.field_coupling * V * (-0.5) / L - ph.field_coupling * V * (L + 0.5) / L
    lat = Lattice(R, L, None, ph, electrodes=(0.12, mu_g, 0.3, mu_b))
    assert abs(lat.reservoir_energy(0, V) - lat.reservoir_energy(1, V)) < 1e-15
    pi = lat.grand_canonical(V)
    for h in (0, 1):
        T, _ = lat.half_step_matrix(h, V)
        assert np.allclose(T.sum(axis=0), 1.0, atol=1e-14)
        assert np.abs(T @ pi - pi).max() < 1e-14


def test_unequal_reservoirs_are_not_in_equilibrium():
    """A reservoir energy difference drives a current: the grand-canonical
    measure of either reservoir is then not stationary (the pin above is not
    vacuous)."""
    ph = _physics(coulomb_kappa_v=0.0)
    lat = Lattice(1, 4, None, ph, electrodes=(0.05, 0.05, 0.05, -0.05))
    pi = lat.grand_canonical(0.0)
    T0, _ = lat.half_step_matrix(0, 0.0)
    T1, _ = lat.half_step_matrix(1, 0.0)
    assert np.abs(T1 @ (T0 @ pi) - pi).max() > 1e-4


def _histogram(lat, ph, R, L, occ0, protocol, steps, D, el):
    p = oracle.OracleParams(ph, [R] * D, [L] * D)
    occ = np.tile(occ0.reshape(-1), D)
    out = oracle.run(p, [protocol] * D, occ, 0, steps, want_dec=False, electrodes=[el] * D)
    idx = np.array([lat.state_of(x) for x in occ.reshape(D, R, L)])
    return np.bincount(idx, minlength=len(lat.states)), out["net"]


@pytest.mark.parametrize("R,L,el,protocol", [
    (1, 5, (0.05, 0.03, 0.06, -0.02), constant(0.35)),
    (1, 4, (0.04, -0.02, 0.04, 0.05), triangle(0.8, 6e-12)),
    (2, 3, (0.06, 0.0, 0.05, 0.01), constant(-0.5)),
])
def test_oracle_matches_exact_chain_with_open_electrodes(R, L, el, protocol):
    """Replica histograms against the exact distribution over every
    configuration (chi-square at 1e-4), and the mean net count per step
    (interior hops and transfers toward site 0's side minus the rest) within
    4 standard errors."""
    ph = _physics()
    lat = Lattice(R, L, None, ph, electrodes=el)
    occ0 = np.zeros((R, L), dtype=np.int8)
    occ0[:, ::2] = 1
    steps, D = 4, 30000
    volts = [oracle.protocol_voltage(protocol[0], protocol[1], n * ph.dt_s) for n in range(steps)]
    P0 = np.zeros(len(lat.states))
    P0[lat.state_of(occ0)] = 1.0
    ex = lat.evolve(P0, volts)
    hist, net = _histogram(lat, ph, R, L, occ0, protocol, steps, D, el)
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
        m, se = net[n].mean(), net[n].std() / math.sqrt(D)
        assert abs(m - ex["net"][n]) < 4 * se + 1e-12, (n, m, ex["net"][n], se)
    # the ion number is not conserved
    occ_counts = {int(lat.states[i].sum()) for i in np.nonzero(hist)[0]}
    assert len(occ_counts) > 1


def test_closed_electrodes_change_nothing():
    ph = _physics(ea_ev=0.08)
    p = oracle.OracleParams(ph, [6, 4], [20, 13])
    occ = oracle.fill(p, [0.3, 0.5])
    a, b = occ.copy(), occ.copy()
    prot = [triangle(1.0, 50e-12), constant(0.4)]
    ra = oracle.run(p, prot, a, 0, 60)
    rb = oracle.run(p, prot, b, 0, 60, electrodes=[None, None])
    assert np.array_equal(a, b) and np.array_equal(ra["net"], rb["net"]) and np.array_equal(ra["dec"], rb["dec"])


def test_open_electrodes_fill_an_empty_lattice():
    """Reservoirs far above the lattice's site energy fill an empty lattice
    (ion number grows) and ones far below empty a full one."""
    ph = _physics(ea_ev=0.05, coulomb_kappa_v=0.0)
    p = oracle.OracleParams(ph, [8], [10])
    empty = np.zeros(80, dtype=np.int8)
    oracle.run(p, [constant(0.0)], empty, 0, 400, electrodes=[(0.02, 0.3, 0.02, 0.3)])
    assert empty.sum() > 70
    full = np.ones(80, dtype=np.int8)
    oracle.run(p, [constant(0.0)], full, 0, 400, electrodes=[(0.02, -0.3, 0.02, -0.3)])
    assert full.sum() < 10
