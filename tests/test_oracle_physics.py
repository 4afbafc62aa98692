"""Pins of the oracle's step against closed forms, the energy function and
invariants (CPU only).  The oracle is kmc_oracle.c; the quantities here are
derived independently from the paper's definitions (see each test)."""
import math

import numpy as np
import pytest

import oracle
from oracle.exact_chain import Lattice
from workloads import FP32, FP64, Physics, constant, small_case, step_then_relax, triangle


def _ea_for(p0: float, ph: Physics) -> float:
    """barrier giving a zero-field hop probability p0 (p = nu0 dt exp(-Ea/kT))"""
    return ph.kT_ev * math.log(ph.nu0_hz * ph.dt_s / p0)


# ----------------------------------------------------------------- energy
@pytest.mark.parametrize("R,L,m,cut,lam", [
    (6, 40, 1, 16, 4.0),      # the cutoff screened kernel of the configs
    (3, 30, 2, 16, 4.0),      # rail_range larger than the ring allows: distinct rails once
    (2, 25, 1, 8, 4.0),       # the two neighbours of a rail are the same rail
    (1, 33, 1, 16, 4.0),      # a single rail
    (9, 24, 4, 23, 0.0),      # unscreened 1/r over the whole rail and +-4 rails
    (5, 20, 4, 19, 0.0),      # +-4 rails on a ring of 5
])
def test_delta_energy_is_energy_difference(R, L, m, cut, lam):
    """The oracle's bond-window sum equals E(after) - E(before) of the lattice
    energy sum_s qV_app(s) x_s + 1/2 sum_{i!=j} K_ij x_i x_j (main text section
    3: bias plus Coulomb field of nearby ions; SI Eq. S1 for the bias drop)."""
    ph = Physics(precision=FP64, coulomb_kappa_v=0.037, screening_sites=lam, cutoff_sites=cut,
                 rail_range=m, field_coupling=0.8)
    lat = Lattice(R, L, None, ph)
    p = oracle.OracleParams(ph, [R], [L])
    rng = np.random.default_rng(R * 100 + L)
    for trial in range(25):
        x = (rng.random((R, L)) < 0.45).astype(np.int8)
        V = float(rng.uniform(-3, 3))
        cands = [(r, s) for r in range(R) for s in range(L - 1) if x[r, s] != x[r, s + 1]]
        for (r, s) in cands[:: max(1, len(cands) // 6)]:
            o, t = (s, s + 1) if x[r, s] else (s + 1, s)
            y = x.copy()
            y[r, o], y[r, t] = 0, 1
            ref = lat.energy(y, V) - lat.energy(x, V)
            got = oracle.delta_energy(p, R, L, x, r, o, t, V)
            assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (trial, r, s, got, ref)
            got32 = oracle.delta_energy(p, R, L, x, r, o, t, V, fp32=True)
            assert abs(got32 - ref) <= 2e-6 * max(1.0, abs(ref))


def test_kernel_special_values():
    """K(ds, dr) = kappa exp(-d/lambda)/d inside the window, zero outside and at
    the origin; the unscreened form is kappa/d."""
    ph = Physics(coulomb_kappa_v=0.025, screening_sites=4.0, cutoff_sites=16, rail_range=1)
    p = oracle.OracleParams(ph, [8], [64])
    assert oracle.kernel(p, 0, 0) == 0.0
    assert oracle.kernel(p, 1, 0) == pytest.approx(0.025 * math.exp(-0.25), rel=1e-15)
    assert oracle.kernel(p, 3, 1) == pytest.approx(0.025 * math.exp(-math.sqrt(10) / 4) / math.sqrt(10), rel=1e-15)
    assert oracle.kernel(p, 16, 0) > 0.0 and oracle.kernel(p, 17, 0) == 0.0
    assert oracle.kernel(p, -16, 1) > 0.0 and oracle.kernel(p, 0, 2) == 0.0
    pu = oracle.OracleParams(ph.replace(screening_sites=0.0, rail_range=4), [8], [64])
    assert oracle.kernel(pu, 3, 4) == pytest.approx(0.025 / 5.0, rel=1e-15)


def test_hop_probability_forms():
    """p = min(nu0 dt exp(-(Ea + dE/2)/kT), 1): the forward/backward ratio of a
    hop and its reverse is exp(-dE/kT) (detailed balance, main text section 3),
    and p saturates at 1."""
    ph = Physics()
    p = oracle.OracleParams(ph, [1], [8])
    for dE in (-0.05, -0.01, 0.0, 0.013, 0.04):
        f = oracle.hop_prob(p, 0.3, dE)
        b = oracle.hop_prob(p, 0.3, -dE)
        assert f / b == pytest.approx(math.exp(-dE / ph.kT_ev), rel=1e-13)
        f32 = oracle.hop_prob(p, 0.3, dE, fp32=True)
        assert f32 == pytest.approx(f, rel=2e-6)
    assert oracle.hop_prob(p, -1.0, 0.0) == 1.0
    # paper constants: nu0 = 1e12 Hz, Ea = 0.3 eV, kT = 0.0259 eV, dt = 1 ps
    assert oracle.hop_prob(p, 0.3, 0.0) == pytest.approx(9.32314e-6, rel=1e-5)


# --------------------------------------------------------------- protocol
def test_protocol_piecewise_linear():
    t, v = triangle(2.0, 100e-9)  # 0 -> +2 at 25 ns -> -2 at 75 ns -> 0 at 100 ns
    f = lambda x: oracle.protocol_voltage(t, v, x)
    assert f(-1e-9) == 0.0
    assert f(0.0) == 0.0
    assert f(12.5e-9) == pytest.approx(1.0, abs=1e-12)
    assert f(25e-9) == pytest.approx(2.0, abs=1e-12)
    assert f(50e-9) == pytest.approx(0.0, abs=1e-12)
    assert f(62.5e-9) == pytest.approx(-1.0, abs=1e-12)
    assert f(100e-9) == 0.0 and f(1.0) == 0.0
    ts, vs = step_then_relax(1.0, 10e-9)   # jump at 10 ns: right-continuous
    g = lambda x: oracle.protocol_voltage(ts, vs, x)
    assert g(9.999e-9) == 1.0 and g(10e-9) == 0.0 and g(20e-9) == 0.0
    assert oracle.protocol_voltage([0.0], [0.7], 5.0) == 0.7
    assert oracle.protocol_voltage([], [], 5.0) == 0.0


# ----------------------------------------------------------------- filling
def test_fill_counts_and_ranks():
    """floor(f L + 1/2) ions per rail (fixed count per rail, SI S2.1), placed on
    the sites with the smallest placement words."""
    wl = small_case(5, 37, filling=0.3)
    p = oracle.params_for(wl)
    occ = oracle.fill(p, [0.3]).reshape(5, 37)
    n = int(math.floor(0.3 * 37 + 0.5))
    assert (occ.sum(axis=1) == n).all()
    for r in range(5):
        words = np.array([oracle.place_word(0, 0, r, s) for s in range(37)])
        chosen = set(np.lexsort((np.arange(37), words))[:n].tolist())
        assert set(np.nonzero(occ[r])[0].tolist()) == chosen
    assert oracle.ions_per_rail(0.2, 128) == 26 and oracle.ions_per_rail(0.3, 1024) == 307


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("precision", [FP64, FP32])
def test_conservation_tallies_deciles(precision):
    """Per step: ions per rail conserved (no inter-rail motion), occupancy stays
    0/1, sum_s s*occ drops by exactly the net hop count toward site 0, and the
    decile counts equal a recount (SI S3 decile observables)."""
    R, L = 6, 50
    wl = small_case(R, L, filling=0.35, precision=precision, ea_ev=0.12,
                    protocol=triangle(3.0, 40e-12))
    p = oracle.params_for(wl)
    occ = oracle.fill(p, wl.filling)
    per_rail = occ.reshape(R, L).sum(axis=1).copy()
    for k in range(40):
        pos_before = int((occ.reshape(R, L) * np.arange(L)).sum())
        out = oracle.run(p, wl.protocols, occ, k, 1)
        x = occ.reshape(R, L)
        assert set(np.unique(x)) <= {0, 1}
        assert (x.sum(axis=1) == per_rail).all()
        pos_after = int((x * np.arange(L)).sum())
        assert pos_before - pos_after == int(out["net"][0, 0])
        dec = np.zeros(10, dtype=np.int64)
        for s in range(L):
            dec[(10 * s) // L] += x[:, s].sum()
        assert (out["dec"][0, 0] == dec).all()


def test_bond_order_does_not_matter():
    """Every decision of a half-step reads the state at its start, so visiting
    the bonds in a random order gives the identical trajectory."""
    wl = small_case(7, 64, filling=0.4, ea_ev=0.1, n_devices=2)
    p = oracle.params_for(wl)
    a = oracle.fill(p, wl.filling)
    b = a.copy()
    ra = oracle.run(p, wl.protocols, a, 0, 30)
    rb = oracle.run(p, wl.protocols, b, 0, 30, shuffle_seed=987654321)
    assert (a == b).all() and (ra["net"] == rb["net"]).all()
    assert np.abs(ra["net"]).sum() > 0


def test_rail_window_light_cone():
    """Updating only rails [lo, hi) reproduces the full run on rails
    [lo + 2k, hi - 2k) after k steps (a rail feels its neighbours only through
    the +-1-rail Coulomb window, one rail per half-step)."""
    wl = small_case(40, 48, filling=0.3, ea_ev=0.1)
    p = oracle.params_for(wl)
    full = oracle.fill(p, wl.filling)
    part = full.copy()
    k = 3
    oracle.run(p, wl.protocols, full, 0, k)
    oracle.run(p, wl.protocols, part, 0, k, rail_lo=10, rail_hi=30)
    F, P_ = full.reshape(40, 48), part.reshape(40, 48)
    assert (F[10 + 2 * k:30 - 2 * k] == P_[10 + 2 * k:30 - 2 * k]).all()


def test_fp32_and_fp64_paths_agree_off_threshold():
    """binary32 and binary64 probabilities differ by rounding only, so the two
    trajectories coincide unless a draw lands within the logged window."""
    wl = small_case(8, 96, filling=0.3, ea_ev=0.12, n_devices=2)
    p64 = oracle.params_for(wl)
    p32 = oracle.params_for(wl, precision=FP32)
    a = oracle.fill(p64, wl.filling)
    b = a.copy()
    ra = oracle.run(p64, wl.protocols, a, 0, 50)
    rb = oracle.run(p32, wl.protocols, b, 0, 50)
    if ra["n_log"] == 0 and rb["n_log"] == 0:
        assert (a == b).all() and (ra["net"] == rb["net"]).all()


# ------------------------------------------------------------- closed forms
def _exact_free_msd(p: float, n_half: int) -> float:
    """A lone ion under the bond checkerboard attempts one direction per
    half-step, keeps it after a hop and reverses it after a failed attempt
    (the bond parity flips every half-step).  With iid Bernoulli(p) hops:
    E[v_i v_j] = p^2 (2p-1)^(j-i-1), E[v_i^2] = p, so
    MSD(N) = N p + 2 p^2 sum_{k=1}^{N-1} (N-k) (2p-1)^(k-1)  (-> 2p/(1-p) per step)."""
    q = 2 * p - 1
    s = sum((n_half - k) * q ** (k - 1) for k in range(1, n_half))
    return n_half * p + 2 * p * p * s


def test_free_diffusion_msd_exact():
    """kappa = 0, V = 0, one ion per rail away from the electrodes: the ensemble
    MSD matches the exact value of the persistent walk; for small p it is the
    free-diffusion law MSD = 2 nu a^2 t with nu = p/dt."""
    ph = Physics(precision=FP64, coulomb_kappa_v=0.0, rail_range=0)
    p0 = 0.2
    ph = ph.replace(ea_ev=_ea_for(p0, ph))
    R, L, steps = 4000, 256, 60
    p = oracle.OracleParams(ph, [R], [L])
    occ = np.zeros((R, L), dtype=np.int8)
    start = 128 + (np.arange(R) % 2)
    occ[np.arange(R), start] = 1
    oracle.run(p, [constant(0.0)], occ, 0, steps, want_dec=False)
    pos = np.argmax(occ.reshape(R, L), axis=1)
    disp = (pos - start).astype(np.float64)
    msd = float((disp ** 2).mean())
    exact = _exact_free_msd(p0, 2 * steps)
    se = float((disp ** 2).std() / math.sqrt(R))
    assert abs(msd - exact) < 4 * se, (msd, exact, se)
    assert abs(disp.mean()) < 4 * disp.std() / math.sqrt(R)
    assert 2 * p0 / (1 - p0) == pytest.approx(exact / steps, rel=0.05)


def _exact_mean_displacement(p_r: float, p_l: float, n_half: int, start_right: bool) -> float:
    """Two-state (attempt direction) chain of the lone ion: after a hop the
    direction is kept, after a failure it reverses."""
    pi_r = 1.0 if start_right else 0.0
    m = 0.0
    for _ in range(n_half):
        m += pi_r * p_r - (1 - pi_r) * p_l
        pi_r = pi_r * p_r + (1 - pi_r) * (1 - p_l)
    return m


def test_dilute_drift_exact():
    """kappa = 0 with a bias: the mean displacement equals the exact two-state
    chain value; its stationary drift 2(p_r - p_l)/(2 - p_r - p_l) per step
    reduces to a nu (e^{-beta qEa/2} - e^{+beta qEa/2}) for small p (a drift
    toward the grounded site 0 for V > 0)."""
    ph = Physics(precision=FP64, coulomb_kappa_v=0.0, rail_range=0)
    p0 = 0.2
    ph = ph.replace(ea_ev=_ea_for(p0, ph))
    R, L, steps, V = 4000, 400, 50, 8.0
    p = oracle.OracleParams(ph, [R], [L])
    occ = np.zeros((R, L), dtype=np.int8)
    start = 200 + (np.arange(R) % 2)
    occ[np.arange(R), start] = 1
    oracle.run(p, [constant(V)], occ, 0, steps, want_dec=False)
    pos = np.argmax(occ.reshape(R, L), axis=1)
    disp = (pos - start).astype(np.float64)
    half = ph.field_coupling * V / L / 2
    p_r = p0 * math.exp(-half / ph.kT_ev)
    p_l = p0 * math.exp(+half / ph.kT_ev)
    for parity in (0, 1):
        sel = (np.arange(R) % 2) == parity
        exact = _exact_mean_displacement(p_r, p_l, 2 * steps, start_right=(parity == 0))
        se = disp[sel].std() / math.sqrt(sel.sum())
        assert abs(disp[sel].mean() - exact) < 4 * se, (parity, disp[sel].mean(), exact, se)
    assert disp.mean() < 0


@pytest.mark.parametrize("R,L,m,cut,lam", [(6, 40, 4, 39, 0.0), (3, 24, 2, 10, 3.0), (9, 32, 4, 31, 0.0), (1, 16, 0, 15, 0.0)])
def test_dense_potential(R, L, m, cut, lam):
    """phi (binary64): (a) one ion alone makes phi = K at every other site and
    0 at its own; (b) phi(t) - K(1,0) - phi(o) equals the Coulomb part of the
    pinned energy change delta_energy - alpha V (t - o)/L for every candidate
    of random states; (c) phi is additive over ions."""
    ph = Physics(precision=FP64, coulomb_kappa_v=0.03, screening_sites=lam, cutoff_sites=cut, rail_range=m)
    p = oracle.OracleParams(ph, [R], [L])
    one = np.zeros(R * L, dtype=np.int8)
    r0, s0 = R // 2, L // 3
    one[r0 * L + s0] = 1
    phi1 = oracle.dense_potential(p, one).reshape(R, L)
    for r in range(R):
        dr = min((r - r0) % R, (r0 - r) % R)
        for s in range(L):
            assert phi1[r, s] == oracle.kernel(p, s - s0, dr), (r, s)
    rng = np.random.default_rng(R + L)
    for trial in range(3):
        occ = (rng.random(R * L) < 0.35).astype(np.int8)
        phi = oracle.dense_potential(p, occ).reshape(R, L)
        # additivity over ions
        acc = np.zeros((R, L))
        for i in np.flatnonzero(occ):
            e = np.zeros(R * L, dtype=np.int8)
            e[i] = 1
            acc += oracle.dense_potential(p, e).reshape(R, L)
        assert np.allclose(acc, phi, rtol=1e-12, atol=1e-15)
        S = occ.reshape(R, L)
        V = 0.37
        k10 = oracle.kernel(p, 1, 0)
        for r in range(R):
            for s in range(L - 1):
                if S[r, s] == S[r, s + 1]:
                    continue
                o, t = (s, s + 1) if S[r, s] else (s + 1, s)
                e_coul = oracle.delta_energy(p, R, L, S, r, o, t, V) - ph.field_coupling * V * (t - o) / L
                assert abs(phi[r, t] - k10 - phi[r, o] - e_coul) <= 1e-12 * (abs(phi[r, t]) + abs(phi[r, o]) + 1e-3)


def test_threaded_oracle_equals_single_thread():
    """The oracle's OpenMP path (rails of a device split over threads inside
    each half-step) gives the single-threaded result: occupancy, per-step net
    hops and deciles, and the same set of logged near-threshold draws."""
    from workloads import small_case
    wl = small_case(24, 96, filling=0.35, precision="fp32", ea_ev=0.05, n_devices=2, seed=9)
    p = oracle.params_for(wl)
    occ0 = oracle.fill(p, wl.filling)
    outs = []
    for threads in (1, 4):
        oracle.set_threads(threads)
        try:
            outs.append(oracle.run(p, wl.protocols, occ0.copy(), 0, 30, log_cap=65536))
        finally:
            oracle.set_threads(1)
    a, b = outs
    assert np.abs(a["net"]).sum() > 100
    for key in ("occ", "net", "dec"):
        assert np.array_equal(a[key], b[key]), key
    assert a["n_log"] == b["n_log"] and a["n_log"] <= 65536

    def as_set(log):
        return {(int(e["d"]), int(e["h"]), int(e["n"]), int(e["r"]), int(e["s"])) for e in log}
    assert as_set(a["log"]) == as_set(b["log"])
