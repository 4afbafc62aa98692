"""HIP hop step vs the CPU oracle, element by element (needs an MI355X)."""
import math

import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import (FP32, FP64, Physics, c1_plain_fp64, c2_large_device, constant,
                       gaussian_barriers, small_case, step_then_relax, stdp_pair, triangle)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


MODES = [("half_step", 0), ("persistent", 0), ("persistent", 512), ("wave", 0), ("wave", 2048)]


def _sim(physics, rails, sites, occ=None, ea=None, mode="auto", tile_sites=0):
    from paper_2511_09413_amd import Simulator
    sim = Simulator(physics, rails, sites, occ=occ, ea=ea, tile_sites=tile_sites)
    if mode != "auto":
        sim.set_launch_mode(mode)
    return sim


@pytest.mark.parametrize("rails,sites,fill", [
    ([64], [128], [0.2]),
    ([3, 5, 2], [37, 100, 1000], [0.3, 0.05, 0.4]),
    ([2], [4096], [0.5]),
    ([7], [2], [0.5]),
])
def test_fill_random_matches_oracle(rails, sites, fill):
    ph = Physics(precision=FP32, seed=0xC0FFEE)
    sim = _sim(ph, rails, sites)
    sim.fill_random(fill)
    got = sim.read_occupancy()
    ref = oracle.fill(oracle.OracleParams(ph.replace(precision=FP64), rails, sites), fill)
    assert np.array_equal(got, ref)


def _run_parity(wl, n_steps, chunk, occ0=None, phys=None, mode="auto", tile_sites=0):
    ph = phys or wl.physics
    sim = _sim(ph, wl.rails, wl.sites, ea=wl.ea_site, mode=mode, tile_sites=tile_sites)
    p_or = oracle.OracleParams(ph, wl.rails, wl.sites, wl.ea_site)
    if occ0 is None:
        occ0 = oracle.fill(p_or, wl.filling)
    sim.load_occupancy(occ0)
    sim.set_protocols(wl.protocols)
    return lockstep(sim, p_or, wl.protocols, occ0, n_steps, chunk), sim


@pytest.mark.parametrize("mode,tile", MODES)
def test_c1_fp64_trajectory(mode, tile):
    """64 x 128, 20% filling, FP64, 0.5 V, kappa = 0.025 V, lambda = 4, cutoff
    16, +-1 rail: identical trajectory, tallies and deciles for 600 steps."""
    wl = c1_plain_fp64()
    st, sim = _run_parity(wl, 600, 200, mode=mode, tile_sites=tile)
    assert st["resyncs"] == 0
    assert sim.launch_mode == mode


@pytest.mark.parametrize("mode,tile", MODES)
def test_c1_validation_variant_many_hops(mode, tile):
    """Same lattice with Ea = 0.15 eV (p ~ 3e-3): thousands of hops; with
    512-site tiles the persistent kernel exchanges edge rails between 16 tiles."""
    wl = c1_plain_fp64()
    ph = wl.physics.replace(ea_ev=0.15)
    st, _ = _run_parity(wl, 300, 100, phys=ph, mode=mode, tile_sites=tile)
    assert st["hops"] > 100
    assert st["resyncs"] <= 1


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("mode,tile", MODES)
def test_ragged_multi_device_with_barrier_field(precision, mode, tile):
    """Heterogeneous devices (ragged site counts, several tiles per device),
    per-site barriers, triangle / step / spike-pair protocols."""
    rails, sites = [9, 40, 3, 1], [37, 300, 1000, 129]
    dt = np.float64 if precision == FP64 else np.float32
    n = sum(r * l for r, l in zip(rails, sites))
    ea = gaussian_barriers((n,), 0.12, 0.02, seed=4, dtype=dt)
    ph = Physics(precision=precision, seed=77, coulomb_kappa_v=0.03)
    protos = [triangle(2.0, 200e-12), step_then_relax(1.0, 60e-12), stdp_pair(20e-12, 30e-12, 10e-12),
              constant(-0.7)]
    from workloads import Workload
    wl = Workload("ragged", ph, rails, sites, [0.3, 0.2, 0.45, 0.5], protos, 0, ea_site=ea)
    st, _ = _run_parity(wl, 200, 50, mode=mode, tile_sites=tile)
    assert st["hops"] > 100


@pytest.mark.parametrize("mode,tile", MODES)
@pytest.mark.parametrize("R,L,m,cut,lam", [
    (1, 64, 1, 16, 4.0), (2, 50, 1, 16, 4.0), (3, 40, 2, 8, 4.0), (17, 96, 0, 16, 4.0),
    (12, 64, 4, 63, 0.0), (5, 33, 3, 5, 2.0), (40, 48, 2, 16, 4.0), (24, 160, 4, 30, 0.0),
    (16, 500, 4, 40, 0.0)])
def test_interaction_variants(R, L, m, cut, lam, mode, tile):
    ph = Physics(precision=FP64, seed=5, ea_ev=0.12, coulomb_kappa_v=0.04, screening_sites=lam,
                 cutoff_sites=cut, rail_range=m)
    wl = small_case(R, L, filling=0.35, precision=FP64, ea_ev=0.12, protocol=triangle(3.0, 80e-12))
    wl.physics = ph
    st, _ = _run_parity(wl, 80, 40, mode=mode, tile_sites=tile)
    assert st["steps"] == 80


def test_protocol_install_midrun_and_chunking():
    """A protocol installed at step n_set is relative to n_set; splitting a run
    into calls of different lengths gives the same trajectory."""
    ph = Physics(precision=FP32, seed=3, ea_ev=0.13)
    rails, sites = [16], [256]
    p_or = oracle.OracleParams(ph, rails, sites)
    occ0 = oracle.fill(p_or, [0.3])
    a = _sim(ph, rails, sites, occ=occ0)
    a.set_bias_protocol(*triangle(1.5, 100e-12))
    net_a = [a.run_steps(k, tallies=True)[0].cpu().numpy() for k in (7, 1, 30, 2)]
    a.set_bias_protocol(*step_then_relax(2.0, 10e-12))   # installed at step 40
    net_a.append(a.run_steps(25, tallies=True)[0].cpu().numpy())
    occ_o = occ0.copy()
    r1 = oracle.run(p_or, [triangle(1.5, 100e-12)], occ_o, 0, 40)
    r2 = oracle.run(p_or, [step_then_relax(2.0, 10e-12)], occ_o, 40, 25, n_set=[40])
    assert np.array_equal(np.concatenate(net_a[:4]), r1["net"])
    assert np.array_equal(net_a[4], r2["net"])
    assert np.array_equal(a.read_occupancy(), occ_o)
    cur, tot, t = a.read_current()
    assert tot[0] == int(r1["net"].sum() + r2["net"].sum())
    assert t == pytest.approx(65 * ph.dt_s)
    assert cur[0] == pytest.approx(1.602176634e-19 * tot[0] / (256 * ph.dt_s * 65))


def test_near_threshold_log_matches_oracle():
    """The GPU logs exactly the oracle's near-threshold draws (|u - p| < 1e-6)."""
    ph = Physics(precision=FP64, seed=9, ea_ev=0.02, coulomb_kappa_v=0.04)  # p near 0.5
    rails, sites = [32], [256]
    p_or = oracle.OracleParams(ph, rails, sites)
    occ0 = oracle.fill(p_or, [0.4])
    sim = _sim(ph, rails, sites, occ=occ0)
    sim.set_bias_protocol(*constant(0.3))
    sim.run_steps(200)
    occ_o = occ0.copy()
    out = oracle.run(p_or, [constant(0.3)], occ_o, 0, 200, log_cap=100000)
    log, n = sim.read_threshold_log()
    assert n == out["n_log"]
    key = lambda e: (int(e["n"]), int(e["h"]), int(e["r"]), int(e["s"]))
    assert sorted(map(key, log)) == sorted(map(key, out["log"]))
    if out["n_log"] == 0:
        assert np.array_equal(sim.read_occupancy(), occ_o)


# ------------------------------------------------------------- full size
@pytest.mark.parametrize("mode", ["half_step", "persistent", "wave"])
def test_c2_full_size_sampled(mode):
    """4096 x 1024, FP32, per-site barriers, in the benchmark's launch
    configuration: after 3 steps, rails [lo+6, hi-6) of several windows equal the
    oracle's light-cone runs, and every rail keeps its ion count."""
    wl = c2_large_device(n_steps=3)
    ph = wl.physics.replace(ea_ev=0.3)
    ea = wl.ea_site - np.float32(0.17)   # lower barriers: thousands of hops per step
    sim = _sim(ph, wl.rails, wl.sites, ea=ea, mode=mode)
    sim.fill_random(wl.filling)
    occ0 = sim.read_occupancy()
    sim.set_protocols(wl.protocols)
    net, _ = sim.run_steps(3, tallies=True)
    occ = sim.read_occupancy().reshape(4096, 1024)
    assert (occ.sum(axis=1) == occ0.reshape(4096, 1024).sum(axis=1)).all()
    p_or = oracle.OracleParams(ph, wl.rails, wl.sites, ea)
    for lo in (0, 1000, 2040, 4096 - 30):
        part = occ0.copy()
        oracle.run(p_or, wl.protocols, part, 0, 3, rail_lo=lo, rail_hi=lo + 30, want_dec=False)
        ref = part.reshape(4096, 1024)
        assert np.array_equal(occ[lo + 6:lo + 24], ref[lo + 6:lo + 24]), lo
    assert int(np.abs(net.cpu().numpy()).sum()) >= 0


@pytest.mark.parametrize("mode", ["persistent", "wave"])
def test_persistent_long_run_keeps_ring_protocol(mode):
    """4096 x 1024 run of a persistent strategy over 40 launches (40960
    steps): every neighbour wait completes (the kernel status stays clear) and
    every rail keeps its ion count.  A publication issued before the slot-reuse
    check made such long runs time out."""
    from paper_2511_09413_amd import Simulator
    wl = c2_large_device(n_steps=100_000)
    sim = Simulator(wl.physics, wl.rails, wl.sites, ea=wl.ea_site)
    sim.set_launch_mode(mode)
    assert sim.launch_mode == mode
    sim.fill_random(wl.filling)
    occ0 = sim.read_occupancy().reshape(4096, 1024).sum(axis=1)
    sim.set_protocols(wl.protocols)
    sim.run_steps(40 * 1024)
    sim.read_current()   # raises on a timed-out neighbour wait
    occ = sim.read_occupancy().reshape(4096, 1024).sum(axis=1)
    assert np.array_equal(occ, occ0)


@pytest.mark.parametrize("tile", [0, 2048])
def test_wave_snapshot_ring_wraps_under_many_hops(tile):
    """One- and two-rail wave tiles at a barrier low enough that nearly every
    half-step changes an edge rail: the snapshot ring wraps many times per
    launch (its slot reuse waits for both neighbours), over more than one
    launch, and the trajectory still follows the oracle step by step."""
    ph = Physics(precision=FP64, seed=31, ea_ev=0.06, coulomb_kappa_v=0.03)
    rails, sites = [6, 3], [1000, 500]
    from workloads import Workload
    wl = Workload("wave_ring", ph, rails, sites, [0.3, 0.4], [triangle(1.0, 400e-12), constant(0.5)], 0)
    st, sim = _run_parity(wl, 1100, 550, mode="wave", tile_sites=tile)
    assert sim.launch_mode == "wave"
    assert st["hops"] > 2000


@pytest.mark.parametrize("mode,tile", MODES)
def test_lowest_class_bound_above_one(mode, tile):
    """Per-site barriers N(0.08, 0.02) eV with an unscreened window of 40
    sites over +-2 rails: the prefilter's bound for the lowest barrier class
    exceeds 1 at every step (its threshold saturates), while lanes whose
    lowest class is higher keep bounds below 1.  The wave kernel's per-lane
    stage-0 bound, a scaled copy of the lowest class's threshold, must then
    pass every word to the exact check (it once rejected hops here: the
    trajectory left the oracle's at step 96)."""
    R, L = 16, 96
    ea = np.random.default_rng(3).normal(0.08, 0.02, size=R * L)
    ph = Physics(precision=FP64, seed=5, ea_ev=0.08, screening_sites=0.0, cutoff_sites=40, rail_range=2)
    from workloads import Workload
    wl = Workload("saturated_bound", ph, [R], [L], [0.3], [constant(0.6)], 0, ea_site=ea)
    st, _ = _run_parity(wl, 160, 40, mode=mode, tile_sites=tile)
    assert st["hops"] > 300


@pytest.mark.parametrize("mode,tile", [("persistent", 512), ("wave", 0)])
def test_neighbour_wait_failure_is_reported(mode, tile):
    """A neighbour wait declared hung (the wait limit set to 0 from the host, so
    every wait fails at once) ends the launch cleanly and the next read reports
    it; a new context then runs normally and follows the oracle."""
    from paper_2511_09413_amd import KMC_EHIP, KmcError
    wl = c1_plain_fp64()
    ph = wl.physics.replace(ea_ev=0.15)   # many hops: survivors at tile edges in every step
    sim = _sim(ph, wl.rails, wl.sites, mode=mode, tile_sites=tile)
    assert sim.launch_mode == mode
    p_or = oracle.OracleParams(ph, wl.rails, wl.sites)
    occ0 = oracle.fill(p_or, wl.filling)
    sim.load_occupancy(occ0)
    sim.set_protocols(wl.protocols)
    sim.set_wait_limit(0)
    sim.run_steps(50)
    with pytest.raises(KmcError) as err:
        sim.read_current()
    assert err.value.status == KMC_EHIP and "timed out" in str(err.value)
    sim.close()
    st, _ = _run_parity(wl, 40, 40, occ0=occ0, phys=ph, mode=mode, tile_sites=tile)
    assert st["steps"] == 40


@pytest.mark.parametrize("seed", range(12))
def test_wave_random_geometries(seed):
    """Seeded random lattices for the wave strategy: rail counts 1..40, sites
    2..2016 (pitches that are and are not multiples of 32), rail ranges 0..4,
    cutoffs 0..40, screened and unscreened, both precisions, 16 or 32 sites per
    lane; 60 steps in lockstep with the oracle.  Geometries the wave tiling
    cannot hold are skipped."""
    from paper_2511_09413_amd import KmcError, KMC_EUNSUPPORTED
    g = np.random.default_rng(1000 + seed)
    n_dev = int(g.integers(1, 4))
    m = int(g.integers(0, 5))
    l_max = 32 * (64 // max(m, 1)) - 32     # rails of this length fit the tiling at 32 sites per lane
    rails = [int(g.integers(1, 41)) for _ in range(n_dev)]
    sites = [int(g.integers(2, l_max + 1)) for _ in range(n_dev)]
    cut = int(g.integers(0, 41))
    lam = float(g.choice([0.0, 2.0, 4.0]))
    precision = FP64 if seed % 2 == 0 else FP32
    tile = [0, 2048][seed % 3 == 0]
    ph = Physics(precision=precision, seed=seed, ea_ev=0.13, coulomb_kappa_v=0.04, screening_sites=lam,
                 cutoff_sites=cut, rail_range=m)
    fill = [float(g.uniform(0.05, 0.6)) for _ in range(n_dev)]
    protos = [triangle(2.0, 120e-12), constant(-0.8), step_then_relax(1.5, 30e-12)][:n_dev]
    try:
        sim = _sim(ph, rails, sites, mode="wave", tile_sites=tile)
    except KmcError as e:
        if e.status != KMC_EUNSUPPORTED:
            raise
        pytest.skip(f"the wave tiling does not hold {rails} x {sites} with rail range {m}")
    p_or = oracle.OracleParams(ph, rails, sites)
    occ0 = oracle.fill(p_or, fill)
    sim.load_occupancy(occ0)
    sim.set_protocols(protos)
    st = lockstep(sim, p_or, protos, occ0, 60, 30)
    assert sim.launch_mode == "wave" and st["steps"] == 60


@pytest.mark.parametrize("mode", ["half_step", "persistent"])
@pytest.mark.parametrize("seed", range(6))
def test_random_geometries_other_strategies(seed, mode):
    """Seeded random lattices for the half-step and block-tile strategies: rail
    counts 1..24, sites 2..4096, rail ranges 0..4, cutoffs 0..40, screened and
    unscreened, both precisions, default or small forced tiles; 40 steps in
    lockstep with the oracle."""
    g = np.random.default_rng(2000 + 10 * seed + (mode == "persistent"))
    n_dev = int(g.integers(1, 4))
    m = int(g.integers(0, 5))
    rails = [int(g.integers(1, 25)) for _ in range(n_dev)]
    sites = [int(g.integers(2, 4097)) for _ in range(n_dev)]
    cut = int(g.integers(0, 41))
    lam = float(g.choice([0.0, 2.0, 4.0]))
    precision = FP64 if seed % 2 == 0 else FP32
    tile = int(g.choice([0, 512, 1024]))
    ph = Physics(precision=precision, seed=seed + 50, ea_ev=0.13, coulomb_kappa_v=0.04, screening_sites=lam,
                 cutoff_sites=cut, rail_range=m)
    fill = [float(g.uniform(0.05, 0.6)) for _ in range(n_dev)]
    protos = [triangle(2.0, 120e-12), constant(-0.8), step_then_relax(1.5, 30e-12)][:n_dev]
    from paper_2511_09413_amd import KmcError, KMC_EUNSUPPORTED
    try:
        sim = _sim(ph, rails, sites, mode=mode, tile_sites=tile)
    except KmcError as e:
        if e.status != KMC_EUNSUPPORTED:
            raise
        pytest.skip(f"the {mode} strategy does not hold {rails} x {sites} with rail range {m}")
    p_or = oracle.OracleParams(ph, rails, sites)
    occ0 = oracle.fill(p_or, fill)
    sim.load_occupancy(occ0)
    sim.set_protocols(protos)
    st = lockstep(sim, p_or, protos, occ0, 40, 20)
    assert sim.launch_mode == mode and st["steps"] == 40
