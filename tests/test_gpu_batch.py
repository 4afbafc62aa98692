"""Batches of heterogeneous devices in one call (needs an MI355X): persistent
launches over groups of whole devices against the oracle, and the full
256-device batch sampled device by device."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available, lockstep
from workloads import FP32, FP64, Physics, c3_batched, constant, step_then_relax, stdp_pair, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

RAILS = [5, 9, 3, 16, 1, 7, 12, 2, 6, 10, 4, 8]
SITES = [64, 130, 33, 96, 257, 48, 80, 500, 17, 112, 75, 40]
FILL = [0.3, 0.1, 0.45, 0.2, 0.5, 0.35, 0.25, 0.05, 0.4, 0.3, 0.15, 0.3]


def _protocols(n):
    kinds = [constant(0.6), triangle(1.0, 200e-12), step_then_relax(1.0, 60e-12), stdp_pair(20e-12, 30e-12),
             constant(-0.4)]
    return [kinds[i % len(kinds)] for i in range(n)]


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("mode,limit,tile_sites", [("persistent", 3, 512), ("persistent", 5, 512),
                                                   ("persistent", 0, 0), ("wave", 3, 0), ("wave", 0, 2048)])
def test_grouped_persistent_batch_matches_oracle(precision, mode, limit, tile_sites):
    """12 devices of different shapes, fillings and protocols; a persistent
    strategy split into groups of at most `limit` tiles (several launches per
    chunk) follows the oracle step by step."""
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=precision, seed=99, ea_ev=0.15)
    protos = _protocols(len(RAILS))
    sim = Simulator(ph, RAILS, SITES, tile_sites=tile_sites)
    if limit:
        sim.set_group_limit(limit)
    sim.set_launch_mode(mode)
    if limit:
        assert sim.n_groups > 1
    p_or = oracle.OracleParams(ph, RAILS, SITES)
    occ0 = oracle.fill(p_or, FILL)
    sim.load_occupancy(occ0)
    sim.set_protocols(protos)
    st = lockstep(sim, p_or, protos, occ0, 400, 150)
    assert st["resyncs"] == 0 and st["hops"] > 100


def test_batch_strategies_agree():
    """Half-step launches, one persistent group and many small groups, and the
    wave strategy (one group, many groups, 32 sites per lane) give the same
    per-step tallies and final state."""
    import torch
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=FP32, seed=5, ea_ev=0.15)
    protos = _protocols(len(RAILS))
    outs = []
    for mode, limit, tile in (("half_step", 0, 512), ("persistent", 0, 512), ("persistent", 3, 512),
                              ("wave", 0, 0), ("wave", 3, 0), ("wave", 0, 2048)):
        sim = Simulator(ph, RAILS, SITES, tile_sites=tile)
        sim.set_group_limit(limit)
        sim.set_launch_mode(mode)
        sim.fill_random(FILL)
        sim.set_protocols(protos)
        net, dec = sim.run_steps(700, tallies=True)
        outs.append((net.cpu(), dec.cpu(), sim.read_occupancy()))
        sim.close()
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])
        assert np.array_equal(o[2], outs[0][2])


@pytest.mark.parametrize("mode", ["persistent", "wave"])
def test_c3_full_batch_sampled(mode):
    """The 256-device batch (1.4e8 sites) in both persistent strategies: after
    4 steps, sampled devices equal the oracle's run of that device alone (the
    devices before it shrunk to 1 x 2 empty sites so its random stream index is
    unchanged), and every rail keeps its ion count."""
    from paper_2511_09413_amd import Simulator
    wl = c3_batched(n_steps=100_000)
    ph = wl.physics.replace(ea_ev=0.2)   # more hops per step than at 0.3 eV
    sim = Simulator(ph, wl.rails, wl.sites)
    sim.set_launch_mode(mode)
    assert sim.launch_mode == mode and sim.n_groups > 1
    sim.fill_random(wl.filling)
    occ0 = sim.read_occupancy()
    sim.set_protocols(wl.protocols)
    sim.run_steps(4)
    occ = sim.read_occupancy()
    offs = np.concatenate([[0], np.cumsum([r * l for r, l in zip(wl.rails, wl.sites)])])
    D = len(wl.rails)
    for d in (0, 1, 77, 200, D - 1):
        a, b = offs[d], offs[d + 1]
        R, L = wl.rails[d], wl.sites[d]
        assert np.array_equal(occ[a:b].reshape(R, L).sum(axis=1), occ0[a:b].reshape(R, L).sum(axis=1))
        rails = [1] * d + [R]
        sites = [2] * d + [L]
        p_or = oracle.OracleParams(ph, rails, sites)
        part = np.concatenate([np.zeros(2 * d, dtype=np.int8), occ0[a:b]])
        oracle.run(p_or, [constant(0.0)] * d + [wl.protocols[d]], part, 0, 4, want_dec=False)
        assert np.array_equal(occ[a:b], part[2 * d:]), d


def test_autotune_leaves_trajectory_and_caches(tmp_path):
    """kmc_autotune times the candidate configurations but restores the state,
    step counter and tallies: afterwards the run equals that of an untuned
    context step for step; a second context with the same shapes takes the
    configuration from the JSON cache without trials."""
    import torch
    from paper_2511_09413_amd import Simulator
    ph = Physics(precision=FP32, seed=21, ea_ev=0.15)
    protos = _protocols(len(RAILS))
    runs = []
    cache = str(tmp_path / "tune.json")
    for tune in (False, True, True):
        sim = Simulator(ph, RAILS, SITES)
        sim.fill_random(FILL)
        sim.set_protocols(protos)
        sim.run_steps(50)
        info = sim.autotune(trial_steps=64, cache=cache) if tune else None
        assert sim.step == 50
        net, dec = sim.run_steps(300, tallies=True)
        runs.append((net.cpu(), dec.cpu(), sim.read_occupancy(), sim.read_current()[1], info))
        sim.close()
    for r in runs[1:]:
        assert torch.equal(r[0], runs[0][0]) and torch.equal(r[1], runs[0][1])
        assert np.array_equal(r[2], runs[0][2]) and np.array_equal(r[3], runs[0][3])
    assert runs[1][4]["cached"] is False and runs[1][4]["us_per_step"] > 0
    assert runs[2][4]["cached"] is True and runs[2][4]["mode"] == runs[1][4]["mode"]
