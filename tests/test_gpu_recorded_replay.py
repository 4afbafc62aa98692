"""The score replay from a recording of the forward's hops (kmc_record_hops)
against the oracle's replay and against the replay that draws its decisions
again (needs an MI355X).

With a recording the replay reads every half-step's accepted hops from the
list the forward wrote instead of drawing the decisions again: the decisions
are the same, and every candidate's term is computed from the same Coulomb
part with the same arithmetic, so the two replays differ only in the order of
their binary64 sums (bounded by 1e-10 of the terms' magnitude, sum of |term|
from the oracle's replay), and both stay within the replay tolerance of
test_gpu_score.py against the oracle.  A half-step whose list overflowed is
drawn again; a replay that does not start from the recording's first step and
state, covers steps not yet run, or follows a protocol install does not use
the recording at all."""
import ctypes as C

import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from test_gpu_score import _tolerance
from workloads import BF16X2, FP32, FP64, Physics, constant, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _setup(ph, rails, sites, filling, protocols, ea=None, mode="auto"):
    from paper_2511_09413_amd import Simulator
    sim = Simulator(ph, rails, sites, ea=ea, mode=mode)
    sim.fill_random(filling)
    sim.set_protocols(protocols)
    return sim


def _counts(sim, n_steps):
    """The recording's per-half-step counts (a view of the caller's buffer)."""
    import torch
    buf = sim._record
    off = (buf.data_ptr() + 255) // 256 * 256 - buf.data_ptr()
    return buf[off:off + 8 * 2 * n_steps].view(torch.int64)


def _replays(sim, occ0, W, n_steps):
    """(recorded replay, replay drawn again) of the steps [0, n_steps)."""
    import torch
    Wt = torch.from_numpy(W)
    g_rec = sim.score_replay(occ0, 0, Wt).cpu().numpy()
    sim.record_hops(0)
    g_draw = sim.score_replay(occ0, 0, Wt).cpu().numpy()
    return g_rec, g_draw


@pytest.mark.parametrize("precision", [FP64, FP32])
@pytest.mark.parametrize("mode", ["wave", "persistent", "half_step"])
def test_recorded_replay_equals_drawn_replay_and_oracle(precision, mode):
    """Two devices of different shapes, a validation barrier (many hops), a
    bias sweep; the forward in each launch strategy records, in two calls."""
    ph = Physics(precision=precision, seed=77, ea_ev=0.15)
    rails, sites = [24, 5], [128, 77]
    protos = [triangle(1.0, 300e-12), constant(-0.4)]
    sim = _setup(ph, rails, sites, [0.3, 0.45], protos, mode=mode)
    n_steps = 300
    occ0 = sim.snapshot()
    sim.record_hops(n_steps, cap=4096)
    sim.run_steps(100)
    sim.run_steps(n_steps - 100)
    counts = _counts(sim, n_steps).cpu().numpy()
    assert counts.sum() > 100 and counts.max() <= 4096
    W = np.random.default_rng(5).normal(size=(n_steps, 2))
    g_rec, g_draw = _replays(sim, occ0, W, n_steps)
    p_or = oracle.OracleParams(ph, rails, sites)
    ref = oracle.score_replay(p_or, protos, occ0.cpu().numpy(), 0, W, coul64=True)
    tol = _tolerance(ref, ph)
    assert np.all(np.abs(g_rec - ref["grad"]) <= tol), (g_rec, ref["grad"], tol)
    assert np.all(np.abs(g_rec - g_draw) <= 1e-10 * ref["mag"]), (g_rec, g_draw)
    sim.close()


def test_overflowed_lists_are_drawn_again():
    """A low barrier and lists of 8 entries: most half-steps overflow and are
    drawn again, the rest read the recording, in one replay; per-site
    barriers, +-2 rails, cutoff 40."""
    R, L = 16, 96
    ph = Physics(precision=FP64, seed=5, ea_ev=0.08, screening_sites=0.0, cutoff_sites=40, rail_range=2)
    ea = np.random.default_rng(3).normal(0.08, 0.02, size=R * L)
    sim = _setup(ph, [R], [L], [0.3], [constant(0.6)], ea=ea)
    n_steps = 120
    occ0 = sim.snapshot()
    sim.record_hops(n_steps, cap=8)
    sim.run_steps(n_steps)
    counts = _counts(sim, n_steps).cpu().numpy()
    assert (counts > 8).sum() > 10 and (counts <= 8).sum() > 10
    W = np.random.default_rng(9).normal(size=(n_steps, 1))
    g_rec, g_draw = _replays(sim, occ0, W, n_steps)
    ref = oracle.score_replay(oracle.OracleParams(ph, [R], [L], ea), [constant(0.6)], occ0.cpu().numpy(), 0, W,
                              coul64=True)
    tol = _tolerance(ref, ph)
    print("rec", g_rec, "draw", g_draw, "oracle", ref["grad"], "tol", tol, "mag", ref["mag"])
    assert np.all(np.abs(g_draw - ref["grad"]) <= tol), "drawn"
    assert np.all(np.abs(g_rec - g_draw) <= 1e-10 * ref["mag"]), "recorded"
    assert np.all(np.abs(g_rec - ref["grad"]) <= tol)
    sim.close()


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_many_hops_per_half_step(precision):
    """A low barrier on 64 x 256 with +-2 rails and cutoff 40: hundreds of
    hops per half-step, many of them on neighbouring rails and sites, so that
    the Coulomb-part update rewrites overlapping windows and the in-place
    flips share state words; against the replay drawn again and the oracle."""
    ph = Physics(precision=precision, seed=21, ea_ev=0.06, cutoff_sites=40, rail_range=2)
    rails, sites = [64], [256]
    protos = [constant(0.5)]
    sim = _setup(ph, rails, sites, [0.3], protos)
    n_steps = 40
    occ0 = sim.snapshot()
    sim.record_hops(n_steps, cap=4096)
    sim.run_steps(n_steps)
    counts = _counts(sim, n_steps).cpu().numpy()
    assert counts.max() <= 4096 and counts.min() > 100, counts
    W = np.random.default_rng(2).normal(size=(n_steps, 1))
    g_rec, g_draw = _replays(sim, occ0, W, n_steps)
    ref = oracle.score_replay(oracle.OracleParams(ph, rails, sites), protos, occ0.cpu().numpy(), 0, W,
                              coul64=True)
    tol = _tolerance(ref, ph)
    assert np.all(np.abs(g_rec - g_draw) <= 1e-10 * ref["mag"]), (g_rec, g_draw)
    assert np.all(np.abs(g_rec - ref["grad"]) <= tol), (g_rec, ref["grad"], tol)
    sim.close()


def test_small_ragged_devices():
    """Three devices of 10, 17 and 33 sites (pitches 16, 32 and 48: rails of
    two to six bytes in the replay's one-bit state, words shared by rails and
    devices) and 3, 2 and 5 rails, a low barrier; recorded replay against the
    replay drawn again and the oracle in both precisions."""
    for precision in (FP64, FP32):
        ph = Physics(precision=precision, seed=31, ea_ev=0.08, cutoff_sites=4, screening_sites=2.0)
        rails, sites = [3, 2, 5], [10, 17, 33]
        protos = [constant(0.6), triangle(1.0, 100e-12), constant(-0.3)]
        sim = _setup(ph, rails, sites, [0.3, 0.4, 0.5], protos)
        n_steps = 200
        occ0 = sim.snapshot()
        sim.record_hops(n_steps, cap=256)
        sim.run_steps(n_steps)
        counts = _counts(sim, n_steps).cpu().numpy()
        assert counts.sum() > 50 and counts.max() <= 256
        W = np.random.default_rng(4).normal(size=(n_steps, 3))
        g_rec, g_draw = _replays(sim, occ0, W, n_steps)
        ref = oracle.score_replay(oracle.OracleParams(ph, rails, sites), protos, occ0.cpu().numpy(), 0, W,
                                  coul64=True)
        tol = _tolerance(ref, ph)
        assert np.all(np.abs(g_rec - g_draw) <= 1e-10 * ref["mag"]), (precision, g_rec, g_draw)
        assert np.all(np.abs(g_rec - ref["grad"]) <= tol), (precision, g_rec, ref["grad"], tol)
        sim.close()


def test_edited_recording_changes_the_result():
    """The replay does take its decisions from the recording: dropping the
    last hop of one list moves the gradient far beyond the summation-order
    bound, and restoring the count restores the result."""
    import torch
    ph = Physics(precision=FP32, seed=12, ea_ev=0.15)
    sim = _setup(ph, [32], [128], [0.3], [constant(0.8)])
    n_steps = 60
    occ0 = sim.snapshot()
    sim.record_hops(n_steps, cap=1024)
    sim.run_steps(n_steps)
    counts = _counts(sim, n_steps)
    c = counts.cpu().numpy()
    hs = int(np.argmax(c > 0))
    assert c[hs] > 0
    W = torch.ones((n_steps, 1), dtype=torch.float64)
    g_rec = sim.score_replay(occ0, 0, W).cpu().numpy()
    counts[hs] -= 1
    g_edit = sim.score_replay(occ0, 0, W).cpu().numpy()
    counts[hs] += 1
    g_again = sim.score_replay(occ0, 0, W).cpu().numpy()
    mag = np.abs(g_rec).max()
    assert np.abs(g_edit - g_rec).max() > 1e-3 * mag
    assert np.abs(g_again - g_rec).max() <= 1e-9 * mag
    sim.close()


def test_recording_is_used_only_where_it_holds():
    """Replays that the recording does not describe (another start state, a
    later first step, steps not yet run, a protocol installed since) equal
    the replay drawn again, not the recorded decisions."""
    import torch
    ph = Physics(precision=FP64, seed=3, ea_ev=0.15)
    proto = [triangle(1.0, 200e-12)]
    sim = _setup(ph, [16], [100], [0.35], proto)
    n_steps = 80
    occ0 = sim.snapshot()
    sim.record_hops(2 * n_steps, cap=2048)
    sim.run_steps(n_steps)
    assert _counts(sim, n_steps).sum().item() > 20
    W = torch.from_numpy(np.random.default_rng(1).normal(size=(n_steps, 1)))
    other = occ0.clone()
    other[:200] = 1 - other[:200]
    # the reference values come from a twin context that never recorded
    twin = _setup(ph, [16], [100], [0.35], proto)
    twin.run_steps(n_steps)
    cases = {
        "other_state": (other, 0, W),
        "later_start": (occ0, 10, W[:40]),
        "not_yet_run": (occ0, 0, torch.cat([W, W[:5]])),
    }
    for name, (o, s0, w) in cases.items():
        g = sim.score_replay(o, s0, w).cpu().numpy()
        t = twin.score_replay(o, s0, w).cpu().numpy()
        assert np.all(np.abs(g - t) <= 1e-9 * np.abs(t).max() + 1e-12), name
    # a protocol install ends the recording
    sim.set_protocols(proto)
    twin.set_protocols(proto)
    g = sim.score_replay(occ0, 0, W).cpu().numpy()
    t = twin.score_replay(occ0, 0, W).cpu().numpy()
    assert np.all(np.abs(g - t) <= 1e-9 * np.abs(t).max())
    sim.close()
    twin.close()


def test_record_arguments():
    from paper_2511_09413_amd import KMC_EINVAL, KMC_EUNSUPPORTED, KmcError, Simulator, lib
    ph = Physics(precision=FP32, seed=1, ea_ev=0.15)
    sim = _setup(ph, [8], [64], [0.3], [constant(0.5)])
    L = lib()
    ctx = C.c_void_p(sim.ctx)
    nbytes = C.c_size_t()
    assert L.kmc_record_bytes(ctx, 10, 0, C.byref(nbytes)) == KMC_EINVAL
    assert L.kmc_record_bytes(ctx, -1, 4, C.byref(nbytes)) == KMC_EINVAL
    assert L.kmc_record_bytes(ctx, 10, 4, C.byref(nbytes)) == 0 and nbytes.value > 0
    buf = sim.torch.empty(nbytes.value + 512, dtype=sim.torch.uint8, device=sim.device)
    base = (buf.data_ptr() + 255) // 256 * 256
    assert L.kmc_record_hops(ctx, C.c_void_p(base + 16), nbytes.value, 10, 4) == KMC_EINVAL     # misaligned
    assert L.kmc_record_hops(ctx, C.c_void_p(base), nbytes.value - 1, 10, 4) == KMC_EINVAL      # too small
    assert L.kmc_record_hops(ctx, C.c_void_p(base), nbytes.value, 10, 4) == 0
    assert L.kmc_record_hops(ctx, None, 0, 0, 0) == 0                                           # ends it
    sim.close()
    dense = Simulator(Physics(precision=BF16X2, screening_sites=0.0, cutoff_sites=63, rail_range=4), [8], [64])
    with pytest.raises(KmcError) as err:
        dense.record_hops(10)
    assert err.value.status == KMC_EUNSUPPORTED
    dense.close()
