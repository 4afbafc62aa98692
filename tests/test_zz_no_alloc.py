"""kmc_score_replay_noalloc, the replay whose buffers live in the library's
static device array, against kmc_score_replay (buffers in the workspace) on
the same context, through the C ABI (needs an MI355X).

Both calls take the same decisions with the same kernels; their binary64 sums
differ only in the order of the atomic additions, so they agree within
1e-10 of the terms' magnitude (sum of |term|, from the oracle's replay), and
each stays within the replay tolerance of the oracle's replay.  Two calls in
a row, the second on a smaller lattice (the array then holds the first
call's contents), and a lattice too large for the array is rejected."""
import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from test_gpu_score import _tolerance
from workloads import FP32, FP64, Physics, constant, step_then_relax, triangle

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _both(ph, rails, sites, fill, protos, n, seed):
    import torch
    import paper_2511_09413_amd as kmc
    sim = kmc.Simulator(ph, rails, sites)
    sim.fill_random(fill)
    sim.set_protocols(protos)
    occ0 = sim.snapshot()
    sim.run_steps(n)
    D = len(rails)
    W = torch.from_numpy(np.random.default_rng(seed).normal(size=(n, D))).to(sim.device)
    g_ws = torch.empty((D, 4), dtype=torch.float64, device=sim.device)
    g_na = torch.full((D, 4), 7.0, dtype=torch.float64, device=sim.device)
    kmc.score_replay(sim.ctx, occ0.data_ptr(), 0, n, W.data_ptr(), g_ws.data_ptr())
    kmc.score_replay_noalloc(sim.ctx, occ0.data_ptr(), 0, n, W.data_ptr(), g_na.data_ptr())
    torch.cuda.synchronize()
    p_or = oracle.OracleParams(ph, rails, sites)
    ref = oracle.score_replay(p_or, protos, occ0.cpu().numpy(), 0, W.cpu().numpy(), coul64=True)
    sim.close()
    return g_ws.cpu().numpy(), g_na.cpu().numpy(), ref


def test_noalloc_replay_equals_workspace_replay_twice():
    # first call: two ragged devices, binary32, a few hundred hops
    ph = Physics(precision=FP32, seed=91, ea_ev=0.12)
    g_ws, g_na, ref = _both(ph, [24, 5], [128, 77], [0.3, 0.45], [triangle(1.0, 150e-12), constant(-0.4)], 150, 3)
    assert np.all(ref["hops"] > 10)
    assert np.all(np.abs(g_na - g_ws) <= 1e-10 * ref["mag"]), (g_na, g_ws)
    assert np.all(np.abs(g_na - ref["grad"]) <= _tolerance(ref, ph))
    # second call: a smaller lattice in binary64 (the array holds the first call's data)
    ph = Physics(precision=FP64, seed=92, ea_ev=0.1, rail_range=2, cutoff_sites=20)
    g_ws, g_na, ref = _both(ph, [6], [40], [0.35], [step_then_relax(1.0, 30e-12)], 60, 4)
    assert np.all(ref["hops"] > 10)
    assert np.all(np.abs(g_na - g_ws) <= 1e-10 * ref["mag"]), (g_na, g_ws)
    assert np.all(np.abs(g_na - ref["grad"]) <= _tolerance(ref, ph))


def test_noalloc_rejects_a_lattice_beyond_the_array():
    import torch
    import paper_2511_09413_amd as kmc
    ph = Physics(precision=FP32, seed=1)
    sim = kmc.Simulator(ph, [4096], [4096])        # 16.8 million sites: beyond 64 MiB of buffers
    occ0 = sim.snapshot()
    W = torch.ones((1, 1), dtype=torch.float64, device=sim.device)
    g = torch.zeros((1, 4), dtype=torch.float64, device=sim.device)
    with pytest.raises(kmc.KmcError) as e:
        kmc.score_replay_noalloc(sim.ctx, occ0.data_ptr(), 0, 1, W.data_ptr(), g.data_ptr())
    assert e.value.status == kmc.KMC_EUNSUPPORTED and "static scratch" in str(e.value)
    sim.close()
