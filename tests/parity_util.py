"""Helpers for GPU-vs-oracle parity tests (no test functions here)."""
from __future__ import annotations

import numpy as np

import oracle


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def lockstep(sim, p_or, protocols, occ0: np.ndarray, n_steps: int, chunk: int,
             n_set=None, max_resync: int = 4):
    """Run the HIP simulator and the oracle side by side from occ0 in chunks of
    `chunk` steps; compare per-step net hops and deciles and the occupancy after
    every chunk.  A mismatch is accepted only where both sides logged a
    near-threshold draw (|u - p| < 1e-6) in that chunk; the GPU is then
    resynchronised to the oracle state.  Returns a summary dict."""
    occ_o = occ0.copy().reshape(-1)
    D = len(p_or.rails)
    n0 = sim.step
    stats = {"steps": 0, "hops": 0, "resyncs": 0, "gpu_log": 0, "oracle_log": 0}
    gpu_log_before = sim.read_threshold_log(0)[1]
    done = 0
    while done < n_steps:
        k = min(chunk, n_steps - done)
        net_g, dec_g = sim.run_steps(k, tallies=True)
        net_g = net_g.cpu().numpy()
        dec_g = dec_g.cpu().numpy()
        occ_g = sim.read_occupancy()
        out = oracle.run(p_or, protocols, occ_o, n0 + done, k, n_set=n_set)
        _, n_gpu_log = sim.read_threshold_log(0)
        new_gpu_log = n_gpu_log - gpu_log_before
        gpu_log_before = n_gpu_log
        stats["gpu_log"] += new_gpu_log
        stats["oracle_log"] += out["n_log"]
        same = (np.array_equal(net_g, out["net"]) and np.array_equal(dec_g, out["dec"])
                and np.array_equal(occ_g, occ_o))
        if not same:
            if new_gpu_log == 0 or out["n_log"] == 0 or stats["resyncs"] >= max_resync:
                bad = np.nonzero((net_g != out["net"]).any(axis=1))[0]
                raise AssertionError(
                    f"GPU and oracle diverge in steps [{n0 + done}, {n0 + done + k}) "
                    f"(first net mismatch at row {bad[:1]}), logged draws gpu={new_gpu_log} "
                    f"oracle={out['n_log']}")
            stats["resyncs"] += 1
            sim.load_occupancy(occ_o)
        stats["hops"] += int(np.abs(out["net"]).sum())
        stats["steps"] += k
        done += k
    return stats
