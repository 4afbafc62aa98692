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


def _first_divergence(net_g, dec_g, net_o, dec_o):
    """(row, device) of the first step whose net hops or decile counts differ,
    or None when every row agrees."""
    bad = (net_g != net_o) | (dec_g != dec_o).any(axis=2)
    rows = np.nonzero(bad.any(axis=1))[0]
    if len(rows) == 0:
        return None
    r = int(rows[0])
    return r, int(np.nonzero(bad[r])[0][0])


def lockstep(sim, p_or, protocols, occ0: np.ndarray, n_steps: int, chunk: int,
             n_set=None, max_resync: int = 4, electrodes=None):
    """Run the HIP simulator and the oracle side by side from occ0 in chunks of
    `chunk` steps; compare per-step net hops and deciles and the occupancy after
    every chunk.  A mismatch is accepted only where it can come from a
    near-threshold draw (|u - p| < 1e-6): both sides must have logged the same
    draw (device, step, half-step, rail, bond) of the device whose rows diverge
    first, at or before the first diverging step (or anywhere in the chunk
    when only the final occupancy differs).  The GPU is then resynchronised to
    the oracle state.  Returns a summary dict (with the oracle's final state
    under "occ")."""
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
        out = oracle.run(p_or, protocols, occ_o, n0 + done, k, n_set=n_set, log_cap=65536, electrodes=electrodes)
        log_g, n_gpu_log = sim.read_threshold_log(65536)
        new_gpu_log = n_gpu_log - gpu_log_before
        gpu_entries = log_g[gpu_log_before:n_gpu_log] if n_gpu_log <= len(log_g) else None
        gpu_log_before = n_gpu_log
        stats["gpu_log"] += new_gpu_log
        stats["oracle_log"] += out["n_log"]
        same = (np.array_equal(net_g, out["net"]) and np.array_equal(dec_g, out["dec"])
                and np.array_equal(occ_g, occ_o))
        if not same:
            div = _first_divergence(net_g, dec_g, out["net"], out["dec"])
            n_lim = n0 + done + (div[0] if div else k - 1)

            def keys(entries, d_sel):
                return {(int(e["d"]), int(e["n"]), int(e["h"]), int(e["r"]), int(e["s"])) for e in entries
                        if int(e["n"]) <= n_lim and (d_sel is None or int(e["d"]) == d_sel)}

            d_sel = div[1] if div else None
            common = set()
            if gpu_entries is not None and out["n_log"] <= len(out["log"]):
                common = keys(gpu_entries, d_sel) & keys(out["log"], d_sel)
            if not common or stats["resyncs"] >= max_resync:
                raise AssertionError(
                    f"GPU and oracle diverge in steps [{n0 + done}, {n0 + done + k}) "
                    f"(first diverging row/device {div}), no near-threshold draw logged by both sides "
                    f"at or before it (gpu={new_gpu_log}, oracle={out['n_log']})")
            stats["resyncs"] += 1
            sim.load_occupancy(occ_o)
        stats["hops"] += int(np.abs(out["net"]).sum())
        stats["steps"] += k
        done += k
    stats["occ"] = occ_o      # the oracle's state after the run
    return stats
