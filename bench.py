"""Benchmark of the rail-KMC hop step on one MI355X.

Workload (default): a single large device, 4096 rails x 1024 sites, 30% filling,
per-site barriers Ea ~ N(0.3, 0.02) eV (binary32), a +-2 V triangular sweep over
1e5 steps of 1 ps, screened Coulomb (lambda = 4 sites, cutoff 16, +-1 rail),
binary32 rates.  A "step" is one full hop step (both bond parities) of the whole
lattice.  Inputs are resident in HBM before the timed region.

Prints one JSON line: site-updates/s (value), effective HBM GB/s of the
algorithmic traffic, the roofline of the dominant kernel and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ = 256, 2.4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--warmup", type=int, default=2_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="auto", choices=["auto", "half_step", "persistent"])
    ap.add_argument("--tile-sites", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(wl, budget_s):
    """The oracle as it stands (single thread) on whole steps of the same
    device, stopping once budget_s of CPU time is spent."""
    import numpy as np
    import oracle
    p = oracle.params_for(wl)
    occ = oracle.fill(p, wl.filling)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        oracle.run(p, wl.protocols, occ, steps, 1, want_dec=False)
        steps += 1
    el = time.perf_counter() - t0
    return {"value": wl.n_sites * steps / el, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} full steps of the 4096x1024 device (single-threaded C oracle, {el:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is a "
              f"design in DESIGN.md, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import c2_large_device

    wl = c2_large_device(n_steps=100_000)
    dev = torch.device("cuda:0")
    sim = kmc.Simulator(wl.physics, wl.rails, wl.sites, ea=wl.ea_site, device="cuda:0", mode=args.mode,
                        tile_sites=args.tile_sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    sim.run_steps(args.warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    sim.run_steps(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    sec = ms / 1e3
    sites = wl.n_sites
    value = sites * args.steps / sec
    # algorithmic HBM traffic per site-update: occupancy 1 B per half-step pass
    # and the binary32 barrier 4 B per half-step pass
    bytes_per_site_update = 10.0
    eff_gbs = bytes_per_site_update * value / 1e9
    launches = 2 * args.steps
    per_launch_s = sec / launches
    cur, tot, t_sim = sim.read_current()
    out = {
        "metric": "site-updates/s (4096x1024 rails)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "rails": 4096, "sites": 1024, "filling": 0.3,
                   "protocol": "triangle +-2 V over 1e5 steps", "ea": "N(0.3,0.02) eV per site",
                   "coulomb": "lambda=4, cutoff=16, +-1 rail", "parallelism": "single GPU"},
        "effective_hbm_gbs": eff_gbs,
        "wall_s": wall,
        "net_hops_total": int(tot[0]),
        "launch_mode": sim.launch_mode,
        "roofline": {"bound": "hbm", "achieved": bytes_per_site_update / 2 * sites / per_launch_s / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_per_site_update / 2 * sites / per_launch_s / 1e9 / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
