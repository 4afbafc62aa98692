"""Benchmark of the rail-KMC hop step on one MI355X.

Workload: a single large device, 4096 rails x 1024 sites, 30% filling,
per-site barriers Ea ~ N(0.3, 0.02) eV (binary32), a +-2 V triangular sweep over
1e5 steps of 1 ps, screened Coulomb (lambda = 4 sites, cutoff 16, +-1 rail),
binary32 rates.  A step is one full hop step (both bond parities) of the whole
lattice.  Inputs are resident in device memory before the timed region.

Prints one JSON line: site-updates/s (value), the roofline of the dominant
kernel (the hop kernel: VALU-bound by the Philox4x32-10 stream), the HBM rate
the kernel's counters measured, the method's algorithmic bytes as an
equivalent rate, and the CPU oracle (all host cores, and one core) timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = one wave64 VALU instruction
# per SIMD every 4 cycles = 3.93e13 32-bit lane-operations per second.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# one Philox4x32-10 block = 10 rounds x (2 v_mad_u64_u32 + 2 v_bitop3_b32)
OPS_PER_PHILOX_BLOCK = 40
# algorithmic bytes per site-update of the method (occupancy 1 B and the
# binary32 barrier 4 B per half-step pass)
BYTES_PER_SITE_UPDATE = 10.0
def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--warmup", type=int, default=2_048)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="auto", choices=["auto", "half_step", "persistent", "wave"])
    ap.add_argument("--tile-sites", type=int, default=0)
    ap.add_argument("--no-record", action="store_true",
                    help="gradient workload: replay without the forward's recording")
    ap.add_argument("--workload", default="large-device",
                    choices=["large-device", "batch", "gradient", "dense", "dense-fixed", "small-fp64", "zone"],
                    help="large-device: 4096x1024 (default); batch: 256 heterogeneous devices; "
                         "gradient: forward + score replay of 512 replicas x 256 x 512; "
                         "dense: 64 replicas x 1024 x 512 with the MFMA long-range potential; "
                         "dense-fixed: the same lattice with the potential kept hop by hop in fixed point; "
                         "small-fp64: 64 x 128 in binary64 (latency); "
                         "zone: the paper's own zone model at Table S2's largest size (128,000 rails x 200)")
    return ap.parse_args()


# counter summaries of the persistent kernels and the sources they were taken from
TRAFFIC = {
    "hop_persistent": ("hop_persistent_c2_traffic.md", "kmc_persistent.hip"),
    "hop_wave": ("hop_wave_c2_traffic.md", "kmc_wave.hip"),
    "replay_stream": ("replay_stream_c5_traffic.md", "kmc_replay.hip"),
    "replay_logged": ("replay_logged_c5_traffic.md", "kmc_replay.hip"),
}


def kernel_sha1(kernel: str) -> str:
    h = hashlib.sha1()
    for f in (TRAFFIC[kernel][1], "kmc_device.h", "kmc_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2511_09413_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of a persistent hop kernel from its counter profile
    summary (the json block), or None when there is none or when the kernel's
    sources changed since the counters were taken."""
    if kernel not in TRAFFIC:
        return None
    path = os.path.join(ROOT, "profiles", TRAFFIC[kernel][0])
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    t = json.loads(m.group(1)) if m else None
    return t if t is not None and t.get("kernel_sha1") == kernel_sha1(kernel) else None


def philox_blocks_per_step(rails, sites) -> int:
    """One 32-bit Philox word per bond and half-step, four words per block."""
    total = 0
    for R, L in zip(rails, sites):
        for h in (0, 1):
            bonds = max(0, (L - h) // 2)
            total += R * ((bonds + 3) // 4)
    return total


def host_cores() -> int:
    """Threads for the all-core oracle leg: OMP_NUM_THREADS when set (the host's
    share of a shared machine), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def host_cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(wl, budget_s, threads):
    import oracle
    oracle.set_threads(threads)
    try:
        p = oracle.params_for(wl)
        occ = oracle.fill(p, wl.filling)
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            oracle.run(p, wl.protocols, occ, steps, 1, want_dec=False)
            steps += 1
        el = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    return wl.n_sites * steps / el, steps, el


def cpu_baseline(wl, budget_s):
    """The oracle as it stands on whole steps of the same device, stopping once
    budget_s of wall time is spent: on all of the host's cores (OpenMP over
    rails inside each half-step, the reported baseline) and on one core."""
    cores = host_cores()
    v_all, s_all, e_all = _oracle_rate(wl, budget_s, cores)
    v_one, s_one, e_one = _oracle_rate(wl, budget_s, 1)
    return {"value": v_all, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{s_all} whole steps of the 4096x1024 device, C oracle on {cores} threads, {e_all:.1f} s",
            "single_core": {"value": v_one, "cores": 1,
                            "sample": f"{s_one} whole steps, single-threaded, {e_one:.1f} s"},
            "host": {"nproc": os.cpu_count(), "cpu_model": host_cpu_model()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for {args.gpus}): the multi-GPU sharding is a design "
              f"note only, nothing here uses a second GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "gradient":
        return bench_gradient(args)
    if args.workload == "dense":
        return bench_dense(args)
    if args.workload == "small-fp64":
        return bench_small(args)
    if args.workload == "zone":
        return bench_zone(args)
    if args.workload == "dense-fixed":
        return bench_dense_fixed(args)
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
    t_wall = time.perf_counter()
    e0.record(stream)
    sim.run_steps(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    sec = e0.elapsed_time(e1) / 1e3
    value = wl.n_sites * args.steps / sec
    cur, tot, t_sim = sim.read_current()   # also checks the kernel status
    mode = sim.launch_mode

    # dominant kernel: hop_wave or hop_persistent (one launch per 1024 steps)
    # or hop_half_step (one launch per half-step)
    if mode in ("persistent", "wave"):
        launches = (args.steps + 1023) // 1024
        kernel = "hop_wave" if mode == "wave" else "hop_persistent"
    else:
        launches = 2 * args.steps
        kernel = "hop_half_step"
    per_launch_s = sec / launches
    blocks_per_launch = philox_blocks_per_step(wl.rails, wl.sites) * args.steps / launches
    achieved = OPS_PER_PHILOX_BLOCK * blocks_per_launch / per_launch_s / 1e12
    t = measured_traffic(kernel)
    traffic = t["hbm_bytes_per_launch"] if t is not None else None
    out = {
        "metric": "site-updates/s (4096x1024 rails)",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "rails": 4096, "sites": 1024, "filling": 0.3,
                   "protocol": "triangle +-2 V over 1e5 steps", "barriers": "N(0.3,0.02) eV per site",
                   "coulomb": "lambda=4, cutoff=16, +-1 rail", "launch_mode": mode},
        "roofline": {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic,
                     "avg_launch_us": per_launch_s * 1e6, "launches": launches},
        # HBM traffic the kernel actually moves (counter record of the same
        # kernel sources, scaled by the copy-kernel calibration), per second
        # of this run's launches; the lattice stays in registers for a launch
        "hbm_measured_gbs": traffic / per_launch_s / 1e9 if traffic is not None else None,
        # the method's algorithmic bytes (occupancy and barrier read per
        # half-step) per second: an equivalent rate, not a fraction of a roof
        "algorithmic_bytes_equivalent_gbs": BYTES_PER_SITE_UPDATE * value / 1e9,
        "wall_s": wall,
        "net_hops_total": int(tot[0]),
        "mean_current_A": float(cur[0]),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    sim.close()


def _timed(fn, stream):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def bench_batch(args):
    """256 heterogeneous devices (rails U{32..1024}, sites U{64..2048}, filling
    U[0.05,0.4], step / triangle / STDP protocols), all advanced by one call."""
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import c3_batched
    steps = args.steps if args.steps != 100_000 else 8192
    wl = c3_batched(n_steps=100_000)
    sim = kmc.Simulator(wl.physics, wl.rails, wl.sites, device="cuda:0", mode=args.mode,
                        tile_sites=args.tile_sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    # the autotuner picks strategy and tile size (trials restore the state)
    # unless a mode or tile size was asked for
    tuned = sim.autotune(trial_steps=256) if args.mode == "auto" and args.tile_sites == 0 else None
    sim.run_steps(args.warmup)
    stream = torch.cuda.current_stream()
    sec = _timed(lambda: sim.run_steps(steps), stream)
    sim.read_current()
    mode = sim.launch_mode
    value = wl.n_sites * steps / sec
    chunks = (steps + 1023) // 1024
    launches = chunks * sim.n_groups if mode in ("persistent", "wave") else 2 * steps
    per_launch_s = sec / launches
    achieved = OPS_PER_PHILOX_BLOCK * philox_blocks_per_step(wl.rails, wl.sites) * steps / sec / 1e12
    out = {
        "metric": "site-updates/s (256-device batch)", "value": value, "unit": "site-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": sec * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": wl.name, "devices": len(wl.rails), "sites_total": wl.n_sites,
                   "launch_mode": mode, "groups": sim.n_groups,
                   "autotuned": None if tuned is None else {k: tuned[k] for k in ("tile_sites", "mode", "us_per_step")}},
        # occupancy read per half-step pass (no barrier field here): an
        # equivalent rate of the method's algorithmic bytes
        "algorithmic_bytes_equivalent_gbs": BYTES_PER_SITE_UPDATE / 5 * 2 * value / 1e9,
        "roofline": {"bound": "alu",
                     "kernel": {"persistent": "hop_persistent", "wave": "hop_wave"}.get(mode, "hop_half_step"),
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "avg_launch_us": per_launch_s * 1e6, "launches": launches},
    }
    sim.close()
    # the same devices run one by one, each alone in its own context (every
    # 8th device), for the batched-versus-plain comparison
    sample = list(range(0, len(wl.rails), 8))
    k_one, t_one, sites_one = 1024, 0.0, 0
    for d in sample:
        one = kmc.Simulator(wl.physics, [wl.rails[d]], [wl.sites[d]], device="cuda:0")
        one.fill_random([wl.filling[d]])
        one.set_protocols([wl.protocols[d]])
        one.run_steps(128)
        t_one += _timed(lambda: one.run_steps(k_one), stream)
        one.read_current()
        sites_one += wl.rails[d] * wl.sites[d]
        one.close()
    out["one_by_one_site_updates_per_s"] = sites_one * k_one / t_one
    out["batched_over_one_by_one"] = value / out["one_by_one_site_updates_per_s"]
    out["one_by_one_sample"] = (f"{len(sample)} devices (every 8th, {sites_one} sites), each alone for {k_one} "
                                f"steps after 128 warm-up steps, automatic launch mode")
    print(json.dumps(out), flush=True)


def bench_small(args):
    """64 x 128 in binary64, 20% filling, 0.5 V: a lattice far too small to
    fill the GPU, so the step time is the latency of the step."""
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import c1_plain_fp64
    steps = args.steps if args.steps != 100_000 else 10_000
    wl = c1_plain_fp64(n_steps=10_000)
    sim = kmc.Simulator(wl.physics, wl.rails, wl.sites, device="cuda:0", mode=args.mode,
                        tile_sites=args.tile_sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    sim.run_steps(min(args.warmup, 1024))
    stream = torch.cuda.current_stream()
    sec = _timed(lambda: sim.run_steps(steps), stream)
    sim.read_current()
    value = wl.n_sites * steps / sec
    out = {
        "metric": "us per step (64x128, binary64)", "value": sec * 1e6 / steps, "unit": "us/step", "n_gpus": 1,
        "steps": steps, "warmup": min(args.warmup, 1024), "ms_per_step": sec * 1e3 / steps,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "fp64", "data": "synthetic",
        "config": {"workload": wl.name, "rails": 64, "sites": 128, "launch_mode": sim.launch_mode,
                   "groups": sim.n_groups},
        "site_updates_per_s": value,
    }
    print(json.dumps(out), flush=True)
    sim.close()


RECORD_CAP = 4096  # accepted hops per half-step kept by the gradient bench's recording
LIMIT_NOTE = {
    "replay_stream": "the kernel issues about 300 VALU instructions per 8-site block and half-step and its VALU "
                     "is about 80 % busy (SQ counters): it is bound by its instruction count, below the HBM roof",
    "replay_logged": "no Philox, prefilter or window sums: per candidate one exponential and the binary64 "
                     "ratio (y - p)/(1 - p): VALU-bound (SQ counters: about 2000 VALU per wavefront at 8 "
                     "wavefronts per SIMD fill the VALU for their lifetime; the HBM at about 55 % of its peak); "
                     "the update of the Coulomb parts after the half-step's hops is a launch of its own",
}


def bench_gradient(args):
    """Forward steps and the score-function replay of 512 replicas of a
    256 x 512 device (1 V for the first half of the run, then 0 V), FP32 step,
    binary64 accumulators.  The forward records its accepted hops
    (kmc_record_hops) and the replay takes its decisions from the recording;
    --no-record times the replay that draws them again."""
    import numpy as np
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import c5_gradient
    steps = args.steps if args.steps != 100_000 else 20_000
    wl = c5_gradient(n_steps=20_000)
    sim = kmc.Simulator(wl.physics, wl.rails, wl.sites, device="cuda:0", mode=args.mode,
                        tile_sites=args.tile_sites)
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    occ0 = sim.snapshot()
    stream = torch.cuda.current_stream()
    D = len(wl.rails)
    W = torch.ones((steps, D), dtype=torch.float64, device="cuda:0")
    sim.score_replay(occ0, 0, W[:min(steps, 64)])      # warm-up of the replay kernels
    record = not args.no_record
    if record:
        sim.record_hops(steps, RECORD_CAP)
    t_fwd = _timed(lambda: sim.run_steps(steps), stream)
    grads = []
    t_rep = _timed(lambda: grads.append(sim.score_replay(occ0, 0, W)), stream)
    g = grads[0].cpu().numpy()
    value = wl.n_sites * steps / (t_fwd + t_rep)
    # The replay kernel's own memory stream, per half-step and site: the
    # padded occupancy read (1 B; one bit in the recorded replay, which keeps
    # the state as bits and flips the hops' sites in place), written again
    # (1 B) only by the kernel that draws the decisions, and the binary32
    # Coulomb part of every bond of the half-step's parity (4 B per two
    # sites); the recomputation after hops touches a few kB.  Against the HBM
    # peak.
    kernel = "replay_logged" if record else "replay_stream"
    per_site = (0.125 + 2) if record else (1 + 1 + 2)
    replay_bytes = 2 * per_site * wl.n_sites * steps
    achieved = replay_bytes / t_rep / 1e9
    t_meas = measured_traffic(kernel)
    out = {
        "metric": "gradient site-updates/s (forward + score replay)", "value": value, "unit": "site-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": (t_fwd + t_rep) * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+f64acc",
        "data": "synthetic",
        "config": {"workload": wl.name, "replicas": D, "theta": ["Ea", "nu0", "kappa", "alpha"],
                   "forward_launch_mode": sim.launch_mode, "recorded_decisions": record},
        "forward_site_updates_per_s": wl.n_sites * steps / t_fwd,
        "replay_site_updates_per_s": wl.n_sites * steps / t_rep,
        "replay_over_forward_time": t_rep / t_fwd,
        "roofline": {"bound": "hbm", "kernel": kernel + "<float,h>", "achieved": achieved,
                     "bytes": ("4.25 B per site and step: occupancy bits in, one binary32 Coulomb part per bond"
                               if record
                               else "8 B per site and step: occupancy in and out, one binary32 Coulomb part "
                                    "per bond"),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": t_meas["hbm_bytes_per_launch"] if t_meas is not None else None,
                     "avg_launch_us": t_rep / (2 * steps) * 1e6, "launches": 2 * steps,
                     "launch_note": "per half-step: the replay kernel and the update of the Coulomb parts; "
                                    "traffic is the replay kernel's own, per half-step",
                     "limit_note": LIMIT_NOTE[kernel]},
        "grad_mean_over_replicas": [float(x) for x in g.mean(axis=0)],
    }
    print(json.dumps(out), flush=True)
    sim.close()


BF16_DENSE_PEAK_TFLOPS = 2500.0


def bench_dense(args):
    """64 replicas of 1024 x 512, unscreened 1/r over the whole rail and +-4
    rails, 1 V, potential of every site on MFMA (BF16 hi/lo, FP32 accumulate),
    binary32 decisions.  The dominant kernel is the potential; it is also timed
    alone (the same kernel through kmc_dense_potential)."""
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import c4_dense
    steps = args.steps if args.steps != 100_000 else 1000
    wl = c4_dense(n_steps=1000)
    sim = kmc.Simulator(wl.physics, wl.rails, wl.sites, device="cuda:0")
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    sim.run_steps(min(args.warmup, 20))
    stream = torch.cuda.current_stream()
    sec = _timed(lambda: sim.run_steps(steps), stream)
    sim.read_current()
    value = wl.n_sites * steps / sec
    n_pot = 200
    t_phi = _timed(lambda: [sim.dense_potential() for _ in range(n_pot)], stream) / n_pot
    M, L, m = sum(wl.rails), wl.sites[0], wl.physics.rail_range
    flops = 2 * 2 * M * L * (m + 1) * L          # hi and lo products, rails at +-dist folded
    achieved = flops / t_phi / 1e12
    out = {
        "metric": "site-updates/s (dense long-range potential)", "value": value, "unit": "site-updates/s",
        "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 20), "ms_per_step": sec * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x2+fp32",
        "data": "synthetic",
        "config": {"workload": wl.name, "replicas": len(wl.rails), "rails": wl.rails[0], "sites": L,
                   "rail_range": m, "kernel": "kappa/d, whole rail"},
        "potential_us": t_phi * 1e6,
        "potential_share_of_step": 2 * t_phi / (sec / steps),
        "roofline": {"bound": "mfma", "kernel": "dense_phi", "achieved": achieved, "peak": BF16_DENSE_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / BF16_DENSE_PEAK_TFLOPS, "traffic": None,
                     "avg_launch_us": t_phi * 1e6, "flop_per_launch": flops},
    }
    sim.close()
    # the same lattice and physics as the plain binary32 step (per-candidate
    # window sums behind the exact prefilter, no potential), a few steps
    from workloads import FP32
    plain = kmc.Simulator(wl.physics.replace(precision=FP32), wl.rails, wl.sites, device="cuda:0")
    plain.fill_random(wl.filling)
    plain.set_protocols(wl.protocols)
    plain.run_steps(2)
    k_plain = 20
    t_plain = _timed(lambda: plain.run_steps(k_plain), stream)
    plain.read_current()
    out["plain_fp32_site_updates_per_s"] = wl.n_sites * k_plain / t_plain
    out["dense_over_plain_fp32"] = value / out["plain_fp32_site_updates_per_s"]
    out["plain_fp32_launch_mode"] = plain.launch_mode
    plain.close()
    print(json.dumps(out), flush=True)


def bench_dense_fixed(args):
    """The dense workload (64 replicas of 1024 x 512, unscreened 1/r over the
    whole rail and +-4 rails, 1 V) with the potential kept hop by hop in fixed
    point (KMC_PHI_FIXED, binary64 decisions): per half-step one decision
    kernel (occupancy, Philox, the exact prefilter, the potential of the rare
    survivors) and one update kernel (the half-step's hops).  Compared with the
    same lattice in the MFMA form (KMC_BF16X2) and in the plain binary32 step
    (window sums behind the prefilter)."""
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import BF16X2, FP32, PHI_FIXED, c4_dense
    steps = args.steps if args.steps != 100_000 else 2000
    wl = c4_dense(n_steps=steps)
    ph = wl.physics.replace(precision=PHI_FIXED)
    sim = kmc.Simulator(ph, wl.rails, wl.sites, device="cuda:0")
    sim.fill_random(wl.filling)
    sim.set_protocols(wl.protocols)
    sim.run_steps(min(args.warmup, 50))
    stream = torch.cuda.current_stream()
    sec = _timed(lambda: sim.run_steps(steps), stream)
    sim.read_current()
    value = wl.n_sites * steps / sec
    half = sec / steps / 2
    # per half-step: the occupancy read once (1 B per site), one Philox block
    # per 8 sites (40 VALU lane-operations)
    hbm = wl.n_sites * 1.0 / half / 1e9
    alu = OPS_PER_PHILOX_BLOCK * (wl.n_sites / 8) / half / 1e12
    fr_h, fr_a = hbm / HBM_PEAK_GBS, alu / VALU_PEAK_TOPS
    roof = ({"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fr_h}
            if fr_h >= fr_a else
            {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": fr_a})
    roof.update({"kernel": "phifix_decide + phifix_update (one half-step)", "traffic": None,
                 "avg_launch_us": half * 1e6, "launches": 2 * steps, "other": {"hbm_frac": fr_h, "alu_frac": fr_a}})
    out = {
        "metric": "site-updates/s (dense long-range potential, fixed point)", "value": value,
        "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 50),
        "ms_per_step": sec * 1e3 / steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i64 potential, f64", "data": "synthetic",
        "config": {"workload": wl.name, "replicas": len(wl.rails), "rails": wl.rails[0], "sites": wl.sites[0],
                   "rail_range": ph.rail_range, "kernel": "kappa/d, whole rail", "precision": "phi_fixed"},
        "roofline": roof,
    }
    sim.close()
    for name, prec in (("dense_bf16x2", BF16X2), ("plain_fp32", FP32)):
        other = kmc.Simulator(wl.physics.replace(precision=prec), wl.rails, wl.sites, device="cuda:0")
        other.fill_random(wl.filling)
        other.set_protocols(wl.protocols)
        other.run_steps(2)
        k = 20
        t = _timed(lambda: other.run_steps(k), stream)
        other.read_current()
        out[name + "_site_updates_per_s"] = wl.n_sites * k / t
        out["fixed_over_" + name] = value / out[name + "_site_updates_per_s"]
        other.close()
    print(json.dumps(out), flush=True)


# the paper's GPU figure for its zone model at 128,000 rails (SI S4, Table S2):
# 10,774,101 rail-steps/s on an unnamed GPU
PAPER_ZONE_RAIL_STEPS_128K = 10_774_101.0


def bench_zone(args):
    """The paper's own zone model (SI S2.1) at Table S2's largest size:
    128,000 rails x 200 columns, 60 ions per rail (30 %), Table S1's constants
    (300 K, effective voltage difference factor 5e-5 V), a 5 V polarisation
    then relaxation; one kernel launch per step.  Value: rail-steps/s, the
    metric of Table S2."""
    import torch
    import paper_2511_09413_amd as kmc
    from workloads import zone_relaxation
    steps = args.steps if args.steps != 100_000 else 20_000
    wl = zone_relaxation(rails=128_000, n_steps=steps)
    sim = kmc.ZoneSimulator(wl.rails, wl.sites, wl.ions, zones=wl.zones, p0=wl.p0, kT_ev=wl.kT_ev,
                            v_factor=wl.v_factor, dt_s=wl.dt_s, seed=wl.seed, occ=wl.occupancy())
    sim.set_bias_protocol(*wl.protocol)
    sim.run_steps(min(args.warmup, 200))
    stream = torch.cuda.current_stream()
    sec = _timed(lambda: sim.run_steps(steps), stream)
    value = wl.rails * steps / sec
    ions = wl.rails * wl.ions
    # per step: the positions read and written (2 B each), one Philox block
    # per two ions (40 VALU lane-operations)
    hbm = 4.0 * ions / (sec / steps) / 1e9
    alu = OPS_PER_PHILOX_BLOCK * (ions / 2) / (sec / steps) / 1e12
    fr_h, fr_a = hbm / HBM_PEAK_GBS, alu / VALU_PEAK_TOPS
    roof = ({"bound": "hbm", "achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": fr_h}
            if fr_h >= fr_a else
            {"bound": "alu", "achieved": alu, "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": fr_a})
    roof.update({"kernel": "zone_step", "traffic": None, "avg_launch_us": sec / steps * 1e6, "launches": steps,
                 "other": {"hbm_frac": fr_h, "alu_frac": fr_a}})
    out = {
        "metric": "rail-steps/s (zone model, 128,000 rails x 200)", "value": value, "unit": "rail-steps/s",
        "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 200), "ms_per_step": sec * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak",
        # the paper's own figure for this metric and workload, on its unnamed GPU
        "vs_baseline": value / PAPER_ZONE_RAIL_STEPS_128K,
        "dtype": "fp64 table, u32 draws", "data": "synthetic",
        "config": {"workload": wl.name, "rails": wl.rails, "sites": wl.sites, "ions_per_rail": wl.ions,
                   "zones": wl.zones, "protocol": "5 V for 5 s, then 0 V; 0.016 s per step"},
        "roofline": roof,
        "paper_rail_steps_per_s": PAPER_ZONE_RAIL_STEPS_128K,
    }
    sim.close()
    if not args.no_cpu_baseline:
        import oracle
        p = oracle.ZoneParams(wl.rails, wl.ions, wl.sites, zones=wl.zones, p0=wl.p0, kT=wl.kT_ev,
                              v_factor=wl.v_factor, dt=wl.dt_s, seed=wl.seed)
        X = wl.X0.copy()
        k, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < min(args.cpu_seconds, 10.0):
            oracle.zone_run(p, wl.protocol, X, k, 1)
            k += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": wl.rails * k / el, "unit": "rail-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{k} whole steps of the 128,000-rail lattice, C oracle, {el:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
