"""Seeded synthetic inputs for the rail-KMC hop step.

This module only *describes* workloads: device shapes, fillings, voltage
protocols as knot lists, per-site barrier fields and physical constants.  It
holds none of the method's arithmetic, and it is the only code that the CPU
oracle (oracle/) and the HIP library binding (paper_2511_09413_amd/) both use.

The paper's experiments use no public dataset; every input here is synthetic,
with the shapes, fillings and protocol shapes of the paper's use cases
(relaxation after a polarising bias step, triangular I-V sweeps, spike-pair
pulses; main text section 4 and SI S2.2) at the sizes of the five benchmark
configurations (C1 plain FP64, C2 single large device, C3 batched ensemble,
C4 dense long-range potential, C5 differentiation).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

FP64 = "fp64"
FP32 = "fp32"
BF16X2 = "bf16x2"
PHI_FIXED = "phi_fixed"

NS = 1e-9


@dataclass
class Physics:
    """Physical and numerical constants of one run (SI units plus eV)."""
    nu0_hz: float = 1e12
    ea_ev: float = 0.3
    kT_ev: float = 0.0259
    dt_s: float = 1e-12
    field_coupling: float = 1.0
    coulomb_kappa_v: float = 0.025
    screening_sites: float = 4.0   # 0 = unscreened 1/r
    cutoff_sites: int = 16         # inclusive cutoff along the rail
    rail_range: int = 1            # rails within this distance interact
    precision: str = FP64
    seed: int = 0

    def replace(self, **kw) -> "Physics":
        return dataclasses.replace(self, **kw)


Protocol = Tuple[List[float], List[float]]  # (knot times in s, knot voltages in V)


@dataclass
class Workload:
    name: str
    physics: Physics
    rails: List[int]
    sites: List[int]
    filling: List[float]
    protocols: List[Protocol]
    n_steps: int
    ea_site: Optional[np.ndarray] = None  # flat, devices concatenated
    notes: str = ""

    @property
    def n_devices(self) -> int:
        return len(self.rails)

    @property
    def n_sites(self) -> int:
        return int(sum(r * l for r, l in zip(self.rails, self.sites)))

    def device_offsets(self) -> List[int]:
        off, out = 0, []
        for r, l in zip(self.rails, self.sites):
            out.append(off)
            off += r * l
        return out


# ---------------------------------------------------------------- protocols
def constant(v: float) -> Protocol:
    return [0.0], [float(v)]


def triangle(amplitude: float, period_s: float) -> Protocol:
    """One period 0 -> +A -> -A -> 0 (the I-V sweep shape, main text Fig. 2)."""
    q = period_s / 4.0
    return [0.0, q, 3 * q, 4 * q], [0.0, amplitude, -amplitude, 0.0]


def step_then_relax(v: float, t_on_s: float) -> Protocol:
    """Polarising bias for t_on, then 0 V (relaxation decay, main text Fig. 1)."""
    return [0.0, t_on_s, t_on_s], [float(v), float(v), 0.0]


def stdp_pair(delta_t_s: float, t_pre_s: float = 50 * NS,
              width_s: float = 10 * NS, pos_v: float = 1.0, neg_v: float = -0.5) -> Protocol:
    """Pre/post spike pair V(t) = s(t - t_pre) - s(t - t_pre - delta_t), with a
    biphasic spike s = +pos for [0, w), neg for [w, 2w), 0 elsewhere."""
    def spike(tau: float) -> float:
        if 0.0 <= tau < width_s:
            return pos_v
        if width_s <= tau < 2 * width_s:
            return neg_v
        return 0.0

    t_post = t_pre_s + delta_t_s
    bps = sorted({t_pre_s, t_pre_s + width_s, t_pre_s + 2 * width_s,
                  t_post, t_post + width_s, t_post + 2 * width_s})
    bps = [b for b in bps if b >= 0.0]
    ts, vs = [0.0], [spike(-t_pre_s) - spike(-t_post)]
    for b in bps:
        left = spike(b - 1e-15 - t_pre_s) - spike(b - 1e-15 - t_post)
        right = spike(b - t_pre_s) - spike(b - t_post)
        ts += [b, b]
        vs += [left, right]
    return ts, vs


# ------------------------------------------------------------------ fields
def gaussian_barriers(shape: Sequence[int], mean: float, std: float, seed: int,
                      dtype=np.float32) -> np.ndarray:
    """Per-site barriers drawn from N(mean, std) with numpy's PCG64 (disordered
    polymer matrix)."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.normal(mean, std, size=tuple(shape)).astype(dtype).reshape(-1)


def sparse_traps(shape: Sequence[int], base: float, fraction: float, depth: float, seed: int,
                 dtype=np.float32, field: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-site barriers with deep traps at a few random positions (the
    charge-trapping effect of scarce defects the paper's conclusion names):
    round(fraction x sites) distinct sites, chosen with numpy's PCG64, get
    `depth` eV more than the rest (`base`, or a given field)."""
    n = int(np.prod(shape))
    out = (np.full(n, base, dtype=np.float64) if field is None
           else np.asarray(field, dtype=np.float64).reshape(-1).copy())
    g = np.random.Generator(np.random.PCG64(seed))
    k = int(round(fraction * n))
    out[g.permutation(n)[:k]] += depth
    return out.astype(dtype)


# --------------------------------------------------------------- workloads
def c1_plain_fp64(n_steps: int = 10_000) -> Workload:
    ph = Physics(precision=FP64, seed=0)
    return Workload("c1_plain_fp64_64x128", ph, [64], [128], [0.2], [constant(0.5)],
                    n_steps, notes="64 rails x 128 sites, 20% filling, 0.5 V, FP64")


def c2_large_device(n_steps: int = 100_000, rails: int = 4096, sites: int = 1024) -> Workload:
    ph = Physics(precision=FP32, seed=0)
    period = n_steps * ph.dt_s
    ea = gaussian_barriers((rails, sites), 0.3, 0.02, seed=2, dtype=np.float32)
    return Workload(f"c2_large_device_{rails}x{sites}", ph, [rails], [sites], [0.3],
                    [triangle(2.0, period)], n_steps, ea_site=ea,
                    notes="4096 rails x 1024 sites, 30% filling, +-2 V triangle, "
                          "Ea ~ N(0.3, 0.02) eV per site, FP32")


def c3_batched(n_steps: int = 100_000, n_devices: int = 256, seed: int = 3,
               max_rails: int = 1024, max_sites: int = 2048) -> Workload:
    ph = Physics(precision=FP32, seed=0)
    g = np.random.Generator(np.random.PCG64(seed))
    rails = g.integers(32, max_rails + 1, size=n_devices).tolist()
    sites = g.integers(64, max_sites + 1, size=n_devices).tolist()
    fill = g.uniform(0.05, 0.4, size=n_devices).tolist()
    kinds = g.integers(0, 3, size=n_devices)
    dts = g.integers(-50, 51, size=n_devices)
    span = n_steps * ph.dt_s
    protos = []
    for k, dtn in zip(kinds, dts):
        if k == 0:
            protos.append(step_then_relax(1.0, 0.5 * span))
        elif k == 1:
            protos.append(triangle(1.0, span))
        else:
            protos.append(stdp_pair(float(dtn) * NS))
    return Workload(f"c3_batched_{n_devices}dev", ph, rails, sites, fill, protos, n_steps,
                    notes="256 devices, rails U{32..1024}, sites U{64..2048}, "
                          "filling U[0.05,0.4]; step/triangle/STDP protocols; FP32")


def c4_dense(n_steps: int = 1000, replicas: int = 64, rails: int = 1024, sites: int = 512) -> Workload:
    ph = Physics(precision=BF16X2, seed=0, screening_sites=0.0, cutoff_sites=sites - 1,
                 rail_range=4)
    return Workload(f"c4_dense_{replicas}x{rails}x{sites}", ph, [rails] * replicas,
                    [sites] * replicas, [0.3] * replicas, [constant(1.0)] * replicas, n_steps,
                    notes="unscreened 1/r over the whole rail and +-4 rails, BF16 hi/lo")


def c5_gradient(n_steps: int = 20_000, replicas: int = 512, rails: int = 256, sites: int = 512,
                ea_ev: float = 0.3) -> Workload:
    ph = Physics(precision=FP32, seed=0, ea_ev=ea_ev)
    t_on = (n_steps // 2) * ph.dt_s
    return Workload(f"c5_gradient_{replicas}x{rails}x{sites}", ph, [rails] * replicas,
                    [sites] * replicas, [0.3] * replicas,
                    [step_then_relax(1.0, t_on)] * replicas, n_steps,
                    notes="1 V pulse for half the run, then relaxation; FP32 step")


def small_case(rails: int, sites: int, filling: float = 0.3, precision: str = FP64,
               ea_ev: float = 0.15, protocol: Optional[Protocol] = None, n_devices: int = 1,
               seed: int = 0, **phys) -> Workload:
    """Validation variant: small lattice, lower barrier so that hops are common."""
    ph = Physics(precision=precision, seed=seed, ea_ev=ea_ev, **phys)
    pr = protocol if protocol is not None else constant(0.5)
    return Workload(f"small_{n_devices}x{rails}x{sites}", ph, [rails] * n_devices,
                    [sites] * n_devices, [filling] * n_devices, [pr] * n_devices, 0)


# ------------------------------------------------------------ zone model
@dataclass
class ZoneWorkload:
    """The paper's own zone model at Table S1/S2 shapes: `rails` rails of
    `sites` columns, `ions` ions per rail at uniformly random columns
    (seeded), a protocol, and the model's constants."""
    name: str
    rails: int
    sites: int
    ions: int
    zones: int
    p0: float
    kT_ev: float
    v_factor: float
    dt_s: float
    seed: int
    protocol: Protocol
    n_steps: int
    X0: np.ndarray   # [rails][ions] 1-based columns, increasing

    def occupancy(self) -> np.ndarray:
        occ = np.zeros((self.rails, self.sites), dtype=np.int8)
        np.put_along_axis(occ, self.X0.astype(np.int64) - 1, 1, axis=1)
        return occ.reshape(-1)


def zone_positions(rails: int, sites: int, ions: int, seed: int) -> np.ndarray:
    """ions distinct columns per rail, uniformly random (PCG64), sorted."""
    g = np.random.Generator(np.random.PCG64(seed))
    keys = g.random((rails, sites))
    cols = np.argsort(keys, axis=1)[:, :ions]
    return (np.sort(cols, axis=1) + 1).astype(np.int32)


def zone_relaxation(rails: int = 4000, sites: int = 200, ion_fraction: float = 0.3, n_steps: int = 187_200,
                    seed: int = 5, p0: float = 0.5, v_factor: float = 5e-5) -> ZoneWorkload:
    """Table S1 defaults (200 columns, 30 % ions, 300 K, a 5 V polarisation
    for 5 s then relaxation at 0 V, the effective voltage difference factor
    5e-5 V) with one step per relaxation time (0.016 s); Table S2 runs 500 to
    128,000 rails for 187,200 steps."""
    dt = 0.016
    ions = int(round(ion_fraction * sites))
    return ZoneWorkload(f"zone_relaxation_{rails}x{sites}", rails, sites, ions, 10, p0, 8.617333262e-5 * 300.0,
                        v_factor, dt, seed, step_then_relax(5.0, 5.0), n_steps,
                        zone_positions(rails, sites, ions, seed + 100))
