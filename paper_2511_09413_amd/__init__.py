"""MI355X rail kinetic Monte Carlo hop step: Python binding of libkmc.so.

Argument marshalling only.  Every step of the hop path runs in the HIP kernels
behind the C ABI (include/kmc.h); PyTorch supplies device memory and streams.
There is no CPU fallback: if the HIP library is missing, loading fails loudly.

Module-level functions carry the C names without the `kmc_` prefix
(init_device, fill_random, set_bias_protocol, run_steps, read_occupancy,
read_current, read_threshold_log, fit_decay, ...).  `Simulator` bundles them with the
torch-owned buffers of one context.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libkmc.so")

KMC_OK, KMC_EINVAL, KMC_EUNSUPPORTED, KMC_EHIP, KMC_ESTATE, KMC_ETOOSMALL = 0, -1, -2, -3, -4, -5
LAUNCH_MODES = {"auto": 0, "half_step": 1, "persistent": 2, "wave": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x2": 2, "phi_fixed": 3}
LOG_DTYPE = np.dtype([("d", np.int32), ("h", np.int32), ("n", np.int64), ("r", np.int32),
                      ("s", np.int32), ("u", np.float64), ("p", np.float64)])


class KmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"kmc status {status}: {message}")
        self.status = status


class kmc_params(C.Structure):
    _fields_ = [("n_devices", C.c_int32), ("rails", C.POINTER(C.c_int32)),
                ("sites", C.POINTER(C.c_int32)), ("nu0_hz", C.c_double), ("ea_ev", C.c_double),
                ("kT_ev", C.c_double), ("dt_s", C.c_double), ("field_coupling", C.c_double),
                ("coulomb_kappa_v", C.c_double), ("screening_sites", C.c_double),
                ("cutoff_sites", C.c_int32), ("rail_range", C.c_int32), ("precision", C.c_int32),
                ("seed", C.c_uint64)]


class kmc_zone_params(C.Structure):
    _fields_ = [("rails", C.c_int32), ("sites", C.c_int32), ("ions_per_rail", C.c_int32), ("zones", C.c_int32),
                ("p0", C.c_double), ("kT_ev", C.c_double), ("hop_over_thickness", C.c_double),
                ("v_factor", C.c_double), ("dt_s", C.c_double), ("seed", C.c_uint64)]


_LIB = None

# Contexts still open when the interpreter exits are destroyed by an atexit
# hook, before the interpreter tears down its modules and before the native
# libraries' own exit handlers run, so that no HIP call comes from a
# finalizer during teardown.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all() -> None:
    for sim in list(_LIVE):
        try:
            sim.close()
        except Exception:
            pass


def lib():
    """Load libkmc.so (built by paper_2511_09413_amd/build.py).  No fallback."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.kmc_build_hash.restype = C.c_char_p
        built = L.kmc_build_hash().decode()
        if os.path.isdir(os.path.join(HERE, "csrc")):
            from .build import source_hash
            if built != source_hash():
                raise ImportError(f"{LIB_PATH} was built from other sources than csrc/ holds now "
                                  f"(run __graft_entry__.build())")
        P, vp = C.POINTER, C.c_void_p
        L.kmc_workspace_bytes.argtypes = [P(kmc_params), P(C.c_size_t)]
        L.kmc_init_device.argtypes = [P(kmc_params), vp, vp, vp, C.c_size_t, vp, P(vp)]
        L.kmc_fill_random.argtypes = [vp, P(C.c_double)]
        L.kmc_load_occupancy.argtypes = [vp]
        L.kmc_set_bias_protocol.argtypes = [vp, C.c_int32, P(C.c_double), P(C.c_double), C.c_int32]
        L.kmc_run_steps.argtypes = [vp, C.c_int64, vp, vp]
        L.kmc_read_occupancy.argtypes = [vp, vp, C.c_size_t]
        L.kmc_read_current.argtypes = [vp, P(C.c_double), P(C.c_int64), P(C.c_double)]
        L.kmc_read_threshold_log.argtypes = [vp, vp, C.c_int64, P(C.c_int64)]
        L.kmc_get_step.argtypes = [vp, P(C.c_int64)]
        L.kmc_set_launch_mode.argtypes = [vp, C.c_int32]
        L.kmc_get_launch_mode.argtypes = [vp, P(C.c_int32)]
        L.kmc_set_tile_sites.argtypes = [vp, C.c_int32]
        L.kmc_score_replay.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, vp]
        L.kmc_score_replay_noalloc.argtypes = [vp, vp, C.c_int64, C.c_int64, vp, vp]
        L.kmc_record_bytes.argtypes = [vp, C.c_int64, C.c_int64, P(C.c_size_t)]
        L.kmc_record_hops.argtypes = [vp, vp, C.c_size_t, C.c_int64, C.c_int64]
        L.kmc_get_persistent_groups.argtypes = [vp, P(C.c_int32)]
        L.kmc_set_persistent_group_limit.argtypes = [vp, C.c_int32]
        L.kmc_set_wait_limit.argtypes = [vp, C.c_int32]
        L.kmc_dense_potential.argtypes = [vp, vp]
        L.kmc_fixed_potential.argtypes = [vp, vp, C.c_int32, P(C.c_int32)]
        L.kmc_set_electrodes.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                         C.c_double]
        L.kmc_autotune.argtypes = [vp, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_double)]
        L.kmc_zone_workspace_bytes.argtypes = [P(kmc_zone_params), P(C.c_size_t)]
        L.kmc_zone_init.argtypes = [P(kmc_zone_params), vp, vp, C.c_size_t, vp, P(vp)]
        L.kmc_zone_load_occupancy.argtypes = [vp]
        L.kmc_zone_set_bias_protocol.argtypes = [vp, P(C.c_double), P(C.c_double), C.c_int32]
        L.kmc_zone_run_steps.argtypes = [vp, C.c_int64, vp, vp]
        L.kmc_zone_read_positions.argtypes = [vp, P(C.c_int32), C.c_size_t]
        L.kmc_zone_get_step.argtypes = [vp, P(C.c_int64)]
        L.kmc_zone_destroy.argtypes = [vp]
        L.kmc_zone_destroy.restype = None
        L.kmc_fit_decay.argtypes = [P(C.c_double), P(C.c_double), C.c_int64, C.c_double, P(C.c_double),
                                    P(C.c_double)]
        L.kmc_last_error.restype = C.c_char_p
        L.kmc_destroy.argtypes = [vp]
        L.kmc_destroy.restype = None
        for name in ("kmc_workspace_bytes", "kmc_init_device", "kmc_fill_random", "kmc_load_occupancy",
                     "kmc_set_bias_protocol", "kmc_run_steps", "kmc_read_occupancy", "kmc_read_current",
                     "kmc_read_threshold_log", "kmc_get_step", "kmc_set_launch_mode", "kmc_get_launch_mode",
                     "kmc_set_tile_sites", "kmc_score_replay", "kmc_get_persistent_groups",
                     "kmc_set_persistent_group_limit", "kmc_set_wait_limit", "kmc_dense_potential", "kmc_fixed_potential",
                     "kmc_set_electrodes",
                     "kmc_autotune", "kmc_fit_decay", "kmc_score_replay_noalloc", "kmc_record_bytes",
                     "kmc_record_hops", "kmc_zone_workspace_bytes",
                     "kmc_zone_init", "kmc_zone_load_occupancy", "kmc_zone_set_bias_protocol", "kmc_zone_run_steps",
                     "kmc_zone_read_positions", "kmc_zone_get_step"):
            getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def _check(status: int) -> None:
    if status != KMC_OK:
        raise KmcError(status, lib().kmc_last_error().decode())


def make_params(physics, rails: Sequence[int], sites: Sequence[int]):
    """kmc_params from a workloads.Physics-like object; returns (struct, keepalive)."""
    r = np.ascontiguousarray(rails, dtype=np.int32)
    s = np.ascontiguousarray(sites, dtype=np.int32)
    p = kmc_params(len(r), r.ctypes.data_as(C.POINTER(C.c_int32)), s.ctypes.data_as(C.POINTER(C.c_int32)),
                   physics.nu0_hz, physics.ea_ev, physics.kT_ev, physics.dt_s, physics.field_coupling,
                   physics.coulomb_kappa_v, physics.screening_sites, physics.cutoff_sites,
                   physics.rail_range, PRECISIONS[physics.precision], physics.seed & 0xFFFFFFFFFFFFFFFF)
    return p, (r, s)


# ---------------------------------------------------------------- C calls
def workspace_bytes(params: kmc_params) -> int:
    out = C.c_size_t(0)
    _check(lib().kmc_workspace_bytes(C.byref(params), C.byref(out)))
    return int(out.value)


def init_device(params: kmc_params, occ_ptr: int, ea_ptr: Optional[int], ws_ptr: int, ws_bytes: int,
                stream: int) -> int:
    h = C.c_void_p(0)
    _check(lib().kmc_init_device(C.byref(params), C.c_void_p(occ_ptr), C.c_void_p(ea_ptr or 0),
                                 C.c_void_p(ws_ptr), ws_bytes, C.c_void_p(stream), C.byref(h)))
    return int(h.value)


def fill_random(ctx: int, filling: Sequence[float]) -> None:
    f = np.ascontiguousarray(filling, dtype=np.float64)
    _check(lib().kmc_fill_random(C.c_void_p(ctx), f.ctypes.data_as(C.POINTER(C.c_double))))


def load_occupancy(ctx: int) -> None:
    _check(lib().kmc_load_occupancy(C.c_void_p(ctx)))


def set_bias_protocol(ctx: int, device: int, t_s: Sequence[float], v_volt: Sequence[float]) -> None:
    t = np.ascontiguousarray(t_s, dtype=np.float64)
    v = np.ascontiguousarray(v_volt, dtype=np.float64)
    if t.shape != v.shape:
        raise ValueError("knot arrays differ in length")
    _check(lib().kmc_set_bias_protocol(C.c_void_p(ctx), device, t.ctypes.data_as(C.POINTER(C.c_double)),
                                       v.ctypes.data_as(C.POINTER(C.c_double)), len(t)))


def run_steps(ctx: int, n_steps: int, net_ptr: int = 0, dec_ptr: int = 0) -> None:
    _check(lib().kmc_run_steps(C.c_void_p(ctx), n_steps, C.c_void_p(net_ptr), C.c_void_p(dec_ptr)))


def read_occupancy(ctx: int, n_sites: int) -> np.ndarray:
    out = np.empty(n_sites, dtype=np.int8)
    _check(lib().kmc_read_occupancy(C.c_void_p(ctx), C.c_void_p(out.ctypes.data), n_sites))
    return out


def read_current(ctx: int, n_devices: int) -> Tuple[np.ndarray, np.ndarray, float]:
    cur = np.zeros(n_devices, dtype=np.float64)
    tot = np.zeros(n_devices, dtype=np.int64)
    t = C.c_double(0.0)
    _check(lib().kmc_read_current(C.c_void_p(ctx), cur.ctypes.data_as(C.POINTER(C.c_double)),
                                  tot.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(t)))
    return cur, tot, float(t.value)


def read_threshold_log(ctx: int, cap: int = 65536) -> Tuple[np.ndarray, int]:
    out = np.zeros(max(cap, 1), dtype=LOG_DTYPE)
    n = C.c_int64(0)
    _check(lib().kmc_read_threshold_log(C.c_void_p(ctx), C.c_void_p(out.ctypes.data), cap, C.byref(n)))
    return out[:min(int(n.value), cap)], int(n.value)


def get_step(ctx: int) -> int:
    n = C.c_int64(0)
    _check(lib().kmc_get_step(C.c_void_p(ctx), C.byref(n)))
    return int(n.value)


def set_launch_mode(ctx: int, mode: str) -> None:
    _check(lib().kmc_set_launch_mode(C.c_void_p(ctx), LAUNCH_MODES[mode]))


def get_launch_mode(ctx: int) -> str:
    m = C.c_int32(0)
    _check(lib().kmc_get_launch_mode(C.c_void_p(ctx), C.byref(m)))
    return {v: k for k, v in LAUNCH_MODES.items()}[int(m.value)]


def set_tile_sites(ctx: int, sites: int) -> None:
    _check(lib().kmc_set_tile_sites(C.c_void_p(ctx), sites))


def score_replay(ctx: int, occ0_ptr: int, step0: int, n_steps: int, weight_ptr: int, grad_ptr: int) -> None:
    _check(lib().kmc_score_replay(C.c_void_p(ctx), C.c_void_p(occ0_ptr), step0, n_steps, C.c_void_p(weight_ptr),
                                  C.c_void_p(grad_ptr)))


def score_replay_noalloc(ctx: int, occ0_ptr: int, step0: int, n_steps: int, weight_ptr: int,
                         grad_ptr: int) -> None:
    _check(lib().kmc_score_replay_noalloc(C.c_void_p(ctx), C.c_void_p(occ0_ptr), step0, n_steps,
                                          C.c_void_p(weight_ptr), C.c_void_p(grad_ptr)))


def fit_decay(t_s: Sequence[float], m: Sequence[float], t0: float, start=None, weights: bool = True):
    """kmc_fit_decay: least-squares C + A exp(-(t - t0)/tau) through (t_s, m).
    Returns ((C, A, tau), d tau / d m as an array, or None when weights=False)."""
    t = np.ascontiguousarray(t_s, dtype=np.float64)
    mm = np.ascontiguousarray(m, dtype=np.float64)
    if t.shape != mm.shape or t.ndim != 1:
        raise ValueError("t_s and m must be 1-D arrays of one length")
    par = np.full(3, np.nan) if start is None else np.ascontiguousarray(start, dtype=np.float64).copy()
    w = np.zeros(len(t)) if weights else None
    PD = C.POINTER(C.c_double)
    _check(lib().kmc_fit_decay(t.ctypes.data_as(PD), mm.ctypes.data_as(PD), len(t), float(t0),
                               par.ctypes.data_as(PD), w.ctypes.data_as(PD) if w is not None else PD()))
    return (float(par[0]), float(par[1]), float(par[2])), w


def destroy(ctx: int) -> None:
    lib().kmc_destroy(C.c_void_p(ctx))


# ------------------------------------------------------------- convenience
class Simulator:
    """One context with torch-owned device buffers (occupancy, barrier field,
    workspace) on one GPU and the current torch stream."""

    def __init__(self, physics, rails: Sequence[int], sites: Sequence[int], occ=None, ea=None,
                 device: str = "cuda:0", mode: str = "auto", tile_sites: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.physics = physics
        self.rails = [int(x) for x in rails]
        self.sites = [int(x) for x in sites]
        self.n_devices = len(self.rails)
        self.n_sites = int(sum(r * l for r, l in zip(self.rails, self.sites)))
        self._params, self._keep = make_params(physics, self.rails, self.sites)
        if occ is None:
            self.occ = torch.zeros(self.n_sites, dtype=torch.int8, device=self.device)
        else:
            self.occ = torch.as_tensor(np.asarray(occ, dtype=np.int8).reshape(-1)).to(self.device)
        self.ea = None
        if ea is not None:
            dt = torch.float64 if physics.precision in ("fp64", "phi_fixed") else torch.float32
            self.ea = torch.as_tensor(np.asarray(ea).reshape(-1)).to(self.device, dt).contiguous()
            if self.ea.numel() != self.n_sites:
                raise ValueError("barrier field size differs from the lattice")
        nbytes = workspace_bytes(self._params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            _LIVE.add(self)
            self.ctx = init_device(self._params, self.occ.data_ptr(),
                                   self.ea.data_ptr() if self.ea is not None else None,
                                   self._ws_ptr, nbytes, self.stream.cuda_stream)
        if tile_sites:
            set_tile_sites(self.ctx, tile_sites)
        if mode != "auto":
            set_launch_mode(self.ctx, mode)

    def fill_random(self, filling: Sequence[float]) -> None:
        fill_random(self.ctx, filling)

    def load_occupancy(self, occ) -> None:
        self.occ.copy_(self.torch.as_tensor(np.asarray(occ, dtype=np.int8).reshape(-1)).to(self.device))
        load_occupancy(self.ctx)

    def set_bias_protocol(self, t_s, v_volt, device: int = -1) -> None:
        set_bias_protocol(self.ctx, device, t_s, v_volt)

    def set_protocols(self, protocols) -> None:
        for d, (t, v) in enumerate(protocols):
            set_bias_protocol(self.ctx, d, t, v)

    def run_steps(self, n_steps: int, tallies: bool = False):
        """Advance n_steps; with tallies=True return (net [n,D], deciles [n,D,10]) torch tensors."""
        torch = self.torch
        if not tallies:
            run_steps(self.ctx, n_steps)
            return None
        net = torch.empty((n_steps, self.n_devices), dtype=torch.int32, device=self.device)
        dec = torch.empty((n_steps, self.n_devices, 10), dtype=torch.int32, device=self.device)
        run_steps(self.ctx, n_steps, net.data_ptr(), dec.data_ptr())
        return net, dec

    def snapshot(self):
        """Device copy of the current occupancy (the start state of a later replay)."""
        return self.occ.clone()

    def record_hops(self, max_steps: int, cap: int = 1024) -> None:
        """Record the accepted hops of the next max_steps steps (kmc_record_hops),
        cap per half-step, so that a score replay of them from the current
        state takes the decisions from the recording; max_steps = 0 ends it.
        The buffer is a device tensor this object keeps."""
        if max_steps == 0:
            _check(lib().kmc_record_hops(C.c_void_p(self.ctx), None, 0, 0, 0))
            self._record = None
            return
        nbytes = C.c_size_t()
        _check(lib().kmc_record_bytes(C.c_void_p(self.ctx), max_steps, cap, C.byref(nbytes)))
        buf = self.torch.empty(nbytes.value + 256, dtype=self.torch.uint8, device=self.device)
        ptr = (buf.data_ptr() + 255) // 256 * 256
        _check(lib().kmc_record_hops(C.c_void_p(self.ctx), C.c_void_p(ptr), nbytes.value, max_steps, cap))
        self._record = buf

    def score_replay(self, occ0, step0: int, weights):
        """Score-function terms of the steps [step0, step0 + len(weights)) replayed
        from occ0 (device int8 tensor), weighted by weights [n_steps, D]; returns
        grad [D, 4] (float64, device) over (Ea shift, nu0, kappa, alpha)."""
        torch = self.torch
        occ0 = torch.as_tensor(occ0).to(self.device, torch.int8).contiguous()
        if occ0.numel() != self.n_sites:
            raise ValueError("occ0 size differs from the lattice")
        w = torch.as_tensor(weights).to(self.device, torch.float64).contiguous()
        if w.dim() != 2 or w.shape[1] != self.n_devices:
            raise ValueError("weights must be [n_steps, n_devices]")
        grad = torch.empty((self.n_devices, 4), dtype=torch.float64, device=self.device)
        score_replay(self.ctx, occ0.data_ptr(), step0, w.shape[0], w.data_ptr(), grad.data_ptr())
        return grad

    def dense_potential(self):
        """Coulomb potential of the current state at every site (float32 device
        tensor, occupancy layout); KMC_BF16X2 contexts only."""
        phi = self.torch.empty(self.n_sites, dtype=self.torch.float32, device=self.device)
        _check(lib().kmc_dense_potential(C.c_void_p(self.ctx), C.c_void_p(phi.data_ptr())))
        return phi

    def set_electrodes(self, ea_ground: float, mu_ground: float, ea_bias: float, mu_bias: float,
                       device: int = -1, open: bool = True) -> None:
        """Open (or close again) the electrodes of one device or of all
        (kmc_set_electrodes): transfer barriers and reservoir energies in eV."""
        _check(lib().kmc_set_electrodes(C.c_void_p(self.ctx), device, 1 if open else 0, ea_ground, mu_ground,
                                        ea_bias, mu_bias))

    def fixed_potential(self, recompute: bool = False):
        """(phi, F): the fixed-point potential of every site (int64 device
        tensor, occupancy layout, units of 2^-F V) of a KMC_PHI_FIXED context;
        recompute=True computes it from scratch from the current state."""
        phi = self.torch.empty(self.n_sites, dtype=self.torch.int64, device=self.device)
        F = C.c_int32(0)
        _check(lib().kmc_fixed_potential(C.c_void_p(self.ctx), C.c_void_p(phi.data_ptr()), 1 if recompute else 0,
                                         C.byref(F)))
        return phi, int(F.value)

    def read_occupancy(self) -> np.ndarray:
        return read_occupancy(self.ctx, self.n_sites)

    def read_current(self):
        return read_current(self.ctx, self.n_devices)

    def read_threshold_log(self, cap: int = 65536):
        return read_threshold_log(self.ctx, cap)

    def autotune(self, trial_steps: int = 256, cache: Optional[str] = None) -> dict:
        """Select the fastest launch strategy and tile size (kmc_autotune; the
        state is restored, no trajectory changes).  With `cache` (a JSON file),
        a configuration measured before for the same shapes, physics and GPU is
        applied without trials, and new results are added to the file."""
        import json
        key = self._tune_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                hit = table[key]
                set_tile_sites(self.ctx, int(hit["tile_sites"]))
                set_launch_mode(self.ctx, hit["mode"])
                return dict(hit, cached=True)
        t, m, us = C.c_int32(0), C.c_int32(0), C.c_double(0.0)
        _check(lib().kmc_autotune(C.c_void_p(self.ctx), trial_steps, C.byref(t), C.byref(m), C.byref(us)))
        out = {"tile_sites": int(t.value), "mode": {1: "half_step", 2: "persistent", 3: "wave"}.get(int(m.value), "auto"),
               "us_per_step": float(us.value), "trial_steps": trial_steps}
        if cache:
            table[key] = out
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return dict(out, cached=False)

    def _tune_key(self) -> str:
        import hashlib
        ph = self.physics
        gpu = self.torch.cuda.get_device_name(self.device)
        desc = repr((self.rails, self.sites, ph.precision, ph.rail_range, ph.cutoff_sites, ph.screening_sites,
                     gpu, self.ea is not None))
        return hashlib.sha1(desc.encode()).hexdigest()

    def set_wait_limit(self, polls: int) -> None:
        """Polls before a persistent kernel's neighbour wait is declared hung
        (kmc_set_wait_limit; 0: every wait fails at once)."""
        _check(lib().kmc_set_wait_limit(C.c_void_p(self.ctx), polls))

    def set_group_limit(self, max_tiles: int) -> None:
        """At most max_tiles workgroup tiles per persistent launch (0 = what fits)."""
        _check(lib().kmc_set_persistent_group_limit(C.c_void_p(self.ctx), max_tiles))

    @property
    def n_groups(self) -> int:
        """Persistent launches per 1024-step chunk (groups of whole devices)."""
        out = C.c_int32(0)
        _check(lib().kmc_get_persistent_groups(C.c_void_p(self.ctx), C.byref(out)))
        return int(out.value)

    @property
    def launch_mode(self) -> str:
        return get_launch_mode(self.ctx)

    def set_launch_mode(self, mode: str) -> None:
        set_launch_mode(self.ctx, mode)

    def set_tile_sites(self, sites: int) -> None:
        set_tile_sites(self.ctx, sites)

    @property
    def step(self) -> int:
        return get_step(self.ctx)

    def close(self) -> None:
        if getattr(self, "ctx", 0):
            destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ zone model
class ZoneSimulator:
    """The paper's zone model (kmc_zone_*): one lattice of `rails` rails of
    `sites` columns with ions_per_rail ions each, torch-owned occupancy and
    workspace on one GPU and the current torch stream."""

    def __init__(self, rails: int, sites: int, ions_per_rail: int, zones: int = 10, p0: float = 0.5,
                 kT_ev: float = 8.617333262e-5 * 300.0, hop_over_thickness: Optional[float] = None,
                 v_factor: float = 5e-5, dt_s: float = 1e-3, seed: int = 0, occ=None, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.rails, self.sites, self.ions, self.zones = int(rails), int(sites), int(ions_per_rail), int(zones)
        self.params = kmc_zone_params(self.rails, self.sites, self.ions, self.zones, p0, kT_ev,
                                      1.0 / sites if hop_over_thickness is None else hop_over_thickness,
                                      v_factor, dt_s, seed & 0xFFFFFFFFFFFFFFFF)
        if occ is None:
            raise ValueError("ZoneSimulator needs an initial occupancy [rails][sites]")
        self.occ = torch.as_tensor(np.asarray(occ, dtype=np.int8).reshape(-1)).to(self.device)
        if self.occ.numel() != self.rails * self.sites:
            raise ValueError("occupancy size differs from rails * sites")
        nbytes = C.c_size_t(0)
        _check(lib().kmc_zone_workspace_bytes(C.byref(self.params), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ws = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p(0)
        with torch.cuda.device(self.device):
            _check(lib().kmc_zone_init(C.byref(self.params), C.c_void_p(self.occ.data_ptr()), C.c_void_p(ws),
                                       nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.ctx = int(h.value)
        _LIVE.add(self)

    def set_bias_protocol(self, t_s, v_volt) -> None:
        t = np.ascontiguousarray(t_s, dtype=np.float64)
        v = np.ascontiguousarray(v_volt, dtype=np.float64)
        if t.shape != v.shape:
            raise ValueError("knot arrays differ in length")
        PD = C.POINTER(C.c_double)
        _check(lib().kmc_zone_set_bias_protocol(C.c_void_p(self.ctx), t.ctypes.data_as(PD), v.ctypes.data_as(PD),
                                                len(t)))

    def load_occupancy(self, occ) -> None:
        self.occ.copy_(self.torch.as_tensor(np.asarray(occ, dtype=np.int8).reshape(-1)).to(self.device))
        _check(lib().kmc_zone_load_occupancy(C.c_void_p(self.ctx)))

    def run_steps(self, n_steps: int, tallies: bool = False):
        """Advance n_steps; with tallies=True return (net [n], zones [n, Z]) torch tensors."""
        torch = self.torch
        if not tallies:
            _check(lib().kmc_zone_run_steps(C.c_void_p(self.ctx), n_steps, None, None))
            return None
        net = torch.empty(n_steps, dtype=torch.int32, device=self.device)
        zones = torch.empty((n_steps, self.zones), dtype=torch.int32, device=self.device)
        _check(lib().kmc_zone_run_steps(C.c_void_p(self.ctx), n_steps, C.c_void_p(net.data_ptr()),
                                        C.c_void_p(zones.data_ptr())))
        return net, zones

    def read_positions(self) -> np.ndarray:
        out = np.zeros((self.rails, self.ions), dtype=np.int32)
        _check(lib().kmc_zone_read_positions(C.c_void_p(self.ctx), out.ctypes.data_as(C.POINTER(C.c_int32)),
                                             out.size))
        return out

    def read_occupancy(self) -> np.ndarray:
        self.torch.cuda.current_stream(self.device).synchronize()
        return self.occ.cpu().numpy()

    @property
    def step(self) -> int:
        n = C.c_int64(0)
        _check(lib().kmc_zone_get_step(C.c_void_p(self.ctx), C.byref(n)))
        return int(n.value)

    def close(self) -> None:
        if getattr(self, "ctx", 0):
            lib().kmc_zone_destroy(C.c_void_p(self.ctx))
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
