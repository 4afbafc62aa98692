"""CPU oracle for the rail-KMC hop step (ctypes wrapper around kmc_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() to
check the GPU result, and by bench.py's cpu_baseline leg.  The product library
never imports this package.  See kmc_oracle.c for the definition of what is
computed and the passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None


class _Params(C.Structure):
    _fields_ = [("n_devices", C.c_int), ("rails", C.POINTER(C.c_int)),
                ("sites", C.POINTER(C.c_int)), ("nu0", C.c_double), ("ea", C.c_double),
                ("kT", C.c_double), ("dt", C.c_double), ("alpha", C.c_double),
                ("kappa", C.c_double), ("lambda_", C.c_double), ("cutoff", C.c_int),
                ("rail_range", C.c_int), ("fp32", C.c_int), ("seed", C.c_uint64),
                ("ea_site", C.POINTER(C.c_double))]


class _Protocol(C.Structure):
    _fields_ = [("t", C.POINTER(C.c_double)), ("v", C.POINTER(C.c_double)),
                ("n_knots", C.c_int), ("n_set", C.c_int64)]


class _Electrodes(C.Structure):
    _fields_ = [("open", C.c_int), ("ea_ground", C.c_double), ("mu_ground", C.c_double),
                ("ea_bias", C.c_double), ("mu_bias", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("shuffle_seed", C.c_uint64), ("rail_lo", C.c_int), ("rail_hi", C.c_int),
                ("score_w", C.POINTER(C.c_double)), ("score_grad", C.POINTER(C.c_double)),
                ("score_mag", C.POINTER(C.c_double)), ("score_sens", C.POINTER(C.c_double)),
                ("score_sens_arg", C.POINTER(C.c_double)), ("score_sens_b", C.POINTER(C.c_double)),
                ("score_hops", C.POINTER(C.c_int64)), ("score_coul64", C.c_int),
                ("electrodes", C.POINTER(_Electrodes))]


class _ZoneParams(C.Structure):
    _fields_ = [("rails", C.c_int), ("ions", C.c_int), ("sites", C.c_int), ("zones", C.c_int),
                ("p0", C.c_double), ("kT", C.c_double), ("hop_over_thickness", C.c_double),
                ("v_factor", C.c_double), ("dt", C.c_double), ("seed", C.c_uint64)]


LOG_DTYPE = np.dtype([("d", np.int32), ("h", np.int32), ("n", np.int64), ("r", np.int32),
                      ("s", np.int32), ("u", np.float64), ("p", np.float64)])


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_hop_word.argtypes = [C.c_uint64, C.c_int, C.c_int64, C.c_int, C.c_int]
        L.orc_hop_word.restype = C.c_uint32
        L.orc_place_word.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int]
        L.orc_place_word.restype = C.c_uint32
        L.orc_electrode_word.argtypes = [C.c_uint64, C.c_int, C.c_int64, C.c_int, C.c_int, C.c_int]
        L.orc_electrode_word.restype = C.c_uint32
        L.orc_electrode_delta_energy.argtypes = [P(_Params), C.c_int, C.c_int, P(C.c_int8), C.c_int, C.c_int,
                                                 C.c_int, C.c_double, C.c_double]
        L.orc_electrode_delta_energy.restype = C.c_double
        L.orc_kernel.argtypes = [P(_Params), C.c_int, C.c_int]
        L.orc_kernel.restype = C.c_double
        L.orc_protocol_voltage.argtypes = [P(C.c_double), P(C.c_double), C.c_int, C.c_double]
        L.orc_protocol_voltage.restype = C.c_double
        L.orc_delta_energy_f64.argtypes = [P(_Params), C.c_int, C.c_int, P(C.c_int8), C.c_int,
                                           C.c_int, C.c_int, C.c_double]
        L.orc_delta_energy_f64.restype = C.c_double
        L.orc_delta_energy_f32.argtypes = L.orc_delta_energy_f64.argtypes
        L.orc_delta_energy_f32.restype = C.c_float
        L.orc_dense_potential.argtypes = [P(_Params), P(C.c_int8), P(C.c_double)]
        L.orc_dense_potential.restype = None
        L.orc_hop_prob_f64.argtypes = [P(_Params), C.c_double, C.c_double]
        L.orc_hop_prob_f64.restype = C.c_double
        L.orc_hop_prob_f32.argtypes = [P(_Params), C.c_double, C.c_float]
        L.orc_hop_prob_f32.restype = C.c_float
        L.orc_ions_per_rail.argtypes = [C.c_double, C.c_int]
        L.orc_ions_per_rail.restype = C.c_int
        L.orc_fill.argtypes = [P(_Params), P(C.c_double), P(C.c_int8)]
        L.orc_run.argtypes = [P(_Params), P(_Protocol), P(C.c_int8), C.c_int64, C.c_int64,
                              P(C.c_int32), P(C.c_int32), P(C.c_int64), C.c_void_p, C.c_int64,
                              P(C.c_int64), P(_Opts)]
        L.orc_run.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_zone_index.argtypes = [C.c_int, C.c_int, C.c_int]
        L.orc_zone_index.restype = C.c_int
        L.orc_zone_table.argtypes = [P(_ZoneParams), C.c_double, P(C.c_int64), P(C.c_double), P(C.c_double),
                                     P(C.c_double)]
        L.orc_zone_table.restype = None
        L.orc_zone_words.argtypes = [C.c_uint64, C.c_int, C.c_int, C.c_int64, P(C.c_uint32), P(C.c_uint32)]
        L.orc_zone_words.restype = None
        L.orc_zone_run.argtypes = [P(_ZoneParams), P(_Protocol), P(C.c_int32), C.c_int64, C.c_int64,
                                   P(C.c_int32), P(C.c_int32), P(C.c_int64)]
        L.orc_zone_run.restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return C.POINTER(ctype)()
    return a.ctypes.data_as(C.POINTER(ctype))


class OracleParams:
    """Holds the C parameter struct and keeps its arrays alive."""

    def __init__(self, physics, rails: Sequence[int], sites: Sequence[int],
                 ea_site: Optional[np.ndarray] = None):
        self._rails = np.ascontiguousarray(rails, dtype=np.int32)
        self._sites = np.ascontiguousarray(sites, dtype=np.int32)
        self._ea = None if ea_site is None else np.ascontiguousarray(ea_site, dtype=np.float64)
        ph = physics
        if ph.precision not in ("fp64", "fp32"):
            raise ValueError("the oracle runs the fp64 or fp32 path")
        self.s = _Params(len(self._rails), _ptr(self._rails, C.c_int), _ptr(self._sites, C.c_int),
                         ph.nu0_hz, ph.ea_ev, ph.kT_ev, ph.dt_s, ph.field_coupling,
                         ph.coulomb_kappa_v, ph.screening_sites, ph.cutoff_sites, ph.rail_range,
                         1 if ph.precision == "fp32" else 0, ph.seed & 0xFFFFFFFFFFFFFFFF,
                         _ptr(self._ea, C.c_double))
        self.physics = physics
        self.rails = [int(x) for x in self._rails]
        self.sites = [int(x) for x in self._sites]

    @property
    def n_sites(self) -> int:
        return int(sum(r * l for r, l in zip(self.rails, self.sites)))


def params_for(workload, **overrides) -> OracleParams:
    ph = workload.physics.replace(**overrides) if overrides else workload.physics
    return OracleParams(ph, workload.rails, workload.sites, workload.ea_site)


def philox(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def hop_word(seed: int, d: int, n: int, r: int, s: int) -> int:
    return int(lib().orc_hop_word(seed, d, n, r, s))


def place_word(seed: int, d: int, r: int, s: int) -> int:
    return int(lib().orc_place_word(seed, d, r, s))


def electrode_word(seed: int, d: int, n: int, r: int, h: int, side: int) -> int:
    return int(lib().orc_electrode_word(seed, d, n, r, h, side))


def electrode_delta_energy(p: OracleParams, R: int, L: int, S: np.ndarray, r: int, side: int, inject: bool,
                           V: float, mu: float) -> float:
    """Energy change of a transfer across the boundary bond of rail r (side 0:
    grounded, 1: biased) from snapshot S of one device, in p's precision."""
    S = np.ascontiguousarray(S, dtype=np.int8).reshape(-1)
    return float(lib().orc_electrode_delta_energy(C.byref(p.s), R, L, _ptr(S, C.c_int8), r, side,
                                                  1 if inject else 0, V, mu))


def _electrodes(electrodes, D):
    """[D] orc_electrodes from None or a per-device list of None (blocking) or
    (ea_ground, mu_ground, ea_bias, mu_bias)."""
    if electrodes is None:
        return None
    if len(electrodes) != D:
        raise ValueError("one electrode entry per device")
    arr = (_Electrodes * D)()
    for d, e in enumerate(electrodes):
        if e is None:
            arr[d] = _Electrodes(0, 0.0, 0.0, 0.0, 0.0)
        else:
            arr[d] = _Electrodes(1, *[float(x) for x in e])
    return arr


def kernel(p: OracleParams, ds: int, dr: int) -> float:
    return float(lib().orc_kernel(C.byref(p.s), ds, dr))


def protocol_voltage(t_k: Sequence[float], v_k: Sequence[float], t_rel: float) -> float:
    t = np.ascontiguousarray(t_k, dtype=np.float64)
    v = np.ascontiguousarray(v_k, dtype=np.float64)
    return float(lib().orc_protocol_voltage(_ptr(t, C.c_double), _ptr(v, C.c_double), len(t), t_rel))


def delta_energy(p: OracleParams, R: int, L: int, S: np.ndarray, r: int, o: int, t: int,
                 V: float, fp32: bool = False) -> float:
    S = np.ascontiguousarray(S, dtype=np.int8).reshape(-1)
    f = lib().orc_delta_energy_f32 if fp32 else lib().orc_delta_energy_f64
    return float(f(C.byref(p.s), R, L, _ptr(S, C.c_int8), r, o, t, V))


def dense_potential(p: OracleParams, occ: np.ndarray) -> np.ndarray:
    """phi at every site (binary64), devices concatenated, [rails*sites] each."""
    o = np.ascontiguousarray(occ, dtype=np.int8).reshape(-1)
    if o.size != p.n_sites:
        raise ValueError("occupancy size mismatch")
    phi = np.zeros(p.n_sites, dtype=np.float64)
    lib().orc_dense_potential(C.byref(p.s), _ptr(o, C.c_int8), _ptr(phi, C.c_double))
    return phi


def hop_prob(p: OracleParams, ea: float, dE: float, fp32: bool = False) -> float:
    if fp32:
        return float(lib().orc_hop_prob_f32(C.byref(p.s), ea, dE))
    return float(lib().orc_hop_prob_f64(C.byref(p.s), ea, dE))


def set_threads(n: int) -> None:
    """OpenMP threads of the plain run path (rails split inside each
    half-step; no effect on results, only on the log's entry order)."""
    lib().orc_set_threads(int(n))


def ions_per_rail(filling: float, L: int) -> int:
    return int(lib().orc_ions_per_rail(filling, L))


def fill(p: OracleParams, filling: Sequence[float]) -> np.ndarray:
    occ = np.zeros(p.n_sites, dtype=np.int8)
    f = np.ascontiguousarray(filling, dtype=np.float64)
    lib().orc_fill(C.byref(p.s), _ptr(f, C.c_double), _ptr(occ, C.c_int8))
    return occ


class Protocols:
    def __init__(self, protocols, n_set: Sequence[int]):
        self._keep = []
        arr = (_Protocol * len(protocols))()
        for i, (pr, ns) in enumerate(zip(protocols, n_set)):
            t = np.ascontiguousarray(pr[0], dtype=np.float64)
            v = np.ascontiguousarray(pr[1], dtype=np.float64)
            self._keep += [t, v]
            arr[i] = _Protocol(_ptr(t, C.c_double), _ptr(v, C.c_double), len(t), int(ns))
        self.arr = arr


def run(p: OracleParams, protocols, occ: np.ndarray, n0: int, n_steps: int,
        n_set: Optional[Sequence[int]] = None, want_dec: bool = True, log_cap: int = 4096,
        shuffle_seed: int = 0, rail_lo: int = 0, rail_hi: int = 0,
        net_total: Optional[np.ndarray] = None, electrodes=None) -> Dict[str, np.ndarray]:
    """Advance `occ` (modified in place) by n_steps steps starting at step n0."""
    D = len(p.rails)
    if len(protocols) != D:
        raise ValueError("one protocol per device")
    occ_c = np.ascontiguousarray(occ, dtype=np.int8).reshape(-1)
    if occ_c.size != p.n_sites:
        raise ValueError("occupancy size mismatch")
    prot = Protocols(protocols, n_set if n_set is not None else [0] * D)
    net = np.zeros((n_steps, D), dtype=np.int32)
    dec = np.zeros((n_steps, D, 10), dtype=np.int32) if want_dec else None
    tot = net_total if net_total is not None else np.zeros(D, dtype=np.int64)
    log = np.zeros(max(log_cap, 1), dtype=LOG_DTYPE)
    n_log = C.c_int64(0)
    el = _electrodes(electrodes, D)
    opts = _Opts(shuffle_seed, rail_lo, rail_hi, None, None, None, None)
    if el is not None:
        opts.electrodes = C.cast(el, C.POINTER(_Electrodes))
    rc = lib().orc_run(C.byref(p.s), prot.arr, _ptr(occ_c, C.c_int8), n0, n_steps,
                       _ptr(net, C.c_int32), _ptr(dec, C.c_int32), _ptr(tot, C.c_int64),
                       log.ctypes.data_as(C.c_void_p), log_cap, C.byref(n_log), C.byref(opts))
    if rc != 0:
        raise ValueError("oracle rejected the run (step counter out of range)")
    if occ_c is not occ:
        occ.reshape(-1)[:] = occ_c
    n_ev = int(n_log.value)
    return {"occ": occ_c, "net": net, "dec": dec, "net_total": tot,
            "log": log[:min(n_ev, log_cap)], "n_log": n_ev}


def score_replay(p: OracleParams, protocols, occ0: np.ndarray, n0: int, weights: np.ndarray,
                 n_set: Optional[Sequence[int]] = None, coul64: bool = False) -> Dict[str, np.ndarray]:
    """Replay the steps [n0, n0 + len(weights)) from occ0 (not modified) and sum,
    per device, the score-function terms of every hop decision weighted by
    weights[k][d] (k = step - n0).  Returns grad, mag (sum of |term|) and sens
    (sum of |W g| p/(1-p)^2), each [D][4] over theta = (Ea shift, nu0, kappa,
    alpha), and the replayed final occupancy.  Also returned, as scales for
    the tolerance of a replay that sums the Coulomb part in another order:
    sens_arg and sens_b [D][4] (see orc_run_opts) and hops [D], the accepted
    hops.  coul64: in the binary32 path the score terms take the Coulomb part
    summed in binary64 and rounded once to binary32 (decisions unchanged)."""
    D = len(p.rails)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    n_steps = w.shape[0]
    if w.shape != (n_steps, D):
        raise ValueError("weights must be [n_steps][n_devices]")
    occ = np.ascontiguousarray(occ0, dtype=np.int8).reshape(-1).copy()
    prot = Protocols(protocols, n_set if n_set is not None else [0] * D)
    grad = np.zeros((D, 4))
    mag = np.zeros((D, 4))
    sens = np.zeros((D, 4))
    sens_arg = np.zeros((D, 4))
    sens_b = np.zeros((D, 4))
    hops = np.zeros(D, dtype=np.int64)
    opts = _Opts(0, 0, 0, _ptr(w, C.c_double), _ptr(grad, C.c_double), _ptr(mag, C.c_double),
                 _ptr(sens, C.c_double), _ptr(sens_arg, C.c_double), _ptr(sens_b, C.c_double),
                 _ptr(hops, C.c_int64), 1 if coul64 else 0)
    n_log = C.c_int64(0)
    rc = lib().orc_run(C.byref(p.s), prot.arr, _ptr(occ, C.c_int8), n0, n_steps, None, None, None,
                       None, 0, C.byref(n_log), C.byref(opts))
    if rc == -2:
        raise ValueError("score replay needs kappa != 0 and nu0 > 0")
    if rc != 0:
        raise ValueError("oracle rejected the run (step counter out of range)")
    return {"grad": grad, "mag": mag, "sens": sens, "sens_arg": sens_arg, "sens_b": sens_b, "hops": hops,
            "occ": occ}


# ---------------------------------------------------------------- zone model
class ZoneParams:
    """Parameters of the paper-literal zone model (kmc_oracle.h, orc_zone_params)."""

    def __init__(self, rails: int, ions: int, sites: int, zones: int = 10, p0: float = 0.5,
                 kT: float = 8.617333262e-5 * 300.0, hop_over_thickness: Optional[float] = None,
                 v_factor: float = 5e-5, dt: float = 1e-3, seed: int = 0):
        self.s = _ZoneParams(rails, ions, sites, zones, p0, kT,
                             1.0 / sites if hop_over_thickness is None else hop_over_thickness,
                             v_factor, dt, seed & 0xFFFFFFFFFFFFFFFF)
        self.rails, self.ions, self.sites, self.zones = rails, ions, sites, zones


def zone_index(x: int, sites: int, zones: int = 10) -> int:
    return int(lib().orc_zone_index(x, sites, zones))


def zone_table(p: ZoneParams, V: float, counts: Sequence[int]):
    """(p_left, p_right, dv_net) of every zone for bias V and zone populations."""
    c = np.ascontiguousarray(counts, dtype=np.int64)
    pl, pr, dv = (np.zeros(p.zones) for _ in range(3))
    lib().orc_zone_table(C.byref(p.s), V, _ptr(c, C.c_int64), _ptr(pl, C.c_double), _ptr(pr, C.c_double),
                         _ptr(dv, C.c_double))
    return pl, pr, dv


def zone_words(seed: int, rail: int, ion: int, n: int):
    wr, wl = C.c_uint32(0), C.c_uint32(0)
    lib().orc_zone_words(seed, rail, ion, n, C.byref(wr), C.byref(wl))
    return int(wr.value), int(wl.value)


def zone_positions(occ: np.ndarray, rails: int, sites: int) -> np.ndarray:
    """Ion-position matrix X [rails][ions] (1-based columns) of an occupancy
    [rails][sites] with the same ion count on every rail."""
    o = np.asarray(occ, dtype=np.int8).reshape(rails, sites)
    cols = [np.nonzero(r)[0] + 1 for r in o]
    if len({len(c) for c in cols}) != 1:
        raise ValueError("every rail needs the same ion count")
    return np.ascontiguousarray(np.array(cols, dtype=np.int32).reshape(rails, -1))


def zone_occupancy(X: np.ndarray, sites: int) -> np.ndarray:
    X = np.asarray(X)
    occ = np.zeros((X.shape[0], sites), dtype=np.int8)
    for i, row in enumerate(X):
        occ[i, row - 1] = 1
    return occ.reshape(-1)


def zone_run(p: ZoneParams, protocol, X: np.ndarray, n0: int, n_steps: int, n_set: int = 0):
    """Advance the ion-position matrix X [rails][ions] (modified in place) by
    n_steps steps from step n0.  Returns net [n], zones [n][Z] and the total."""
    Xc = np.ascontiguousarray(X, dtype=np.int32)
    if Xc.shape != (p.rails, p.ions):
        raise ValueError("X must be [rails][ions]")
    prot = Protocols([protocol], [n_set])
    net = np.zeros(n_steps, dtype=np.int32)
    zones = np.zeros((n_steps, p.zones), dtype=np.int32)
    tot = C.c_int64(0)
    rc = lib().orc_zone_run(C.byref(p.s), prot.arr, _ptr(Xc, C.c_int32), n0, n_steps, _ptr(net, C.c_int32),
                            _ptr(zones, C.c_int32), C.byref(tot))
    if rc != 0:
        raise ValueError("oracle rejected the run (step counter out of range)")
    if Xc is not X:
        X[...] = Xc
    return {"X": Xc, "net": net, "zones": zones, "net_total": int(tot.value)}
