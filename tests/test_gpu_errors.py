"""Context-level errors through the C ABI leave the state untouched (needs an
MI355X).

Every rejected call below is made on a context that has already run; the
context then runs on, and its trajectory must equal that of a twin context
that never saw the bad calls (same seed, same start, same protocol).  A
poisoned context (a neighbour wait declared hung from the host, as in the
failure-path test) answers every later call with KMC_ESTATE."""
import ctypes as C

import numpy as np
import pytest

import oracle
from parity_util import gpu_available
from workloads import c1_plain_fp64

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PD = C.POINTER(C.c_double)


def _arr(x):
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a, a.ctypes.data_as(PD)


def _pair(ea=0.15):
    from paper_2511_09413_amd import Simulator
    wl = c1_plain_fp64()
    ph = wl.physics.replace(ea_ev=ea)
    p_or = oracle.OracleParams(ph, wl.rails, wl.sites)
    occ0 = oracle.fill(p_or, wl.filling)
    sims = []
    for _ in range(2):
        s = Simulator(ph, wl.rails, wl.sites)
        s.load_occupancy(occ0)
        s.set_protocols(wl.protocols)
        s.run_steps(30)
        sims.append(s)
    return sims, wl


def _same_future(a, b, steps=60):
    na, da = a.run_steps(steps, tallies=True)
    nb, db = b.run_steps(steps, tallies=True)
    assert a.step == b.step
    assert np.array_equal(na.cpu().numpy(), nb.cpu().numpy())
    assert np.array_equal(da.cpu().numpy(), db.cpu().numpy())
    assert np.array_equal(a.read_occupancy(), b.read_occupancy())
    ca, ta, tta = a.read_current()
    cb, tb, ttb = b.read_current()
    assert np.array_equal(ta, tb) and tta == ttb


def test_rejected_calls_leave_the_state_untouched():
    from paper_2511_09413_amd import (KMC_EINVAL, KMC_ETOOSMALL, KMC_EUNSUPPORTED, lib)
    (sim, twin), wl = _pair()
    L = lib()
    ctx = C.c_void_p(sim.ctx)
    step_before = sim.step
    occ_before = sim.read_occupancy()
    expect = []

    t, tp = _arr([0.0, 2e-12, 1e-12])                # unsorted knot times
    v, vp = _arr([0.0, 1.0, 2.0])
    expect.append((L.kmc_set_bias_protocol(ctx, -1, tp, vp, 3), KMC_EINVAL))
    t0, tp0 = _arr([0.0])
    v0, vp0 = _arr([3.0])
    expect.append((L.kmc_set_bias_protocol(ctx, -1, tp0, vp0, 0), KMC_EINVAL))      # no knots
    t65, tp65 = _arr(np.arange(65) * 1e-12)
    v65, vp65 = _arr(np.ones(65))
    expect.append((L.kmc_set_bias_protocol(ctx, -1, tp65, vp65, 65), KMC_EINVAL))  # 65 knots
    expect.append((L.kmc_set_bias_protocol(ctx, 1, tp0, vp0, 1), KMC_EINVAL))      # device 1 of 1
    expect.append((L.kmc_set_bias_protocol(ctx, -1, None, vp0, 1), KMC_EINVAL))
    tn, tpn = _arr([0.0, np.nan])
    expect.append((L.kmc_set_bias_protocol(ctx, -1, tpn, vp, 2), KMC_EINVAL))             # NaN knot
    expect.append((L.kmc_run_steps(ctx, -1, None, None), KMC_EINVAL))
    expect.append((L.kmc_run_steps(ctx, 1 << 33, None, None), KMC_EUNSUPPORTED))
    f, fp = _arr([1.5])
    expect.append((L.kmc_fill_random(ctx, fp), KMC_EINVAL))
    expect.append((L.kmc_fill_random(ctx, None), KMC_EINVAL))
    small = np.zeros(sim.n_sites - 1, dtype=np.int8)
    expect.append((L.kmc_read_occupancy(ctx, C.c_void_p(small.ctypes.data), small.size), KMC_ETOOSMALL))
    expect.append((L.kmc_read_occupancy(ctx, None, sim.n_sites), KMC_EINVAL))
    n_ev = C.c_int64(0)
    expect.append((L.kmc_read_threshold_log(ctx, None, -1, C.byref(n_ev)), KMC_EINVAL))
    expect.append((L.kmc_read_threshold_log(ctx, None, 4, C.byref(n_ev)), KMC_EINVAL))
    expect.append((L.kmc_set_launch_mode(ctx, 7), KMC_EINVAL))
    w = sim.torch.zeros((4, 1), dtype=sim.torch.float64, device=sim.device)
    g = sim.torch.zeros((1, 4), dtype=sim.torch.float64, device=sim.device)
    expect.append((L.kmc_score_replay(ctx, None, 0, 4, C.c_void_p(w.data_ptr()), C.c_void_p(g.data_ptr())),
                   KMC_EINVAL))
    expect.append((L.kmc_score_replay(ctx, C.c_void_p(sim.occ.data_ptr()), 0, -2, C.c_void_p(w.data_ptr()),
                                      C.c_void_p(g.data_ptr())), KMC_EINVAL))
    for i, (got, want) in enumerate(expect):
        assert got == want, (i, got, want, L.kmc_last_error().decode())
        assert L.kmc_last_error().decode() != ""
    assert sim.step == step_before
    assert np.array_equal(sim.read_occupancy(), occ_before)
    _same_future(sim, twin)
    sim.close()
    twin.close()


def test_small_workspace_and_bad_arguments_at_init():
    from paper_2511_09413_amd import KMC_EINVAL, KMC_ETOOSMALL, lib, make_params, workspace_bytes
    import torch
    wl = c1_plain_fp64()
    params, keep = make_params(wl.physics, wl.rails, wl.sites)
    need = workspace_bytes(params)
    occ = torch.zeros(wl.rails[0] * wl.sites[0], dtype=torch.int8, device="cuda:0")
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda:0")
    base = (ws.data_ptr() + 255) // 256 * 256
    L = lib()
    h = C.c_void_p(0)
    st = torch.cuda.current_stream().cuda_stream
    assert L.kmc_init_device(C.byref(params), C.c_void_p(occ.data_ptr()), None, C.c_void_p(base), need - 1,
                             C.c_void_p(st), C.byref(h)) == KMC_ETOOSMALL
    assert "workspace too small" in L.kmc_last_error().decode()
    assert L.kmc_init_device(C.byref(params), C.c_void_p(occ.data_ptr()), None, C.c_void_p(base + 8), need,
                             C.c_void_p(st), C.byref(h)) == KMC_EINVAL
    assert L.kmc_init_device(C.byref(params), None, None, C.c_void_p(base), need, C.c_void_p(st),
                             C.byref(h)) == KMC_EINVAL
    assert h.value is None
    # the same buffers then work
    assert L.kmc_init_device(C.byref(params), C.c_void_p(occ.data_ptr()), None, C.c_void_p(base), need,
                             C.c_void_p(st), C.byref(h)) == 0
    L.kmc_destroy(h)


def test_poisoned_context_answers_estate():
    """After the hung-wait failure (forced from the host with a wait limit of
    0, so every kernel still exits normally) every call on the context
    returns KMC_ESTATE; destroying it is still allowed."""
    from paper_2511_09413_amd import (KMC_EHIP, KMC_ESTATE, KmcError, Simulator, lib)
    wl = c1_plain_fp64()
    ph = wl.physics.replace(ea_ev=0.15)
    sim = Simulator(ph, wl.rails, wl.sites, mode="wave")
    p_or = oracle.OracleParams(ph, wl.rails, wl.sites)
    sim.load_occupancy(oracle.fill(p_or, wl.filling))
    sim.set_protocols(wl.protocols)
    sim.set_wait_limit(0)
    sim.run_steps(50)
    with pytest.raises(KmcError) as err:
        sim.read_current()
    assert err.value.status == KMC_EHIP
    L = lib()
    ctx = C.c_void_p(sim.ctx)
    t, tp = _arr([0.0])
    out = np.zeros(sim.n_sites, dtype=np.int8)
    calls = [
        L.kmc_run_steps(ctx, 1, None, None),
        L.kmc_read_occupancy(ctx, C.c_void_p(out.ctypes.data), out.size),
        L.kmc_read_current(ctx, None, None, None),
        L.kmc_set_bias_protocol(ctx, -1, tp, tp, 1),
        L.kmc_load_occupancy(ctx),
        L.kmc_set_launch_mode(ctx, 0),
    ]
    assert calls == [KMC_ESTATE] * len(calls), calls
    assert "poisoned" in L.kmc_last_error().decode()
    sim.close()


def test_zone_rejected_calls_leave_the_state_untouched():
    from paper_2511_09413_amd import KMC_EINVAL, KMC_ETOOSMALL, KmcError, ZoneSimulator, lib
    from workloads import zone_positions
    rails, sites, ions = 96, 40, 12
    X0 = zone_positions(rails, sites, ions, seed=4)
    occ = np.zeros((rails, sites), dtype=np.int8)
    for r in range(rails):
        occ[r, X0[r] - 1] = 1
    sims = [ZoneSimulator(rails, sites, ions, p0=0.6, v_factor=2e-3, seed=9, occ=occ) for _ in range(2)]
    for s in sims:
        s.set_bias_protocol([0.0, 1.0], [2.0, -2.0])
        s.run_steps(10)
    sim, twin = sims
    L = lib()
    ctx = C.c_void_p(sim.ctx)
    X_before = sim.read_positions()
    t, tp = _arr([0.0, 2.0, 1.0])
    v, vp = _arr([0.0, 1.0, 2.0])
    assert L.kmc_zone_set_bias_protocol(ctx, tp, vp, 3) == KMC_EINVAL
    assert L.kmc_zone_set_bias_protocol(ctx, tp, vp, 0) == KMC_EINVAL
    assert L.kmc_zone_run_steps(ctx, -3, None, None) == KMC_EINVAL
    small = np.zeros(rails * ions - 1, dtype=np.int32)
    assert L.kmc_zone_read_positions(ctx, small.ctypes.data_as(C.POINTER(C.c_int32)), small.size) == KMC_ETOOSMALL
    bad = occ.copy()
    bad[5, :] = 0                                  # a rail without its ions
    with pytest.raises(KmcError) as err:
        sim.load_occupancy(bad)
    assert err.value.status == KMC_EINVAL
    assert sim.step == twin.step == 10
    assert np.array_equal(sim.read_positions(), X_before)
    na, za = sim.run_steps(40, tallies=True)
    nb, zb = twin.run_steps(40, tallies=True)
    assert np.array_equal(na.cpu().numpy(), nb.cpu().numpy())
    assert np.array_equal(za.cpu().numpy(), zb.cpu().numpy())
    assert np.array_equal(sim.read_positions(), twin.read_positions())
    assert np.array_equal(sim.read_occupancy(), twin.read_occupancy())
    sim.close()
    twin.close()
