"""The C ABI library: it loads, exports every function include/kmc.h declares,
and validates parameters on the host before touching a GPU (CPU only)."""
import ctypes as C
import os
import re

import pytest

import paper_2511_09413_amd as kmc
from workloads import Physics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:kmc_status|const char \*|void)\s*\**\s*(kmc_\w+)\s*\(", text, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "kmc_init_device" in names and "kmc_run_steps" in names and len(names) >= 12
    L = kmc.lib()
    for n in names:
        assert hasattr(L, n), n


def _status(physics, rails, sites):
    p, keep = kmc.make_params(physics, rails, sites)
    out = C.c_size_t(0)
    return kmc.lib().kmc_workspace_bytes(C.byref(p), C.byref(out)), out.value


def test_validation_errors_without_gpu():
    ok, nbytes = _status(Physics(), [64], [128])
    assert ok == kmc.KMC_OK and nbytes > 2 * 64 * 128
    assert _status(Physics(), [64], [1])[0] == kmc.KMC_EINVAL
    assert _status(Physics(), [0], [8])[0] == kmc.KMC_EINVAL
    assert _status(Physics(), [4], [5000])[0] == kmc.KMC_EUNSUPPORTED
    assert _status(Physics(kT_ev=0.0), [4], [8])[0] == kmc.KMC_EINVAL
    assert _status(Physics(dt_s=-1.0), [4], [8])[0] == kmc.KMC_EINVAL
    assert _status(Physics(rail_range=5), [4], [8])[0] == kmc.KMC_EUNSUPPORTED
    assert _status(Physics(cutoff_sites=-1), [4], [8])[0] == kmc.KMC_EINVAL
    assert b"cutoff" in kmc.lib().kmc_last_error()
    with pytest.raises(kmc.KmcError):
        kmc.workspace_bytes(kmc.make_params(Physics(screening_sites=-1.0), [4], [8])[0])


def test_workspace_scales_with_lattice():
    a = _status(Physics(), [64], [128])[1]
    b = _status(Physics(), [4096], [1024])[1]
    assert b > 2 * 4096 * 1024 and 16 * a < b


def test_workspace_holds_the_replay_buffers():
    """Outside the dense precision the workspace holds the score replay's
    per-bond Coulomb parts (one value of the path precision per site) and its
    hop list (16 bytes per entry, at least 4096 entries)."""
    from workloads import FP32, FP64
    for prec, size in ((FP32, 4), (FP64, 8)):
        small = _status(Physics(precision=prec), [64], [128])[1]
        large = _status(Physics(precision=prec), [4096], [1024])[1]
        n_small, n_large = 64 * 128, 4096 * 1024
        assert large - small >= size * (n_large - n_small)
        assert small >= size * n_small + 16 * 4096


def test_native_decay_fit_matches_the_oracle_fit():
    """kmc_fit_decay (host arithmetic in the library, parameterised by the
    decay rate) against the oracle's Gauss-Newton fit in (C, A, tau): the same
    least-squares minimum and the same implicit-function weights, on a
    noise-free curve (exact recovery) and on noisy curves."""
    import numpy as np
    from oracle import relaxation as rx
    t0 = 3e-9
    t = np.linspace(t0, t0 + 30e-9, 500)
    exact = rx.decay_model(t, t0, 0.22, 0.31, 5e-9)
    (c, a, tau), w = kmc.fit_decay(t, exact, t0)
    assert abs(tau - 5e-9) <= 1e-9 * 5e-9 and abs(c - 0.22) <= 1e-9 and abs(a - 0.31) <= 1e-9
    for seed in range(4):
        m = exact + np.random.default_rng(seed).normal(0.0, 0.02, len(t))
        ref, _ = rx.fit_decay(t, m, t0)
        w_ref = rx.tau_weights(t, m, t0, ref)
        got, w = kmc.fit_decay(t, m, t0)
        assert np.allclose(got, ref, rtol=1e-9, atol=0.0), (got, ref)
        assert np.abs(w - w_ref).max() <= 1e-8 * np.abs(w_ref).max()
        # a starting point is used, and gives the same minimum
        again, _ = kmc.fit_decay(t, m, t0, start=(0.1, 0.5, 2e-9), weights=False)
        assert np.allclose(again, ref, rtol=1e-9, atol=0.0)


def test_native_decay_fit_errors():
    import numpy as np
    t = np.linspace(0.0, 1.0, 10)
    with pytest.raises(kmc.KmcError) as e:
        kmc.fit_decay(t[:3], t[:3], 0.0)
    assert e.value.status == kmc.KMC_EINVAL
    with pytest.raises(kmc.KmcError):
        kmc.fit_decay(np.zeros(10), t, 0.0)            # every time equals t0
    bad = t.copy()
    bad[4] = np.nan
    with pytest.raises(kmc.KmcError):
        kmc.fit_decay(t, bad, 0.0)
    with pytest.raises(kmc.KmcError) as e:
        kmc.fit_decay(t, np.full(10, 0.3), 0.0)       # a flat curve has no decay time
    assert e.value.status in (kmc.KMC_EUNSUPPORTED, kmc.KMC_EINVAL)
