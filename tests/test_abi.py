"""The C ABI library loads and exports every declared entry point; host-side
argument and state checks work without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2303_10521_amd import _abi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emrt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(emrt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.fail("libemrt.so is not built (run __graft_entry__.build())")
    return A.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(A.SIGNATURES), "ctypes signatures and header disagree"


def _cfg(lib, **kw):
    c = A.Config()
    lib.emrt_config_default(ctypes.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_config_defaults(lib):
    c = _cfg(lib)
    assert c.n_freq == 1 and c.freq_hz[0] == 28e9 and c.max_reflections == 3
    assert c.tx_power_w == 100.0 and c.rx_sphere_k == 1.0 and c.diff_max_leg_m == 250.0
    assert c.ray_regroup == 0 and c.dyn_rebuild_ratio == 0.0


@pytest.mark.parametrize("kw,status", [
    (dict(max_reflections=6), A.EMRT_E_UNSUPPORTED),
    (dict(n_freq=0), A.EMRT_E_UNSUPPORTED),
    (dict(n_freq=5), A.EMRT_E_UNSUPPORTED),
    (dict(rays_per_tx=0), A.EMRT_E_INVALID),
    (dict(rx_sphere_k=0.0), A.EMRT_E_INVALID),
    (dict(path_capacity=0), A.EMRT_E_INVALID),
    (dict(antenna_mode=7), A.EMRT_E_INVALID),
    (dict(diffraction=3), A.EMRT_E_INVALID),
    (dict(diffraction=2), A.EMRT_E_UNSUPPORTED),
    (dict(ray_regroup=2), A.EMRT_E_INVALID),
    (dict(ray_regroup=-1), A.EMRT_E_INVALID),
    (dict(dyn_rebuild_ratio=-1.0), A.EMRT_E_INVALID),
    (dict(dyn_rebuild_ratio=float("nan")), A.EMRT_E_INVALID),
])
def test_ctx_create_rejects_bad_config(lib, kw, status):
    c = _cfg(lib, **kw)
    ctx = ctypes.c_void_p()
    assert lib.emrt_ctx_create(ctypes.byref(c), ctypes.byref(ctx)) == status
    assert not ctx.value


def test_workspace_and_state_checks(lib):
    c = _cfg(lib, rays_per_tx=1000)
    ctx = ctypes.c_void_p()
    assert lib.emrt_ctx_create(ctypes.byref(c), ctypes.byref(ctx)) == A.EMRT_OK
    try:
        # order: bind before sizing, step before scene
        assert lib.emrt_bind_workspace(ctx, ctypes.c_void_p(4096), 1 << 20) == A.EMRT_E_STATE
        assert lib.emrt_step(ctx, 1) == A.EMRT_E_STATE
        bad = A.Sizes(3, 1, 1, 1, 0, 1)
        nbytes = ctypes.c_size_t()
        assert lib.emrt_workspace_size(ctx, ctypes.byref(bad), ctypes.byref(nbytes)) == A.EMRT_E_INVALID
        big = A.Sizes(3, 1, 1, 1, 5000, 1)
        assert lib.emrt_workspace_size(ctx, ctypes.byref(big), ctypes.byref(nbytes)) == A.EMRT_E_UNSUPPORTED
        ok = A.Sizes(8, 4, 2, 1, 2, 3)
        assert lib.emrt_workspace_size(ctx, ctypes.byref(ok), ctypes.byref(nbytes)) == A.EMRT_OK
        assert nbytes.value > 2 * 1000 * 36  # at least the two ray buffers
        assert lib.emrt_bind_workspace(ctx, None, nbytes.value) == A.EMRT_E_WORKSPACE
        assert lib.emrt_bind_workspace(ctx, ctypes.c_void_p(4096), 1024) == A.EMRT_E_WORKSPACE
        buf = ctypes.create_string_buffer(256)
        assert lib.emrt_last_error(ctx, buf, 256) == A.EMRT_OK
        assert b"small" in buf.value
        assert lib.emrt_read_channels(ctx, None) == A.EMRT_E_INVALID
        refl = (ctypes.c_double * 2)(0.8, 0.9)
        assert lib.emrt_set_reflection_coefficients(ctx, None, 2) == A.EMRT_E_INVALID
        assert lib.emrt_set_reflection_coefficients(ctx, refl, 2) == A.EMRT_E_STATE  # no scene yet
        ids = (ctypes.c_int32 * 2)(0, 1)
        assert lib.emrt_step_rx(ctx, ids, 2, 100) == A.EMRT_E_STATE  # no scene yet
    finally:
        assert lib.emrt_ctx_destroy(ctx) == A.EMRT_OK


def test_status_strings(lib):
    for s in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert lib.emrt_status_string(s)
    assert lib.emrt_status_string(-99) == b"unknown status"
