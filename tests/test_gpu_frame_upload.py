"""Host-pointer frame upload (emrt_set_frame_host) against device-pointer frames
(emrt_set_frame).

Both entry points end in the same scatter into the workspace, so a context fed
host arrays and one fed the same values as device tensors must give
bit-identical channels and path lists over discovery and cached frames.  The
host arrays are read before the call returns: overwriting them straight after
the call changes nothing.  A null orientation array means zeros, and the
error cases match emrt_set_frame's.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import workload  # noqa: E402

pytestmark = pytest.mark.gpu


def _tracer(w):
    from paper_2303_10521_amd import Tracer

    sc = w.scene
    return Tracer(sc, sc.n_tx, sc.n_rx, freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections,
                  rays_per_tx=100_000, diffraction=int(w.diffraction), path_capacity=1 << 20)


def _snapshot(tr):
    ch = tr.channels()
    out = {k: ch[k].cpu().numpy().copy() for k in ("H", "P_coh", "P_inc", "tau_mean", "fd_mean", "n_paths")}
    p = tr.flat_paths(cap=64)
    out["keys"] = p["key"].copy()
    out["a"] = p["a"].copy()
    out["fd"] = p["fd"].copy()
    return out


def _on_device(fr):
    class F:
        pass

    g = F()
    g.t = fr.t
    for k in ("obj_xform", "obj_vel", "tx_pos", "tx_vel", "tx_orient", "rx_pos", "rx_vel"):
        setattr(g, k, torch.as_tensor(np.asarray(getattr(fr, k), np.float64), device="cuda"))
    return g


def _host_desc(tr, fr, frame, orient=True):
    from paper_2303_10521_amd import _abi as A

    arrs = [np.array(getattr(fr, k), np.float64, order="C", copy=True)  # own copies: the test overwrites them
            for k in ("obj_xform", "obj_vel", "tx_pos", "tx_vel", "tx_orient", "rx_pos", "rx_vel")]
    ptrs = [a.ctypes.data for a in arrs]
    if not orient:
        ptrs[4] = None
    return A.FrameDesc(frame, float(fr.t), tr.n_tx, tr.n_rx, *ptrs), arrs


def test_host_frames_equal_device_frames():
    w = workload("district")
    sc = w.scene
    host, dev = _tracer(w), _tracer(w)
    try:
        times = [0.0, 0.01, 0.02, 0.5]
        discover = [True, False, True, False]
        for f, (t, d) in enumerate(zip(times, discover)):
            fr = sc.frame(t)
            desc, arrs = _host_desc(host, fr, f)
            assert host.lib.emrt_set_frame_host(host.ctx, ctypes.byref(desc)) == 0
            for a in arrs:  # the call has copied them
                a[...] = np.nan
            host.step(d)
            dev.set_frame(_on_device(fr), f)
            dev.step(d)
            assert host.sync() == 0 and dev.sync() == 0
            a, b = _snapshot(host), _snapshot(dev)
            assert a["keys"].shape[0] > 0
            for k in a:
                assert np.array_equal(a[k], b[k]), (f, k)
    finally:
        host.close()
        dev.close()


def test_binding_uses_the_host_entry_for_numpy_frames():
    w = workload("toy")
    sc = w.scene
    a, b = _tracer(w), _tracer(w)
    try:
        fr = sc.frame(0.0)
        a.set_frame(fr, 0)  # numpy arrays: emrt_set_frame_host
        b.set_frame(_on_device(fr), 0)
        for tr in (a, b):
            tr.step(True)
            tr.sync()
        x, y = _snapshot(a), _snapshot(b)
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    finally:
        a.close()
        b.close()


def test_null_orientation_is_zeros():
    w = workload("toy")
    sc = w.scene
    a, b = _tracer(w), _tracer(w)
    try:
        fr = sc.frame(0.0)
        fr.tx_orient = np.zeros_like(np.asarray(fr.tx_orient, np.float64))
        d0, _ = _host_desc(a, fr, 0, orient=False)
        assert a.lib.emrt_set_frame_host(a.ctx, ctypes.byref(d0)) == 0
        b.set_frame(_on_device(fr), 0)
        for tr in (a, b):
            tr.step(True)
            tr.sync()
        x, y = _snapshot(a), _snapshot(b)
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    finally:
        a.close()
        b.close()


def test_host_frame_errors():
    w = workload("toy")
    sc = w.scene
    tr = _tracer(w)
    try:
        fr = sc.frame(0.0)
        d, arrs = _host_desc(tr, fr, 0)
        d.n_rx = tr.n_rx + 1
        assert tr.lib.emrt_set_frame_host(tr.ctx, ctypes.byref(d)) == -1  # EMRT_E_INVALID
        d, arrs = _host_desc(tr, fr, 0)
        d.rx_pos = None
        assert tr.lib.emrt_set_frame_host(tr.ctx, ctypes.byref(d)) == -1
        assert tr.lib.emrt_set_frame_host(tr.ctx, None) == -1
        d, arrs = _host_desc(tr, fr, 0)
        assert tr.lib.emrt_set_frame_host(tr.ctx, ctypes.byref(d)) == 0
        tr.step(True)
        assert tr.sync() == 0
    finally:
        tr.close()
