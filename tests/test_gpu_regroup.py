"""Regrouping of the rays between bounces (emrt_config.ray_regroup).

The rays entering bounces 2..K are sorted by origin cell and direction octant
before they are traced.  A ray's hits, captures and reflections do not depend
on where in the live buffer it sits, so a context that regroups and one that
keeps the append order must give bit-identical channels, path lists and
per-bounce ray counts, on discovery and cached frames, on the transmitter-side
launch and on a receiver-side launch.  The city parity test also runs its
full-size frame regrouped against the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import workload  # noqa: E402

pytestmark = pytest.mark.gpu


def _tracer(w, regroup, **kw):
    from paper_2303_10521_amd import Tracer

    sc = w.scene
    args = dict(freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=kw.pop("rays", 200_000),
                diffraction=int(w.diffraction), path_capacity=1 << 20, ray_regroup=regroup)
    args.update(kw)
    return Tracer(sc, sc.n_tx, sc.n_rx, **args)


def _snapshot(tr):
    ch = tr.channels()
    out = {k: ch[k].cpu().numpy().copy() for k in ("H", "P_coh", "P_inc", "tau_mean", "tau_rms", "fd_mean", "n_paths")}
    p = tr.flat_paths(cap=64)
    out["keys"] = p["key"].copy()
    out["a"] = p["a"].copy()
    out["rays"] = np.array(tr.stats()["rays_per_bounce"])
    return out


def _equal(a, b, what):
    for k in a:
        assert a[k].shape == b[k].shape, (what, k)
        assert np.array_equal(a[k], b[k]), (what, k)


@pytest.mark.parametrize("name", ["district", "toy"])
def test_regroup_gives_the_same_results(name):
    w = workload(name)
    sc = w.scene
    on, off = _tracer(w, 1), _tracer(w, 0)
    try:
        assert w.max_reflections >= 2
        for f, discover in enumerate((True, False, True)):
            fr = sc.frame(f * w.frame_dt * 3)
            for tr in (on, off):
                tr.set_frame(fr, f)
                tr.step(discover)
                tr.sync()
            a, b = _snapshot(on), _snapshot(off)
            if discover:
                assert a["rays"][2] > 0  # bounces that were regrouped
            _equal(a, b, (name, f))
        # a receiver-side launch
        rx = list(range(4))  # 4 x 50,000 rays: within the launch capacity of both workloads
        for tr in (on, off):
            tr.step_rx(rx, 50_000)
            tr.sync()
        _equal(_snapshot(on), _snapshot(off), (name, "rx"))
    finally:
        on.close()
        off.close()
