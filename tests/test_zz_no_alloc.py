"""emrt_bind_static_workspace, the entry point for callers that cannot
allocate device memory, against emrt_bind_workspace with a caller buffer.

The same kernels run on the same inputs, so a discovery frame and a cached
frame give identical channels and path lists either way.  Two binds of the
static array in a row, the second with a smaller input, both match; sizes
beyond the static array are refused with the sizes named.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import city  # noqa: E402
from synth.city import Frame  # noqa: E402
from tests import parity as P  # noqa: E402

pytestmark = pytest.mark.gpu


def _subset(fr, n_rx):
    return Frame(t=fr.t, obj_xform=fr.obj_xform, obj_vel=fr.obj_vel, tx_pos=fr.tx_pos, tx_vel=fr.tx_vel,
                 rx_pos=fr.rx_pos[:n_rx], rx_vel=fr.rx_vel[:n_rx], tx_orient=fr.tx_orient)


def _run(sc, fr, static, **cfg):
    """A discovery frame then a cached frame; channels and path lists of both."""
    from paper_2303_10521_amd import Tracer

    before = torch.cuda.memory_allocated()
    tr = Tracer(sc, len(fr.tx_pos), len(fr.rx_pos), static_workspace=static, **cfg)
    grown = torch.cuda.memory_allocated() - before
    if static:
        assert tr.workspace is None
        assert grown < tr.workspace_bytes // 4  # only the scene arrays went through torch
    out = []
    for disc in (True, False):
        tr.set_frame(fr)
        tr.step(disc)
        assert tr.sync() == 0
        ch = P.gpu_channels_np(tr.channels())
        p = tr.flat_paths(cap=64)
        out.append((ch, p))
    nbytes = tr.workspace_bytes
    tr.close()
    return out, nbytes


def _same(a, b):
    for (ch_a, p_a), (ch_b, p_b) in zip(a, b):
        for k in ch_a:
            assert np.array_equal(ch_a[k], ch_b[k]), k
        for k in ("key", "tri_ids", "a", "tau", "fd", "angles"):
            assert np.array_equal(p_a[k], p_b[k]), k


def test_static_workspace_matches_caller_workspace_twice():
    from paper_2303_10521_amd import _abi as A

    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    cfg = dict(freq_hz=list(w.freqs_hz), max_reflections=w.max_reflections, rays_per_tx=w.rays_per_tx,
               path_capacity=1 << 16)
    ref1, n1 = _run(sc, fr, False, **cfg)
    got1, _ = _run(sc, fr, True, **cfg)
    _same(ref1, got1)
    assert len(got1[0][1]["key"]) > 50
    # the second bind, with a smaller input: 5 receivers, 4,000 rays, K = 2
    fr2 = _subset(fr, 5)
    cfg2 = dict(cfg, rays_per_tx=4000, max_reflections=2, path_capacity=1 << 12)
    ref2, n2 = _run(sc, fr2, False, **cfg2)
    got2, _ = _run(sc, fr2, True, **cfg2)
    _same(ref2, got2)
    assert n2 < n1 <= A.STATIC_WORKSPACE_BYTES
    assert len(got2[0][1]["key"]) > 5


def test_static_workspace_refuses_sizes_beyond_it():
    from paper_2303_10521_amd import Tracer
    from paper_2303_10521_amd import _abi as A
    from paper_2303_10521_amd.tracer import EmrtError

    w = city.workload("district")
    sc = w.scene
    with pytest.raises(EmrtError) as e:
        Tracer(sc, sc.n_tx, sc.n_rx, static_workspace=True, freq_hz=[28e9], max_reflections=4, rays_per_tx=1_000_000,
               diffraction=1, path_capacity=1 << 22)
    assert e.value.status == A.EMRT_E_WORKSPACE
    assert "static workspace holds" in str(e.value)
