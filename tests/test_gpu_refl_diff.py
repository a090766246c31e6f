"""Paths with one reflection and one diffraction on the GPU (diffraction = 2)
against the oracle, through the C ABI.

* A box on a ground plane with receivers all round it: the transmitter-side
  step (reflection then diffraction) and the receiver-side step (diffraction
  then reflection) against the oracle's same launches -- path sets, per-path
  gain, delay and Doppler, channels.
* The toy city, transmitter side, with the first-order diffraction and the
  specular paths alongside.
* The adjoint over such paths: gradients against the oracle's central
  differences and dual numbers (the reflection face's permittivity enters them too).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from synth import city  # noqa: E402
from tests import parity as P  # noqa: E402
from tests.oracle_util import static_frame  # noqa: E402
from tests.test_gpu_backward_launch import _compare  # noqa: E402

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the first run of these tests ended in a GPU memory fault whose cause was not found; "
                            "diffraction = 2 is refused by emrt_ctx_create until it is"),
]


def _box_scene():
    tx = np.array([[-30.0, 20.0, 2.0]])
    rx = np.array([[x, y, z] for x in (-20.0, 20.0, 60.0) for y in (-20.0, 60.0, 75.0) for z in (1.5, 12.0, 25.0)
                   if not (0 <= x <= 40 and 0 <= y <= 40)])
    sc = city.with_static_rx(city.tiny_box_ground(refl=(0.0, 0.0)), rx)
    sc.tx_pos = tx
    return sc, tx, rx


def _tracer(sc, n_tx, n_rx, rays, K=2, **kw):
    from paper_2303_10521_amd import Tracer

    return Tracer(sc, n_tx, n_rx, freq_hz=[28e9], max_reflections=K, rays_per_tx=rays, diffraction=2,
                  path_capacity=1 << 16, **kw)


def test_box_on_ground_both_launch_sides():
    sc, tx, rx = _box_scene()
    fr = static_frame(tx, rx)
    os_ = O.OracleScene(sc)
    n = 200_000
    tr = _tracer(sc, 1, len(rx), n)
    tr.set_frame(fr)
    tr.step(True)
    assert tr.sync() == 0
    p = tr.flat_paths(cap=256)
    ref = O.run_frame(os_, fr, n, 2, [28e9], diffraction=2)
    assert (ref.keys[:, 2] == 3).sum() >= 5
    assert (p["key"][:, 2] == 3).sum() >= 5
    _compare(p, P.gpu_channels_np(tr.channels()), ref, os_, fr, len(rx))
    tr.close()
    # receiver side, from a fresh context (first step: no cache)
    per = n // len(rx)
    tr = _tracer(sc, 1, len(rx), n)
    tr.set_frame(fr)
    tr.step_rx(list(range(len(rx))), per)
    assert tr.sync() == 0
    p = tr.flat_paths(cap=256)
    ref = O.run_frame(os_, fr, per, 2, [28e9], diffraction=2, rx_sources=list(range(len(rx))))
    assert (ref.keys[:, 2] == 4).sum() >= 5
    assert (p["key"][:, 2] == 4).sum() >= 5
    _compare(p, P.gpu_channels_np(tr.channels()), ref, os_, fr, len(rx))
    tr.close()


def test_toy_city_with_combined_paths():
    w = city.workload("toy")
    sc = w.scene
    fr = sc.frame(0.0)
    os_ = O.OracleScene(sc)
    tr = _tracer(sc, sc.n_tx, sc.n_rx, 50_000, K=3)
    tr.set_frame(fr)
    tr.step(True)
    assert tr.sync() == 0
    p = tr.flat_paths(cap=256)
    ref = O.run_frame(os_, fr, 50_000, 3, [28e9], diffraction=2)
    assert (ref.keys[:, 2] == 3).any()
    _compare(p, P.gpu_channels_np(tr.channels()), ref, os_, fr, sc.n_tx * sc.n_rx)
    tr.close()


def test_adjoint_over_combined_paths():
    from tests.test_gpu_adjoint import _check, _cotangents, _link_mask, _oracle_grads

    sc, tx, rx = _box_scene()
    sc = city.with_static_rx(city.tiny_box_ground(refl=(0.0, 0.0)), rx)
    fr = static_frame(tx, rx)
    n = 200_000
    tr = _tracer(sc, 1, len(rx), n, adjoint_materials=2)
    tr.set_frame(fr)
    tr.step(True)
    assert tr.sync() == 0
    gk = tr.flat_paths(cap=256)["key"]
    assert (gk[:, 2] == 3).any()
    os_ = O.OracleScene(sc)
    ref = O.run_frame(os_, fr, n, 2, [28e9], diffraction=2)
    nl = len(rx)
    mask = _link_mask(gk, ref.keys, len(rx), nl)
    assert mask.mean() >= 0.9
    GH, GP = _cotangents(1, nl, 7, 1e6)
    GH[:, ~mask] = 0
    GP[:, ~mask] = 0
    g = tr.backward(torch.as_tensor(GH), torch.as_tensor(GP))
    wants = _oracle_grads(os_, os_.geometry(fr.obj_xform), fr, ref.keys, [28e9], GH, GP, len(rx))
    got = {k: v.cpu().numpy() for k, v in g.items()}
    _check(got, wants, ("grad_tx_pos", "grad_eps"))
    tr.close()
