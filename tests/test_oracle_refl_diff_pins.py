"""Pins of the oracle's paths with one reflection and one diffraction
(reflection then diffraction, type 3; diffraction then reflection, type 4).

On a box standing on a perfectly conducting ground (constant reflection
coefficient 1, whose field is a conductor's image), against:

* image theory: a reflection off the ground followed by diffraction at the
  box's vertical corner equals the plain diffraction of the transmitter's
  image below the ground, computed in the scene without ground (the same
  Keller point, length and complex gain); likewise a diffraction followed by
  a ground reflection equals the diffraction toward the receiver's image;
* reciprocity: the reflection-diffraction path from A to B and the
  diffraction-reflection path from B to A have the same gain;
* brute force: every (face, edge) combination that validates outside its
  margin is found by the transmitter-side launch (reflection first) or the
  receiver-side launch (diffraction first), and nothing invalid is.
"""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from synth import city
from tests.oracle_util import key_set, static_frame

FREQS = [3.5e9, 28e9]
CORNER = ((0.0, 40.0, 0.0), (0.0, 40.0, 30.0))  # vertical edge between the west and north walls
GROUND = 0


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


def _edge(os_, g, ends):
    for e in range(os_.E):
        p = g.edge_p[e]
        a, b = tuple(p[:3]), tuple(p[3:])
        if {a, b} == set(ends):
            return e
    raise AssertionError("edge not found")


def _eval_key(sc, key, tx, rx):
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    k = np.array([key], np.int32)
    valid, amb, _, pts = O.validate(os_, g, k, tx, rx)
    assert valid[0] and not amb[0]
    a, tau, fd, _, _ = O.evaluate(os_, g, k, pts, static_frame(tx, rx), FREQS)
    return a[0], tau[0], pts[0]


def _scenes():
    with_ground = city.tiny_box_ground(refl=(1.0, 1.0))
    box = dataclasses.replace(city.tiny_wedge(size=40.0, height=30.0), material_refl=np.array([1.0]))
    return with_ground, box


def test_reflection_then_diffraction_is_the_image_source_diffraction():
    a_sc, b_sc = _scenes()
    tx = np.array([[-30.0, 20.0, 2.0]])
    rx = np.array([[20.0, 70.0, 25.0]])
    oa, ob = O.OracleScene(a_sc), O.OracleScene(b_sc)
    ea = _edge(oa, oa.geometry(np.zeros((0, 3, 4))), CORNER)
    eb = _edge(ob, ob.geometry(np.zeros((0, 3, 4))), CORNER)
    amp, tau, pts = _eval_key(a_sc, [0, 0, 3, 2, GROUND, ea, -1, -1, -1], tx, rx)
    img = tx * np.array([1.0, 1.0, -1.0])
    amp_d, tau_d, pts_d = _eval_key(b_sc, [0, 0, 2, 1, eb, -1, -1, -1, -1], img, rx)
    assert abs(pts[0, 2]) < 1e-12  # reflection point on the ground
    np.testing.assert_allclose(pts[1], pts_d[0], rtol=0, atol=1e-9)  # same Keller point
    assert abs(tau - tau_d) <= 1e-12 * tau_d
    np.testing.assert_allclose(amp, amp_d, rtol=1e-10)


def test_diffraction_then_reflection_is_the_image_receiver_diffraction():
    a_sc, b_sc = _scenes()
    tx = np.array([[20.0, 70.0, 25.0]])
    rx = np.array([[-30.0, 20.0, 2.0]])
    oa, ob = O.OracleScene(a_sc), O.OracleScene(b_sc)
    ea = _edge(oa, oa.geometry(np.zeros((0, 3, 4))), CORNER)
    eb = _edge(ob, ob.geometry(np.zeros((0, 3, 4))), CORNER)
    amp, tau, pts = _eval_key(a_sc, [0, 0, 4, 2, ea, GROUND, -1, -1, -1], tx, rx)
    img = rx * np.array([1.0, 1.0, -1.0])
    amp_d, tau_d, pts_d = _eval_key(b_sc, [0, 0, 2, 1, eb, -1, -1, -1, -1], tx, img)
    assert abs(pts[1, 2]) < 1e-12
    np.testing.assert_allclose(pts[0], pts_d[0], rtol=0, atol=1e-9)
    assert abs(tau - tau_d) <= 1e-12 * tau_d
    np.testing.assert_allclose(amp, amp_d, rtol=1e-10)


def test_reciprocity_of_the_two_orders():
    a_sc, _ = _scenes()
    oa = O.OracleScene(a_sc)
    e = _edge(oa, oa.geometry(np.zeros((0, 3, 4))), CORNER)
    A = np.array([[-30.0, 20.0, 2.0]])
    B = np.array([[20.0, 70.0, 25.0]])
    a1, t1, _ = _eval_key(a_sc, [0, 0, 3, 2, GROUND, e, -1, -1, -1], A, B)
    a2, t2, _ = _eval_key(a_sc, [0, 0, 4, 2, e, GROUND, -1, -1, -1], B, A)
    assert abs(t1 - t2) <= 1e-12 * t1
    np.testing.assert_allclose(a1, a2, rtol=1e-9)


def test_brute_force_discovery_of_both_orders():
    sc = city.tiny_box_ground(refl=(0.8, 0.9))
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[-30.0, 20.0, 2.0]])
    xs = np.array([-20.0, 20.0, 60.0])
    rx = np.array([[x, y, z] for x in xs for y in (-20.0, 60.0, 75.0) for z in (1.5, 12.0, 25.0)
                   if not (0 <= x <= 40 and 0 <= y <= 40)])
    fr = static_frame(tx, rx)
    fwd = O.run_frame(os_, fr, 200000, 2, [28e9], diffraction=2, want_robust=False)
    bwd = O.run_frame(os_, fr, 200000, 2, [28e9], diffraction=2, want_robust=False,
                      rx_sources=list(range(len(rx))))
    rd = [[0, r, 3, 2, f, e, -1, -1, -1] for r in range(len(rx)) for f in range(os_.F) for e in range(os_.E)]
    dr = [[0, r, 4, 2, e, f, -1, -1, -1] for r in range(len(rx)) for f in range(os_.F) for e in range(os_.E)]
    for keys, found in ((np.array(rd, np.int32), fwd), (np.array(dr, np.int32), bwd)):
        valid, amb, _, _ = O.validate(os_, g, keys, tx, rx)
        brute = key_set(keys[valid & ~amb])
        typ = int(keys[0, 2])
        got = key_set(found.keys[found.keys[:, 2] == typ])
        assert len(brute) >= 5, typ
        assert got <= key_set(keys[valid])
        assert not (brute - got), (typ, sorted(brute - got))
