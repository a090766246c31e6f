"""Pins of the coherence statistics oracle (Section III-B, Eq (1), Eq (2)).

* Eq (2): a value worked by hand for the paper's formula as printed, and the
  dependence it fixes (T_c ~ 1 / (f_D theta^2), T_c -> 0 as R -> 1).
* Eq (1) (read as the normalised autocovariance of g = |h|): closed forms for
  a cosine, R(k) -> cos(w k), and for an AR(1) process, R(k) -> rho^k.
* Spatial-consistency triggers: receivers moving past a box building; the
  frame where the line of sight appears and the frame where a reflection
  leaves the face follow from the geometry in closed form.
"""
import math

import numpy as np
import pytest

from oracle import coherence as Co
from oracle import oracle as O
from synth import city
from tests.oracle_util import spec_key


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


def test_coherence_time_worked_value():
    # R = 0.5, f_c = 28 GHz, |v| = 10 m/s, theta = 0.2 rad:
    # f_D = 28e9 * 10 / 299792458 = 933.96 Hz; sqrt(1/R^4 - 1) = sqrt(15) = 3.8730;
    # T_c = 3.8730 / (2 pi * 933.96 * 0.04) = 0.016500 s
    v = np.array([[10.0, 0.0, 0.0]])
    k = np.array([[math.cos(0.2), math.sin(0.2), 0.0]])
    tc = Co.coherence_time(0.5, 28e9, v, k)[0]
    assert abs(tc - 0.016500) < 2e-6


def test_coherence_time_dependences():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(50, 3)) * 5
    k = rng.normal(size=(50, 3))
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    base = Co.coherence_time(0.5, 28e9, v, k)
    assert np.allclose(Co.coherence_time(0.5, 28e9, 2 * v, k), base / 2, rtol=1e-12)  # 1 / f_D
    assert np.allclose(Co.coherence_time(0.5, 3.5e9, v, k), base * 8, rtol=1e-12)  # 1 / f_c
    assert np.allclose(Co.coherence_time(0.5, 28e9, -v, k), base, rtol=1e-12)  # line of motion only
    assert np.all(Co.coherence_time(0.999999, 28e9, v, k) < 1e-3 * base)  # R -> 1
    assert np.all(np.isinf(Co.coherence_time(0.5, 28e9, np.zeros((3, 3)), k[:3])))  # no motion
    # small angles: theta^-2
    for th in (0.01, 0.02, 0.04):
        kk = np.array([[math.cos(th), math.sin(th), 0.0]])
        t = Co.coherence_time(0.5, 28e9, np.array([[10.0, 0, 0]]), kk)[0]
        assert abs(t * th * th - 3.8729833 / (2 * math.pi * 933.9589)) < 1e-6


def test_autocovariance_of_a_cosine():
    w = 2 * math.pi / 50.0
    t = np.arange(200000)
    g = 2.0 + np.cos(w * t + 0.3)
    r = Co.autocovariance(g, [1, 2, 5, 12, 25])
    assert np.allclose(r, np.cos(w * np.array([1, 2, 5, 12, 25])), atol=2e-3)


def test_autocovariance_of_ar1():
    rng = np.random.default_rng(1)
    rho, n = 0.8, 400000
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0] / math.sqrt(1 - rho * rho)
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    g = 5.0 + x
    r = Co.autocovariance(g, [1, 2, 3, 4])
    assert np.allclose(r, rho ** np.array([1, 2, 3, 4]), atol=1e-2)
    assert np.all(np.isnan(Co.autocovariance(g[:3], [3, 4])))


def _box_scene():
    return city.tiny_wedge(size=40.0, height=30.0, eps=city.EPS_CONCRETE)


def test_line_of_sight_trigger_at_the_frame_it_appears():
    """Tx (-50, 20, 10) west of the box [0,40]^2 x [0,30]; Rx at x = 100,
    z = 1.5, y = 70.5 + t: the sight line clears the box iff it passes north
    of both x = 0 and x = 40, i.e. y > 80, first at t = 10."""
    sc = _box_scene()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[-50.0, 20.0, 10.0]])
    los_prev, sets_prev, fired = None, None, []
    for t in range(16):
        rx = np.array([[100.0, 70.5 + t, 1.5]])
        valid, amb, _, _ = O.validate(os_, g, np.array([spec_key(0, 0, [])]), tx, rx)
        assert not amb[0]
        los = np.array([bool(valid[0])])
        sets = [frozenset()]
        trig = Co.triggers(los_prev, los, sets_prev, sets)
        fired.append(int(trig[0]))
        los_prev, sets_prev = los, sets
    assert fired == [0] * 10 + [1] + [0] * 5


def test_first_order_set_trigger_when_a_reflection_leaves_the_face():
    """Tx (-50, 20, 10) and Rx (-30, y, 1.5) west of the box: the reflection
    point on the face x = 0 is at y_s = 0.625 y + 7.5, inside the face for
    y <= 52; with y = 45.5 + t it leaves at t = 7."""
    sc = _box_scene()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[-50.0, 20.0, 10.0]])
    face_keys = np.array([spec_key(0, 0, [f]) for f in range(os_.F)], np.int32)
    los_prev, sets_prev, fired = None, None, []
    for t in range(12):
        rx = np.array([[-30.0, 45.5 + t, 1.5]])
        valid, amb, _, _ = O.validate(os_, g, face_keys, tx, rx)
        assert not amb.any()
        keys = face_keys[valid]
        sets = Co.first_order_sets(keys, 1, 1)
        lv, _, _, _ = O.validate(os_, g, np.array([spec_key(0, 0, [])]), tx, rx)
        los = np.array([bool(lv[0])])
        trig = Co.triggers(los_prev, los, sets_prev, sets)
        fired.append(int(trig[0]))
        los_prev, sets_prev = los, sets
    assert fired == [0] * 7 + [2] + [0] * 4
