"""Pins of the oracle outputs that the first pin suite left open: the RMS
delay spread, the departure and arrival angles, rotated object transforms,
and the frame-to-frame bookkeeping of the path cache.

Each is checked against a value worked out by hand or a closed form of the
geometry, not against the oracle's own formula:
  * tau_rms of two paths with powers 3:1 is sqrt(3)/4 |tau_1 - tau_2|;
  * the line of sight and the ground bounce leave and arrive at the angles
    of the transmitter-receiver (or image-receiver) direction;
  * a 90 degree yaw maps local vertices to hand-computed float32 points (a
    transposed rotation maps them elsewhere), and a wall placed by that
    transform reflects with the image length of its world plane;
  * a cached frame keeps exactly the cached keys that still validate, and a
    discovery frame keeps the valid keys of the cache together with the
    newly discovered ones (the cache / "visibility hash table" with deletion,
    Section III-B).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from synth import city
from tests.oracle_util import C0, key_set, spec_key, static_frame

F28 = 28e9


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


# --------------------------------------------------------------------------
# RMS delay spread
# --------------------------------------------------------------------------

def test_rms_delay_spread_by_hand():
    """Two paths, powers 3:1 at the first carrier and 1:1 at the second,
    delays 1 and 2 us: mean 1.25 / 1.5 us, RMS spread sqrt(3)/4 / 1/2 us."""
    keys = np.array([spec_key(0, 0, []), spec_key(0, 0, [3])], np.int32)
    a = np.array([[math.sqrt(3.0), 1.0], [1.0j, -1.0]])
    tau = np.array([1e-6, 2e-6])
    fd = np.zeros((2, 2))
    ch = O.reduce_links(keys, a, tau, fd, 1, 1, p_tx=1.0)
    assert abs(ch["tau_mean"][0, 0] - 1.25e-6) < 1e-18
    assert abs(ch["tau_rms"][0, 0] - math.sqrt(3.0) / 4.0 * 1e-6) < 1e-18
    assert abs(ch["tau_mean"][1, 0] - 1.5e-6) < 1e-18
    assert abs(ch["tau_rms"][1, 0] - 0.5e-6) < 1e-18
    # a link with one path has no spread; a link with no path reports zeros
    ch1 = O.reduce_links(keys[:1], a[:1], tau[:1], fd[:1], 1, 2, p_tx=1.0)
    assert ch1["tau_rms"][0, 0] == 0.0 and ch1["tau_mean"][0, 0] == 1e-6
    assert ch1["tau_rms"][0, 1] == 0.0 and ch1["tau_mean"][0, 1] == 0.0


def test_rms_delay_spread_two_ray_ground_closed_form():
    """Ground only: the link's two paths have delays d/c and r/c (r the image
    distance) and powers |lambda/(4 pi d)|^2 and |Gamma_v lambda/(4 pi r)|^2;
    the power-weighted RMS spread of two delays is sqrt(w1 w2)/(w1 + w2) |dt|."""
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    tx = np.array([[0.0, 0.0, 25.0]])
    rx = np.array([[60.0, -80.0, 1.5]])
    fr = static_frame(tx, rx)
    res = O.run_frame(os_, fr, 20000, 1, [F28])
    assert len(res.keys) == 2
    d = float(np.linalg.norm(rx - tx))
    r = float(np.linalg.norm(rx - tx * np.array([1, 1, -1])))
    i_los = int(np.nonzero(res.keys[:, 2] == 0)[0][0])
    w = np.abs(res.a[:, 0]) ** 2
    w_los, w_gnd = w[i_los], w[1 - i_los]
    lam = C0 / F28
    assert abs(w_los - (lam / (4 * math.pi * d)) ** 2) < 1e-12 * w_los
    want = math.sqrt(w_los * w_gnd) / (w_los + w_gnd) * (r - d) / C0
    assert abs(res.channels["tau_rms"][0, 0] - want) < 1e-9 * want
    assert abs(res.channels["tau_mean"][0, 0] - (w_los * d + w_gnd * r) / (w_los + w_gnd) / C0) < 1e-18


# --------------------------------------------------------------------------
# departure and arrival angles
# --------------------------------------------------------------------------

def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


@pytest.mark.parametrize("phi_deg", [0.0, 37.0, 135.0, -100.0])
def test_angles_line_of_sight_and_ground_bounce(phi_deg):
    """AoD = (azimuth, elevation) of the first leg, AoA = (azimuth, elevation)
    of the direction back along the last leg.  Line of sight: azimuth phi,
    elevation atan2(h_r - h_t, d); arrival azimuth phi + pi, elevation
    atan2(h_t - h_r, d).  Ground bounce: both legs lie in the vertical plane
    of phi and make the angle atan2(h_t + h_r, d) with the ground."""
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    phi = math.radians(phi_deg)
    ht, hr, d = 30.0, 1.5, 140.0
    tx = np.array([[3.0, -7.0, ht]])
    rx = np.array([[3.0 + d * math.cos(phi), -7.0 + d * math.sin(phi), hr]])
    fr = static_frame(tx, rx)
    keys = np.array([spec_key(0, 0, []), spec_key(0, 0, [0])], np.int32)
    valid, amb, tri, pts = O.validate(os_, g, keys, tx, rx)
    assert valid.all() and not amb.any()
    _, _, _, aod, aoa = O.evaluate(os_, g, keys, pts, fr, [F28])
    # line of sight
    assert abs(_wrap(aod[0, 0] - phi)) < 1e-12
    assert abs(aod[0, 1] - math.atan2(hr - ht, d)) < 1e-12
    assert abs(_wrap(aoa[0, 0] - (phi + math.pi))) < 1e-12
    assert abs(aoa[0, 1] - math.atan2(ht - hr, d)) < 1e-12
    # ground bounce: leaves downward, arrives from below
    el = math.atan2(ht + hr, d)
    assert abs(_wrap(aod[1, 0] - phi)) < 1e-12
    assert abs(aod[1, 1] + el) < 1e-12
    assert abs(_wrap(aoa[1, 0] - (phi + math.pi))) < 1e-12
    assert abs(aoa[1, 1] + el) < 1e-12


def test_angles_wall_bounce_mirror_azimuth():
    """A bounce off the vertical wall x = 50: the departure azimuth points at
    the receiver's image (100 - x_r, y_r), the arrival azimuth back at the
    transmitter's image (100 - x_t, y_t); elevations from the unfolded length."""
    sc = city.tiny_ground_wall(wall_x=50.0)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[0.0, 0.0, 10.0]])
    rx = np.array([[20.0, 35.0, 2.0]])
    fr = static_frame(tx, rx)
    key = np.array([spec_key(0, 0, [1])], np.int32)
    valid, amb, tri, pts = O.validate(os_, g, key, tx, rx)
    assert valid[0] and not amb[0]
    _, _, _, aod, aoa = O.evaluate(os_, g, key, pts, fr, [F28])
    img_rx = np.array([100.0 - 20.0, 35.0, 2.0])
    v = img_rx - tx[0]
    assert abs(aod[0, 0] - math.atan2(v[1], v[0])) < 1e-12
    assert abs(aod[0, 1] - math.atan2(v[2], math.hypot(v[0], v[1]))) < 1e-12
    img_tx = np.array([100.0, 0.0, 10.0])
    u = img_tx - rx[0]
    assert abs(aoa[0, 0] - math.atan2(u[1], u[0])) < 1e-12
    assert abs(aoa[0, 1] - math.atan2(u[2], math.hypot(u[0], u[1]))) < 1e-12


# --------------------------------------------------------------------------
# rotated object transforms
# --------------------------------------------------------------------------

# local wall in the plane y = 0, x in [-30, 70], z in [0, 30] (asymmetric in
# x, so a transposed rotation puts it elsewhere)
_WALL_LOCAL = [(-30.0, 0.0, 0.0), (70.0, 0.0, 0.0), (70.0, 0.0, 30.0), (-30.0, 0.0, 30.0)]


def _ground_and_dynamic_wall():
    g = [(-500.0, -500.0, 0.0), (500.0, -500.0, 0.0), (500.0, 500.0, 0.0), (-500.0, 500.0, 0.0)]
    verts = np.array(g + _WALL_LOCAL, np.float32)
    tris = np.array([(0, 1, 2), (0, 2, 3), (4, 5, 6), (4, 6, 7)], np.int32)
    sc = city._static_scene(verts, tris, [0, 0, 1, 1], [0, 1], 2, [city.EPS_GROUND, city.EPS_CONCRETE],
                            [0, 0, 10], 500, face_mat=[0, 1])
    sc.object_dynamic = np.array([0, 1], np.uint8)
    return sc


def _yaw90(t):
    """Rotation by +90 degrees about z: (x, y, z) -> (-y, x, z), then t."""
    x = np.zeros((1, 3, 4))
    x[0, :, :3] = [[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]
    x[0, :, 3] = t
    return x


def test_yaw90_world_vertices_by_hand():
    """Local (x, 0, z) -> world (20.1 - 0, x + 5, z) as float32; the static
    ground is untouched.  (A transposed rotation would give y = 5 - x.)"""
    sc = _ground_and_dynamic_wall()
    os_ = O.OracleScene(sc)
    g = os_.geometry(_yaw90([20.1, 5.0, 0.0]))
    want = np.array([(np.float32(20.1), x + 5.0, z) for (x, _, z) in _WALL_LOCAL], np.float32)
    assert np.array_equal(g.verts[4:], want)
    assert np.array_equal(g.verts[:4], sc.verts[:4])
    # 180 degrees (heading along -x): (x, y, z) -> (-x, -y, z); exact sums
    x = np.zeros((1, 3, 4))
    x[0, :, :3] = np.diag([-1.0, -1.0, 1.0])
    x[0, :, 3] = [0.5, 0.25, 1.0]
    g2 = os_.geometry(x)
    want2 = np.array([(0.5 - x_, 0.25, z + 1.0) for (x_, _, z) in _WALL_LOCAL], np.float32)
    assert np.array_equal(g2.verts[4:], want2)


def test_yaw90_wall_reflection_length_and_doppler():
    """The yawed wall lies in the world plane x = 20 with y in [-25, 75].  A
    receiver at (5, 80, 4) sees the transmitter (0, 0, 10) reflected with the
    image length |(40, 0, 10) - rx| = sqrt(7661) (the reflection point, y =
    45.7, is off the wall a transposed rotation would make).  Moving the wall
    along +x at 3 m/s moves the image at 6 m/s: f_D = -(1/lambda) 6 (40 - 5) / L."""
    sc = _ground_and_dynamic_wall()
    os_ = O.OracleScene(sc)
    tx = np.array([[0.0, 0.0, 10.0]])
    rx = np.array([[5.0, 80.0, 4.0]])
    fr = static_frame(tx, rx, obj_xform=_yaw90([20.0, 5.0, 0.0]), obj_vel=np.array([[3.0, 0.0, 0.0]]))
    g = os_.geometry(fr.obj_xform)
    key = np.array([spec_key(0, 0, [1])], np.int32)
    valid, amb, tri, pts = O.validate(os_, g, key, tx, rx)
    assert valid[0] and not amb[0]
    L = math.sqrt(7661.0)
    _, tau, fd, _, _ = O.evaluate(os_, g, key, pts, fr, [F28])
    assert abs(tau[0] * C0 - L) < 1e-9
    assert abs(pts[0, 0, 0] - 20.0) < 1e-12 and abs(pts[0, 0, 1] - 80.0 * 4.0 / 7.0) < 1e-9
    lam = C0 / F28
    assert abs(fd[0, 0] - (-(6.0 * 35.0 / L) / lam)) < 1e-6
    # discovery finds it too, and the transposed rotation loses it
    res = O.run_frame(os_, fr, 40000, 1, [F28])
    assert tuple(spec_key(0, 0, [1])) in key_set(res.keys)
    xt = _yaw90([20.0, 5.0, 0.0])
    xt[0, :, :3] = xt[0, :, :3].T
    gt = os_.geometry(xt)
    valid_t, _, _, _ = O.validate(os_, gt, key, tx, rx)
    assert not valid_t[0]


# --------------------------------------------------------------------------
# the path cache across frames
# --------------------------------------------------------------------------

def test_cache_bookkeeping_cached_and_discovery_frames():
    """cache_t = valid_t(cache_{t-1}) on a cached frame and
    valid_t(cache_{t-1} U discovered_t) on a discovery frame; line of sight is
    tested for every link every frame and never cached."""
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr0 = sc.frame(0.0)
    N, K = 20000, 2
    f0 = O.run_frame(os_, fr0, N, K, [F28], want_robust=False)
    c0 = O.cache_of(f0)
    assert len(c0) > 20 and not np.any(c0[:, 2] == O.LOS)
    # frame 1: receivers moved by a few metres (some cached keys break)
    fr1 = sc.frame(0.0)
    fr1.rx_pos = fr1.rx_pos + np.random.default_rng(4).normal(0, 3.0, fr1.rx_pos.shape) * np.array([1, 1, 0])
    g1 = os_.geometry(fr1.obj_xform)
    cached = O.run_frame(os_, fr1, N, K, [F28], discover=False, cache=c0)
    v_c0, _, _, _ = O.validate(os_, g1, c0, fr1.tx_pos, fr1.rx_pos)
    los = O.los_keys(sc.n_tx, sc.n_rx)
    v_los, _, _, _ = O.validate(os_, g1, los, fr1.tx_pos, fr1.rx_pos)
    assert 0 < v_c0.sum() < len(c0)  # the move dropped some keys and kept others
    assert key_set(cached.keys) == key_set(c0[v_c0]) | key_set(los[v_los])
    assert key_set(O.cache_of(cached)) == key_set(c0[v_c0])
    # frame 2: discovery with the cache of frame 1
    c1 = O.cache_of(cached)
    fr2 = sc.frame(0.0)
    fr2.rx_pos = fr1.rx_pos + np.array([1.5, -2.0, 0.0])
    g2 = os_.geometry(fr2.obj_xform)
    disc = O.run_frame(os_, fr2, N, K, [F28], cache=c1, want_robust=False)
    fresh = O.run_frame(os_, fr2, N, K, [F28], want_robust=False)  # discovery alone
    v_c1, _, _, _ = O.validate(os_, g2, c1, fr2.tx_pos, fr2.rx_pos)
    assert key_set(disc.keys) == key_set(fresh.keys) | key_set(c1[v_c1])
    # the union is not trivial: the cache contributes keys the rays missed, or discovery adds new ones
    assert key_set(disc.keys) != key_set(c1[v_c1]) or key_set(disc.keys) != key_set(fresh.keys)


def test_coplanar_overlapping_faces_make_a_reflection_ambiguous():
    """Two squares of different objects in the plane z = 2 that overlap on
    x in [5, 10] (like the roofs of two overlapping vehicles).  A reflection
    off the first at x = 3 is valid and unambiguous; at x = 6 the second
    square touches both legs at the reflection point, so whether it blocks
    them is a rounding matter and the key is ambiguous."""
    sq = lambda x0, x1: [(x0, 0.0, 2.0), (x1, 0.0, 2.0), (x1, 10.0, 2.0), (x0, 10.0, 2.0)]
    g4 = [(-500.0, -500.0, 0.0), (500.0, -500.0, 0.0), (500.0, 500.0, 0.0), (-500.0, 500.0, 0.0)]
    verts = np.array(g4 + sq(0.0, 10.0) + sq(5.0, 15.0), np.float32)
    tris = np.array([(0, 1, 2), (0, 2, 3), (4, 5, 6), (4, 6, 7), (8, 9, 10), (8, 10, 11)], np.int32)
    sc = city._static_scene(verts, tris, [0, 0, 1, 1, 2, 2], [0, 1, 2], 3, [city.EPS_GROUND, city.EPS_METAL],
                            [0, 0, 10], 500, face_mat=[0, 1, 1])
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[2.0, 5.0, 10.0]])
    rx = np.array([[4.0, 5.0, 10.0], [10.0, 5.0, 10.0]])
    keys = np.array([spec_key(0, 0, [1]), spec_key(0, 1, [1])], np.int32)
    valid, amb, _, pts = O.validate(os_, g, keys, tx, rx)
    assert valid[0] and not amb[0] and abs(pts[0, 0, 0] - 3.0) < 1e-12
    assert amb[1] and abs(pts[1, 0, 0] - 6.0) < 1e-12
