"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than its own formulas:
closed forms (Friis, the two-ray ground model, path sets and image lengths
for perpendicular and parallel planes), textbook alternates (Snell forms of the Fresnel
coefficients, Keller's GTD coefficient), library routines (scipy's Fresnel
integrals and Faddeeva-based erfcx), invariants (reciprocity, energy bound,
continuity of the total field across shadow and reflection boundaries,
Doppler as the time derivative of the path length) and the paper's own
printed numbers (Eq (3), the speed ratios of Table III).
"""
import math
import os

import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from synth import city
from tests.oracle_util import C0, key_set, spec_key, static_frame

F28 = 28e9


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build()


# --------------------------------------------------------------------------
# free space and the Fresnel coefficients
# --------------------------------------------------------------------------

def test_friis_line_of_sight():
    """|a|^2 P_tx equals Friis P_tx (lambda / 4 pi d)^2; phase -k d; delay d/c."""
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[1.25, -3.5, 10.0]])
    rx = np.array([[123.4, 56.7, 3.0]])
    fr = static_frame(tx, rx)
    keys = O.los_keys(1, 1)
    valid, amb, tri, pts = O.validate(os_, g, keys, tx, rx)
    assert valid[0] and not amb[0]
    for f in (3.5e9, 28e9):
        a, tau, fd, aod, aoa = O.evaluate(os_, g, keys, pts, fr, [f])
        d = float(np.linalg.norm(rx - tx))
        lam = C0 / f
        friis = (lam / (4 * math.pi * d)) ** 2
        assert abs(abs(a[0, 0]) ** 2 - friis) <= 1e-12 * friis
        ph = -2 * math.pi * math.fmod(d / lam, 1.0)
        assert abs(np.angle(a[0, 0] * np.exp(-1j * ph))) < 1e-8
        assert abs(tau[0] - d / C0) <= 1e-15 * d / C0
        assert fd[0, 0] == 0.0


def _snell(eps, th):
    n = math.sqrt(eps)
    tt = math.asin(math.sin(th) / n)
    return -math.sin(th - tt) / math.sin(th + tt), math.tan(th - tt) / math.tan(th + tt)


@pytest.mark.parametrize("eps", [2.25, 5.3, 15.0])
@pytest.mark.parametrize("deg", [5.0, 30.0, 45.0, 70.0, 89.0])
def test_fresnel_matches_snell_forms(eps, deg):
    """Lossless dielectric: Gamma_TE = -sin(t-t')/sin(t+t'), Gamma_TM = tan(t-t')/tan(t+t')."""
    th = math.radians(deg)
    te, tm = O.fresnel_gamma(complex(eps, 0.0), math.cos(th))
    rte, rtm = _snell(eps, th)
    assert abs(te - rte) < 1e-12
    assert abs(tm - rtm) < 1e-12


def test_fresnel_special_cases():
    eps = 5.3 - 0.2j
    te, tm = O.fresnel_gamma(eps, 1.0)
    n = np.sqrt(eps)
    assert abs(te - (1 - n) / (1 + n)) < 1e-14  # normal incidence
    assert abs(tm + te) < 1e-14  # Gamma_TM = -Gamma_TE at normal incidence
    # Brewster angle of a real permittivity: Gamma_TM = 0
    thb = math.atan(math.sqrt(5.3))
    _, tmb = O.fresnel_gamma(5.3 + 0j, math.cos(thb))
    assert abs(tmb) < 1e-14
    # metal (eps'' -> infinity): |Gamma| -> 1, PEC signs TE -> -1, TM -> +1
    te, tm = O.fresnel_gamma(1.0 - 1e6j, math.cos(math.radians(40)))
    assert abs(te + 1) < 5e-3 and abs(tm - 1) < 5e-3
    # passivity of lossy media
    for deg in np.linspace(0, 89.9, 50):
        te, tm = O.fresnel_gamma(15 - 1.5j, math.cos(math.radians(deg)))
        assert abs(te) <= 1 + 1e-15 and abs(tm) <= 1 + 1e-15


# --------------------------------------------------------------------------
# path search: closed-form path sets and lengths
# --------------------------------------------------------------------------

def _discover(sc, tx, rx, N, K, diffraction=False, rx_vel=None):
    os_ = O.OracleScene(sc)
    fr = static_frame(tx, rx, rx_vel=rx_vel)
    res = O.run_frame(os_, fr, N, K, [F28], diffraction=diffraction)
    return os_, fr, res


def test_two_ray_ground():
    """Ground only: exactly LoS + ground bounce; the sum matches the two-ray
    model lambda/(4 pi)[e^{-jkd}/d + Gamma_v e^{-jkr}/r], r the image distance."""
    sc = city.tiny_ground()
    tx = np.array([[0.0, 0.0, 10.0]])
    rx = np.array([[80.0, 30.0, 1.5]])
    os_, fr, res = _discover(sc, tx, rx, 20000, 2)
    assert key_set(res.keys) == {tuple(spec_key(0, 0, [])), tuple(spec_key(0, 0, [0]))}
    lam = C0 / F28
    k = 2 * math.pi / lam
    d = float(np.linalg.norm(rx - tx))
    img = tx * np.array([1, 1, -1])
    r = float(np.linalg.norm(rx - img))
    cos_i = (10.0 + 1.5) / r
    _, g_v = _snell_lossy(city.EPS_GROUND, cos_i)
    h = lam / (4 * math.pi) * (np.exp(-1j * k * d) / d + g_v * np.exp(-1j * k * r) / r)
    assert abs(res.channels["H"][0, 0] - h) < 1e-9 * abs(h)


def _snell_lossy(eps, c):
    """Fresnel coefficients via the complex transmission angle (Snell's law)."""
    s = math.sqrt(1 - c * c)
    n = np.sqrt(complex(eps))
    st = s / n
    ct = np.sqrt(1 - st * st)
    if ct.real < 0:
        ct = -ct
    te = (c - n * ct) / (c + n * ct)
    tm = (n * c - ct) / (n * c + ct)
    return te, tm


def _mirror(p, axis, at):
    q = np.array(p, np.float64).copy()
    q[axis] = 2 * at - q[axis]
    return q


@pytest.mark.parametrize("K", [2, 3])
@pytest.mark.parametrize("z_rx", [1.5, 6.0])
def test_ground_and_wall_corner_paths(K, z_rx):
    """Perpendicular ground + wall: exactly four paths for K >= 2 -- LoS, G, W
    and ONE double bounce.  Both double bounces share the image
    (2w - x_t, y_t, -z_t); walking from Rx towards it, the plane crossed first
    is the last reflection, so exactly one of (G, W) / (W, G) exists (corner
    reflector).  Lengths are |Rx - image(Tx)|."""
    wall_x = 50.0
    sc = city.tiny_ground_wall(wall_x=wall_x)
    tx = np.array([[0.0, 0.0, 10.0]])
    rx = np.array([[30.0, 20.0, z_rx]])
    os_, fr, res = _discover(sc, tx, rx, 40000, K)
    dbl = _mirror(_mirror(tx[0], 2, 0.0), 0, wall_x)
    t_wall = (wall_x - rx[0, 0]) / (dbl[0] - rx[0, 0])
    t_ground = rx[0, 2] / (rx[0, 2] - dbl[2])
    last_is_wall = t_wall < t_ground
    want = {(): tx[0], (0,): _mirror(tx[0], 2, 0.0), (1,): _mirror(tx[0], 0, wall_x),
            ((0, 1) if last_is_wall else (1, 0)): dbl}
    assert key_set(res.keys) == {tuple(spec_key(0, 0, list(f))) for f in want}
    for row, tau in zip(res.keys, res.tau):
        faces = tuple(int(x) for x in row[4:4 + row[3]])
        L = float(np.linalg.norm(rx[0] - want[faces]))
        assert abs(tau * C0 - L) < 1e-9 * L


@pytest.mark.parametrize("K", [3, 5])
def test_street_canyon_one_plus_2k(K):
    """Two parallel walls, no ground: 1 + 2K paths for K reflections, lengths
    from the unfolded images (K = 5 is the deepest order the method runs)."""
    gap = 20.0
    sc = city.tiny_canyon(gap=gap)
    tx = np.array([[0.0, 2.0, 0.0]])
    rx = np.array([[90.0, -5.0, 3.0]])
    os_, fr, res = _discover(sc, tx, rx, 60000, K)
    assert len(res.keys) == 1 + 2 * K
    walls = {0: -gap / 2, 1: gap / 2}
    for row, tau in zip(res.keys, res.tau):
        faces = [int(x) for x in row[4:4 + row[3]]]
        assert all(faces[i] != faces[i + 1] for i in range(len(faces) - 1))
        img = tx[0].copy()
        for f in faces:
            img = _mirror(img, 1, walls[f])
        L = float(np.linalg.norm(rx[0] - img))
        assert abs(tau * C0 - L) < 1e-9 * L
    orders = sorted(int(r[3]) for r in res.keys)
    assert orders == [0] + [k for k in range(1, K + 1) for _ in range(2)]


def test_brute_force_image_enumeration_toy_city():
    """Every face sequence of order <= 2 that the image method validates (and
    that is not within a validation margin) is found by SBR discovery with a
    dense launch; SBR finds nothing else."""
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr = sc.frame(0.0)
    g = os_.geometry(fr.obj_xform)
    res = O.run_frame(os_, fr, 400000, 2, [F28], want_robust=False)
    F = os_.F
    seqs = [[f] for f in range(F)] + [[f, h] for f in range(F) for h in range(F) if f != h]
    keys = np.array([spec_key(0, r, s) for r in range(len(fr.rx_pos)) for s in seqs], np.int32)
    valid, amb, _, _ = O.validate(os_, g, keys, fr.tx_pos, fr.rx_pos)
    brute = key_set(keys[valid & ~amb])
    found = key_set(res.keys[res.keys[:, 2] == 1])
    assert found <= key_set(keys[valid])
    missing = brute - found
    assert len(brute) > 30
    assert not missing, sorted(missing)


def test_reciprocity_swap_tx_rx():
    """Swapping Tx and Rx (vertical iso antennas at both ends) gives the
    reversed key set and identical complex gains."""
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    a_pos = np.array([[0.0, 0.0, 25.0]])
    b_pos = sc.frame(0.0).rx_pos[2:3]
    fa = static_frame(a_pos, b_pos)
    fb = static_frame(b_pos, a_pos)
    ra = O.run_frame(os_, fa, 200000, 3, [F28], want_robust=False)
    rb = O.run_frame(os_, fb, 200000, 3, [F28], want_robust=False)

    def rev(k):
        k = list(k)
        n = k[3]
        return tuple(k[:4] + list(reversed(k[4:4 + n])) + k[4 + n:])

    ka = {tuple(int(x) for x in r): i for i, r in enumerate(ra.keys) if not ra.ambiguous[i]}
    kb = {rev(tuple(int(x) for x in r)): i for i, r in enumerate(rb.keys) if not rb.ambiguous[i]}
    common = set(ka) & set(kb)
    assert len(common) >= 0.9 * max(len(ka), len(kb)) and len(common) > 5
    # legs are summed in the opposite order: L/lambda ~ 1e4 cycles at 28 GHz, so
    # double rounding of L moves the phase by ~1e-11 rad
    for k in common:
        x, y = ra.a[ka[k], 0], rb.a[kb[k], 0]
        assert abs(x - y) <= 1e-10 * abs(x)


def test_energy_bound_specular():
    """|a_i| <= lambda / (4 pi d_LoS) for every specular path when all |Gamma| <= 1."""
    w = city.workload("toy")
    os_ = O.OracleScene(w.scene)
    fr = w.scene.frame(0.0)
    res = O.run_frame(os_, fr, w.rays_per_tx, w.max_reflections, w.freqs_hz, want_robust=False)
    lam = C0 / w.freqs_hz[0]
    for row, a in zip(res.keys, res.a[:, 0]):
        d = float(np.linalg.norm(fr.rx_pos[row[1]] - fr.tx_pos[row[0]]))
        assert abs(a) <= lam / (4 * math.pi * d) * (1 + 1e-12)


# --------------------------------------------------------------------------
# Doppler: Eq (3), time derivative of path length, Table III speed ratios
# --------------------------------------------------------------------------

def test_doppler_eq3_line_of_sight():
    """Section III-C Eq (3): f_d = f_c (v / c) cos(theta), static base station."""
    sc = city.tiny_ground()
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[0.0, 0.0, 30.0]])
    rx = np.array([[200.0, 50.0, 1.5]])
    v = np.array([[-12.0, 7.0, 0.0]])
    fr = static_frame(tx, rx, rx_vel=v)
    keys = O.los_keys(1, 1)
    valid, amb, tri, pts = O.validate(os_, g, keys, tx, rx)
    for f in (3e9, 30e9):
        _, _, fd, _, _ = O.evaluate(os_, g, keys, pts, fr, [f])
        to_tx = (tx - rx)[0]
        cos_t = float(v[0] @ to_tx / (np.linalg.norm(v) * np.linalg.norm(to_tx)))
        want = f * np.linalg.norm(v) / C0 * cos_t
        assert abs(fd[0, 0] - want) < 1e-9


def _vehicle_scene():
    """Ground + one metal vehicle box (dynamic object 1)."""
    vv, vt, vf = city.vehicle_template()
    gv = [(-500, -500, 0), (500, -500, 0), (500, 500, 0), (-500, 500, 0)]
    verts = np.concatenate([np.array(gv, np.float64), vv]).astype(np.float32)
    tris = np.concatenate([np.array([(0, 1, 2), (0, 2, 3)]), vt + 4]).astype(np.int32)
    tri_face = np.concatenate([[0, 0], vf + 1]).astype(np.int32)
    sc = city._static_scene(verts, tris, tri_face, [0] + [1] * 6, 2, [city.EPS_GROUND, city.EPS_METAL], [0, 0, 10],
                            500, face_mat=[0] + [1] * 6)
    sc.object_dynamic = np.array([0, 1], np.uint8)
    return sc


def _veh_xform(p):
    x = np.zeros((1, 3, 4))
    x[0, :, :3] = np.eye(3)
    x[0, :, 3] = p
    return x


def test_doppler_is_path_length_rate_moving_reflector():
    """f_D = -(1/lambda) dL/dt for a fixed key with a moving reflector and a
    moving receiver: compared with a central difference of the exact image
    length, error O(h^2).  The step (2^-10 s) and the vehicle velocity are
    dyadic so the float32 world vertices at t +- h are exact."""
    sc = _vehicle_scene()
    os_ = O.OracleScene(sc)
    tx = np.array([[5.0, -20.0, 1.5]])
    rx0 = np.array([[25.0, -25.0, 1.0]])
    vrx = np.array([[-3.0, 1.0, 0.0]])
    p0 = np.array([15.0, 0.0, 0.0])
    vveh = np.array([8.0, -4.0, 0.0])
    face_side = 1 + 2  # vehicle face facing -y
    key = np.array([spec_key(0, 0, [face_side])], np.int32)

    def at(t):
        fr = static_frame(tx, rx0 + vrx * t, rx_vel=vrx, obj_xform=_veh_xform(p0 + vveh * t), obj_vel=vveh[None])
        g = os_.geometry(fr.obj_xform)
        valid, amb, tri, pts = O.validate(os_, g, key, fr.tx_pos, fr.rx_pos)
        assert valid[0]
        return O.evaluate(os_, g, key, pts, fr, [F28])

    _, _, fd0, _, _ = at(0.0)
    h = 2.0 ** -10
    _, tp, _, _, _ = at(h)
    _, tm, _, _, _ = at(-h)
    lam = C0 / F28
    fd_num = -(tp[0] - tm[0]) * C0 / (2 * h) / lam
    assert abs(fd0[0, 0]) > 10.0
    assert abs(fd0[0, 0] - fd_num) < 1e-5


def test_doppler_linear_in_speed_table3(tmp_path):
    """Table III: at fixed geometry the mean Doppler shift and the RMS Doppler
    spread scale with speed (the paper's 10 -> 50 m/s rows are exactly x5).
    The oracle's Doppler statistics scale by exactly 5 when every velocity does."""
    rows = _table3()
    for (v1, d1, m1, s1), (v2, d2, m2, s2) in [(rows[0], rows[2]), (rows[1], rows[3])]:
        assert d1 == d2 and v2 / v1 == 5.0
        assert abs(m2 / m1 - 5.0) < 1e-9
        assert abs(s2 / s1 - 5.0) < 0.15  # 0.34 / 0.07 is rounded in the table
    w = city.workload("toy")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr = sc.frame(0.0)
    fr.rx_vel = np.random.default_rng(5).normal(0, 10, fr.rx_vel.shape)
    r1 = O.run_frame(os_, fr, 20000, 3, [30e9], want_robust=False)
    fr.rx_vel = fr.rx_vel * 5.0
    r5 = O.run_frame(os_, fr, 20000, 3, [30e9], want_robust=False)
    assert key_set(r1.keys) == key_set(r5.keys)
    np.testing.assert_allclose(r5.fd, 5.0 * r1.fd, rtol=1e-12, atol=1e-9)
    for name in ("fd_mean", "fd_rms"):
        np.testing.assert_allclose(r5.channels[name], 5.0 * r1.channels[name], rtol=1e-9, atol=1e-9)


def _table3():
    path = os.path.join(os.path.dirname(__file__), "golden", "table3_doppler.txt")
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append(tuple(float(x) for x in line.split()))
    return rows


def test_power_weighted_doppler_statistics_by_hand():
    """Mean Doppler shift and RMS spread (Section V-D) are power-weighted
    moments: two paths with powers 3:1 and shifts 100, -20 Hz give mean 70 Hz
    and RMS spread sqrt(0.75*30^2 + 0.25*90^2) = 51.96... Hz."""
    keys = np.array([spec_key(0, 0, []), spec_key(0, 0, [3])], np.int32)
    a = np.array([[math.sqrt(3.0)], [1.0j]])
    fd = np.array([[100.0], [-20.0]])
    tau = np.array([1e-6, 2e-6])
    ch = O.reduce_links(keys, a, tau, fd, 1, 1, p_tx=1.0)
    assert abs(ch["fd_mean"][0, 0] - 70.0) < 1e-12
    assert abs(ch["fd_rms"][0, 0] - math.sqrt(0.75 * 900 + 0.25 * 8100)) < 1e-9
    assert abs(ch["tau_mean"][0, 0] - 1.25e-6) < 1e-18
    assert abs(ch["P_inc"][0, 0] - 4.0) < 1e-12
    assert abs(ch["P_coh"][0, 0] - abs(math.sqrt(3) + 1j) ** 2) < 1e-12


# --------------------------------------------------------------------------
# diffraction: Fresnel integral, UTD limits and field continuity
# --------------------------------------------------------------------------

def _F_scipy(X):
    u = math.sqrt(2 * X / math.pi)
    S, C = sp.fresnel(u)
    integral = math.sqrt(math.pi / 2) * ((0.5 - C) - 1j * (0.5 - S))
    return 2j * math.sqrt(X) * np.exp(1j * X) * integral


@pytest.mark.parametrize("X", [1e-6, 1e-3, 0.05, 0.5, 1.0, 3.0, 6.0, 6.3, 10.0, 30.0, 100.0, 1e3])
def test_transition_function_vs_scipy_fresnel(X):
    ref = _F_scipy(X)
    got = O.utd_F(X)
    assert abs(got - ref) < 2e-12 * max(1.0, abs(ref)) + 1e-9 * abs(ref) * (X > 50)


@pytest.mark.parametrize("v", [0.0, 0.3, 1.0, 2.0, 2.49, 2.51, 4.0, 10.0, 50.0])
def test_erfcx_vs_scipy(v):
    w = v * np.exp(1j * math.pi / 4)
    assert abs(O.erfcx_diag(v) - sp.erfcx(w)) < 1e-13 * max(1.0, abs(sp.erfcx(w)))


def test_transition_function_asymptotes():
    for X in (1e3, 1e4, 1e5):
        assert abs(O.utd_F(X) - (1 + 0.5j / X - 0.75 / X ** 2)) < 5 / X ** 3
    for X in (1e-8, 1e-6):
        assert abs(O.utd_F(X) - math.sqrt(math.pi * X) * np.exp(1j * math.pi / 4)) < 3 * X


def _keller(n, k, beta0, php, ph):
    c = np.exp(-1j * math.pi / 4) * math.sin(math.pi / n) / (n * math.sqrt(2 * math.pi * k) * math.sin(beta0))
    t1 = 1 / (math.cos(math.pi / n) - math.cos((ph - php) / n))
    t2 = 1 / (math.cos(math.pi / n) - math.cos((ph + php) / n))
    return c * (t1 - t2), c * (t1 + t2)


@pytest.mark.parametrize("php,ph", [(0.4, 2.0), (1.0, 4.2), (2.5, 0.3), (0.7, 3.3)])
def test_utd_reduces_to_keller_gtd_far_from_boundaries(php, ph):
    """kL -> infinity away from shadow/reflection boundaries: F -> 1 and the
    UTD coefficient of a perfectly conducting wedge is Keller's GTD form."""
    n, k, beta0 = 1.5, 2 * math.pi / (C0 / F28), 1.1
    L = 1e7
    ds, dh = O.utd_D(n, k, L, beta0, php, ph, complex(1, -1e30), complex(1, -1e30))
    ks, kh = _keller(n, k, beta0, php, ph)
    assert abs(ds - ks) < 1e-5 * abs(ks)
    assert abs(dh - kh) < 1e-5 * abs(kh)


def _wedge_total_field(os_, g, tx, rx, f, extra_keys=()):
    fr = static_frame(tx, rx)
    keys = [O.los_keys(1, 1)[0]] + [np.array(k, np.int32) for k in extra_keys]
    for e in range(os_.E):
        keys.append(np.array([0, 0, 2, 1, e, -1, -1, -1, -1], np.int32))
    keys = np.array(keys, np.int32)
    valid, amb, tri, pts = O.validate(os_, g, keys, tx, rx, diff_max_leg=1e9)
    a, _, _, _, _ = O.evaluate(os_, g, keys[valid], pts[valid], fr, [f])
    parts = {tuple(int(x) for x in k): v for k, v in zip(keys[valid], a[:, 0])}
    return sum(parts.values()), parts


def _jump(field_at, deltas=(1e-6, 2e-6)):
    """Discontinuity of field_at(angle offset) at offset 0: the difference
    D(d) = E(+d) - E(-d) = J + c d for a field with a jump J, so two offsets
    extrapolate J and remove the smooth variation."""
    d1, d2 = deltas
    D1 = field_at(+d1)[0] - field_at(-d1)[0]
    D2 = field_at(+d2)[0] - field_at(-d2)[0]
    return (d2 * D1 - d1 * D2) / (d2 - d1)


@pytest.mark.parametrize("f", [1e9, 28e9])
@pytest.mark.parametrize("z_tx", [10.0, 17.0])
def test_total_field_continuous_across_shadow_boundary(f, z_tx):
    """GO + UTD total field is continuous across the incident shadow boundary
    of a vertical box corner: the line-of-sight term jumps, the total does not."""
    sc = city.tiny_wedge(size=40.0, height=30.0, eps=city.EPS_METAL)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    tx = np.array([[-30.0, -20.0, z_tx]])
    corner = np.array([0.0, 40.0, 0.0])  # north-west corner: its boundary runs outside the box
    dirn = (corner - tx[0])[:2]
    dirn /= np.linalg.norm(dirn)
    R = 25.0

    def at(delta):
        ang = math.atan2(dirn[1], dirn[0]) + delta
        rx = np.array([[corner[0] + R * math.cos(ang), corner[1] + R * math.sin(ang), 12.0]])
        return _wedge_total_field(os_, g, tx, rx, f)

    los = tuple(O.los_keys(1, 1)[0])
    assert (los in at(-1e-6)[1]) != (los in at(1e-6)[1])  # line of sight on exactly one side
    go_jump = abs(at(-1e-6)[1].get(los, 0) - at(1e-6)[1].get(los, 0))
    assert abs(_jump(at)) < 1e-5 * go_jump


@pytest.mark.parametrize("eps", [city.EPS_METAL, city.EPS_CONCRETE, 5.3 + 0j])
@pytest.mark.parametrize("case", ["roof", "wall"])
def test_total_field_continuous_across_reflection_boundary(eps, case):
    """GO + UTD total field is continuous across a reflection boundary of the
    roof edge shared by the south wall (face 0, the 0-face) and the roof
    (face 4, the n-face): the reflected GO term exists on one side only and
    the lossy Luebbers term (R_n T3 for the roof, R_0 T4 for the wall)
    cancels its jump.  The edge is perpendicular to the plane of incidence,
    so the TE/TM split is exact."""
    sc = city.tiny_wedge(size=40.0, height=30.0, eps=eps)
    os_ = O.OracleScene(sc)
    g = os_.geometry(np.zeros((0, 3, 4)))
    edge_pt = np.array([20.0, 0.0, 30.0])
    if case == "roof":
        face, tx = 4, np.array([[20.0, 15.0, 45.0]])
        img = tx[0] * np.array([1, 1, -1]) + np.array([0, 0, 60.0])
    else:
        face, tx = 0, np.array([[20.0, -15.0, 20.0]])
        img = tx[0] * np.array([1, -1, 1])
    d = edge_pt - img
    d /= np.linalg.norm(d)
    R = 25.0

    def at(delta):
        # rotate the boundary direction about the edge (x axis)
        ang = math.atan2(d[2], d[1]) + delta
        rx = np.array([[20.0, edge_pt[1] + R * math.cos(ang), edge_pt[2] + R * math.sin(ang)]])
        return _wedge_total_field(os_, g, tx, rx, 1e9, extra_keys=[spec_key(0, 0, [face])])

    rk = tuple(spec_key(0, 0, [face]))
    assert (rk in at(-1e-6)[1]) != (rk in at(1e-6)[1])
    go_jump = abs(at(-1e-6)[1].get(rk, 0) - at(1e-6)[1].get(rk, 0))
    assert abs(_jump(at)) < 1e-5 * go_jump


def test_keller_point_equal_angles_and_discovery():
    """Diffraction discovery on a box: captured edges yield valid diffraction
    paths whose Keller points make equal angles with the edge (Keller's law)."""
    sc = city.tiny_wedge(size=40.0, height=30.0)
    tx = np.array([[-30.0, 20.0, 40.0]])
    rx = np.array([[60.0, 70.0, 1.5], [20.0, -30.0, 5.0]])
    os_, fr, res = _discover(sc, tx, rx, 200000, 1, diffraction=True)
    g = os_.geometry(np.zeros((0, 3, 4)))
    dk = res.keys[res.keys[:, 2] == 2]
    assert len(dk) >= 2
    for row, p in zip(res.keys, res.points):
        if row[2] != 2:
            continue
        e = row[4]
        ev = g.edge_p[e, 3:] - g.edge_p[e, :3]
        ev /= np.linalg.norm(ev)
        q = p[0]
        si = (q - tx[0]) / np.linalg.norm(q - tx[0])
        so = (rx[row[1]] - q) / np.linalg.norm(rx[row[1]] - q)
        assert abs(si @ ev - so @ ev) < 1e-12


# --------------------------------------------------------------------------
# scene preprocessing
# --------------------------------------------------------------------------

def test_wedge_edges_of_boxes():
    sc = city.tiny_wedge()
    os_ = O.OracleScene(sc)
    assert os_.E == 8
    assert np.allclose(os_.edge_n, 1.5)
    lens = sorted(np.linalg.norm(sc.verts[os_.edges[:, 0]] - sc.verts[os_.edges[:, 1]], axis=1))
    assert np.allclose(lens, [30, 30, 30, 30, 40, 40, 40, 40])


def test_wedge_edges_city_with_t_junctions():
    """Walls split in 3 columns with an unsplit roof (T-junctions on the roof
    border): still 8 wedge edges per building and 12 per vehicle."""
    p = city.CityParams(3, "uniform", 3, 1, 1, 5, 1, np.array([[0.0, 0.0]]), None, 0, 4, False, 0, 0, 7)
    sc = city.make_city(p)
    os_ = O.OracleScene(sc)
    assert os_.E == 9 * 8 + 5 * 12
    assert np.allclose(os_.edge_n, 1.5)
    assert np.all(os_.edges[:, 2] < os_.edges[:, 3])


def test_world_transform_rounding_rule():
    """Dynamic vertices: float32(((r0 x + r1 y) + r2 z) + t) in double, no FMA."""
    w = city.workload("district")
    sc = w.scene
    os_ = O.OracleScene(sc)
    fr = sc.frame(0.37)
    g = os_.geometry(fr.obj_xform)
    dyn = np.nonzero(os_.vdyn >= 0)[0]
    x = sc.verts[dyn].astype(np.float64)
    m = fr.obj_xform[os_.vdyn[dyn]]
    want = np.empty_like(x)
    for i in range(3):
        s = m[:, i, 0] * x[:, 0]
        s = s + m[:, i, 1] * x[:, 1]
        s = s + m[:, i, 2] * x[:, 2]
        s = s + m[:, i, 3]
        want[:, i] = s
    assert np.array_equal(g.verts[dyn], want.astype(np.float32))
    st = np.nonzero(os_.vdyn < 0)[0]
    assert np.array_equal(g.verts[st], sc.verts[st])


def test_fibonacci_lattice_covers_sphere():
    N = 4000
    d = O.fib_dirs(N, np.arange(N)).astype(np.float64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    assert np.linalg.norm(d.mean(0)) < 1e-3
    z = d[:, 2]
    assert np.allclose(z, 1 - (2 * np.arange(N) + 1) / N, atol=1e-7)
    # every direction's nearest neighbour is within twice the mean spacing
    g = d @ d.T
    np.fill_diagonal(g, -2)
    nn = np.arccos(np.clip(g.max(1), -1, 1))
    assert nn.max() < 2 * math.sqrt(4 * math.pi / N)
