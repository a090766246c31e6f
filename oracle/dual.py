"""Oracle gradient by forward-mode dual numbers.

TEST INFRASTRUCTURE ONLY (as ``oracle.py``): only ``tests/`` import this
module.  It shares no code with the GPU library.

The paper computes channels, not gradients; the gradients are a reading (an
extension with the path topology held fixed).  This module evaluates, path
by path in plain Python, the same quantities as the C oracle's
``orc_image_points`` and ``orc_eval`` (image method for specular paths,
Keller's point on the edge for diffraction, Fresnel reflection with the
polarisation tracked bounce by bounce, UTD with Luebbers' lossy faces, the
short-dipole or vertical isotropic antenna, Section II-A and Section IV),
but in numbers that carry, beside each value, its derivatives with respect
to

  * the transmitter position (3 real tangents) and the dipole orientation
    theta, phi (2 real tangents): the interaction points are rebuilt from the
    transmitter in the same numbers, so their motion is part of the
    derivative;
  * each material permittivity eps_m (one complex tangent each; the
    amplitude is holomorphic in eps).

For a real loss L of the per-link sums H (and P_coh = P_tx |H|^2) with
cotangent g = G_H + 2 P_tx G_P H, dL/dx = sum Re(conj(g) da/dx) for a real
parameter x and dL/dRe eps + j dL/dIm eps = sum g conj(da/deps).

Derivatives flow through every smooth step; the discrete choices (which
branch of a normal-incidence basis, the integer nearest to a UTD argument,
the shadow-boundary limit) are taken on the values, as the topology is
held fixed.  The value of the UTD transition function F comes from the C
oracle (``utd_F``); its derivative is F'(X) = F (j + 1/(2X)) - j.
"""
from __future__ import annotations

import cmath
import math
from typing import Dict, Optional, Sequence

import numpy as np

from oracle import oracle as O

C0 = O.C0


class Dual:
    """A real or complex value v and its derivatives d (complex array) along
    the tangent directions."""

    __slots__ = ("v", "d")

    def __init__(self, v, d: np.ndarray) -> None:
        self.v = v
        self.d = d

    # arithmetic with duals and with plain numbers
    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.d + o.d)
        return Dual(self.v + o, self.d)

    __radd__ = __add__

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v - o.v, self.d - o.d)
        return Dual(self.v - o, self.d)

    def __rsub__(self, o):
        return Dual(o - self.v, -self.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.d * o.v + o.d * self.v)
        return Dual(self.v * o, self.d * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            q = self.v / o.v
            return Dual(q, (self.d - o.d * q) / o.v)
        return Dual(self.v / o, self.d / o)

    def __rtruediv__(self, o):
        q = o / self.v
        return Dual(q, -self.d * (q / self.v))


def val(x):
    return x.v if isinstance(x, Dual) else x


def _lift(fv, dfv, x):
    """f(x) for a dual x: value fv, chain rule with f'(x) = dfv."""
    if isinstance(x, Dual):
        return Dual(fv, x.d * dfv)
    return fv


def dsqrt(x):
    v = val(x)
    if isinstance(v, complex):
        s = cmath.sqrt(v)
    else:
        s = math.sqrt(v)
    return _lift(s, 0.5 / s if s != 0 else 0.0, x)


def dsin(x):
    v = val(x)
    return _lift(math.sin(v), math.cos(v), x)


def dcos(x):
    v = val(x)
    return _lift(math.cos(v), -math.sin(v), x)


def dacos(x):
    v = val(x)
    return _lift(math.acos(v), -1.0 / math.sqrt(1.0 - v * v), x)


def datan2(y, x):
    yv, xv = val(y), val(x)
    r = math.atan2(yv, xv)
    inv = 1.0 / (xv * xv + yv * yv)
    d = 0.0
    if isinstance(y, Dual):
        d = d + y.d * (xv * inv)
    if isinstance(x, Dual):
        d = d - x.d * (yv * inv)
    return Dual(r, d) if isinstance(d, np.ndarray) else r


def dabs(x):
    return -x if val(x) < 0 else x


# 3-vectors as tuples of numbers or duals
def vadd(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def vsub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def vmul(a, s):
    return (a[0] * s, a[1] * s, a[2] * s)


def vdot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def vcross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def vlen(a):
    return dsqrt(vdot(a, a))


def vnorm(a):
    return vmul(a, 1.0 / vlen(a))


def vval(a):
    return np.array([float(val(x)) for x in a])


# ------------------------------------------------------------------ model --
class _Model:
    """The scene at one frame, with the permittivities as dual numbers."""

    def __init__(self, os_: O.OracleScene, g: O.FrameGeom, nt: int, eps_first: int) -> None:
        self.plane = g.plane
        self.verts = g.verts.astype(np.float64)
        self.edges = os_.edges
        self.edge_n = os_.edge_n
        self.face_material = os_.face_material
        self.refl = os_.material_refl
        self.nt = nt
        mats = os_.materials[:, 0] + 1j * os_.materials[:, 1]
        self.eps = []
        for m, e in enumerate(mats):
            d = np.zeros(nt, np.complex128)
            d[eps_first + m] = 1.0
            self.eps.append(Dual(complex(e), d))

    # material reflection coefficients (TE, TM) at incidence cosine c: a
    # constant magnitude g > 0 with a perfect conductor's signs, else Fresnel
    # for a half space of permittivity eps (principal square root)
    def gammas(self, m: int, c):
        if self.refl[m] > 0.0:
            return -float(self.refl[m]), float(self.refl[m])
        eps = self.eps[m]
        rt = dsqrt(eps - (1.0 - c * c))
        return (c - rt) / (c + rt), (eps * c - rt) / (eps * c + rt)

    def face(self, f: int):
        p = self.plane[f]
        return (float(p[0]), float(p[1]), float(p[2])), float(p[3])

    def wedge(self, e: int):
        row = self.edges[e]
        P0 = tuple(self.verts[row[0]])
        P1 = tuple(self.verts[row[1]])
        ev = np.subtract(P1, P0)
        ln = float(np.linalg.norm(ev))
        e_ = ev / ln
        r0 = self.verts[row[4]] - np.asarray(P0)
        rn = self.verts[row[5]] - np.asarray(P0)
        t0 = r0 - e_ * np.dot(r0, e_)
        t0 = t0 / np.linalg.norm(t0)
        tn = rn - e_ * np.dot(rn, e_)
        tn = tn / np.linalg.norm(tn)
        n0 = np.cross(e_, t0)
        if np.dot(n0, tn) > 0:
            n0 = -n0
        # plain floats: a numpy scalar on the left of a dual would not defer to it
        fl = lambda v: tuple(float(x) for x in v)  # noqa: E731
        return {"P0": fl(P0), "e": fl(e_), "t0": fl(t0), "n0": fl(n0), "n": float(self.edge_n[e]),
                "f0": int(row[2]), "fn": int(row[3])}


def _mirror(p, n, d):
    return vsub(p, vmul(n, 2.0 * (vdot(n, p) - d)))


def _keller(w, a, b):
    """Point of the edge line where the unfolded path a -> Q -> b is
    shortest: the axial coordinates interpolated by the radial distances."""
    za = vdot(vsub(a, w["P0"]), w["e"])
    zb = vdot(vsub(b, w["P0"]), w["e"])
    ra = vlen(vsub(vsub(a, w["P0"]), vmul(w["e"], za)))
    rb = vlen(vsub(vsub(b, w["P0"]), vmul(w["e"], zb)))
    return vadd(w["P0"], vmul(w["e"], za + (zb - za) * ra / (ra + rb)))


def _points(md: _Model, key, s, r):
    """Interaction points of a key (image method / Keller point)."""
    typ, order = int(key[2]), int(key[3])
    if typ == 0:
        return []
    if typ == 1:
        img = [s]
        for i in range(1, order + 1):
            n, d = md.face(int(key[3 + i]))
            img.append(_mirror(img[-1], n, d))
        pts = [None] * order
        cur = r
        for i in range(order, 0, -1):
            n, d = md.face(int(key[3 + i]))
            dv = vsub(img[i], cur)
            cur = vadd(cur, vmul(dv, (d - vdot(n, cur)) / vdot(n, dv)))
            pts[i - 1] = cur
        return pts
    if typ == 2:
        return [_keller(md.wedge(int(key[4])), s, r)]
    rd = typ == 3
    f, e = (int(key[4]), int(key[5])) if rd else (int(key[5]), int(key[4]))
    w = md.wedge(e)
    n, d = md.face(f)
    a = _mirror(s, n, d) if rd else s
    b = r if rd else _mirror(r, n, d)
    Q = _keller(w, a, b)
    dv = vsub(a if rd else b, Q)
    P = vadd(Q, vmul(dv, (d - vdot(n, Q)) / vdot(n, dv)))
    return [P, Q] if rd else [Q, P]


def _antenna(mode, k, th, ph):
    if mode == 1:
        st, ct, sp, cp = dsin(th), dcos(th), dsin(ph), dcos(ph)
        u = (st * cp, st * sp, ct)
        return vmul(vsub(u, vmul(k, vdot(u, k))), math.sqrt(1.5))
    e = vsub((0.0, 0.0, 1.0), vmul(k, k[2]))
    if math.sqrt(float(val(vdot(e, e)))) < 1e-12:
        e = vsub((1.0, 0.0, 0.0), vmul(k, k[0]))
    return vnorm(e)


def _reflect(md: _Model, E, ki, ko, f):
    n, _ = md.face(f)
    if float(val(vdot(n, ki))) > 0:
        n = (-n[0], -n[1], -n[2])
    c = -vdot(ki, n)
    sv = vcross(ki, n)
    if math.sqrt(float(val(vdot(sv, sv)))) < 1e-12:
        sv = vcross(n, (0.0, 0.0, 1.0))
        if np.linalg.norm(sv) < 1e-12:
            sv = vcross(n, (1.0, 0.0, 0.0))
    sv = vnorm(sv)
    pin, pout = vcross(sv, ki), vcross(sv, ko)
    te, tm = md.gammas(int(md.face_material[f]), c)
    es, ep = vdot(sv, E) * te, vdot(pin, E) * tm
    return vadd(vmul(sv, es), vmul(pout, ep))


def _phase(L, lam):
    """exp(-j 2 pi frac(L / lambda)); derivative -j k p dL."""
    x = float(val(L)) / lam
    p = cmath.exp(-2j * math.pi * (x - round(x)))
    return _lift(p, -1j * (2 * math.pi / lam) * p, L)


def _utd_F(X):
    xv = float(val(X))
    if xv <= 0:
        return 0.0
    f = O.utd_F(xv)
    return _lift(f, f * complex(0.5 / xv, 1.0) - 1j, X)


def _utd_term(sg, beta, n, kL):
    N = round((float(val(beta)) + sg * math.pi) / (2 * math.pi * n))
    eps = math.pi + sg * (beta - 2 * math.pi * n * N)
    if abs(float(val(eps))) < 1e-4:
        ev = float(val(eps))
        sgn = 1.0 if ev > 0 else (-1.0 if ev < 0 else 0.0)
        e4 = cmath.exp(1j * math.pi / 4)
        return (dsqrt(2 * math.pi * kL) * sgn - kL * eps * (2 * e4)) * (n * e4)
    c = dcos((2 * math.pi * n * N - beta) * 0.5)
    x = (math.pi + sg * beta) / (2 * n)
    return _utd_F(kL * 2.0 * c * c) * (dcos(x) / dsin(x))


def _utd_D(md: _Model, n, k, L, beta0, php, ph, m0, mn):
    sb = dsin(beta0)
    Cc = (-cmath.exp(-1j * math.pi / 4) / (2 * n * math.sqrt(2 * math.pi * k))) / sb
    kL = L * k
    t1 = _utd_term(+1, ph - php, n, kL)
    t2 = _utd_term(-1, ph - php, n, kL)
    t3 = _utd_term(+1, ph + php, n, kL)
    t4 = _utd_term(-1, ph + php, n, kL)
    r0te, r0tm = md.gammas(m0, sb * dabs(dsin(php)))
    rnte, rntm = md.gammas(mn, sb * dabs(dsin(n * math.pi - ph)))
    return (Cc * (t1 + t2 + rnte * t3 + r0te * t4), Cc * (t1 + t2 + rntm * t3 + r0tm * t4))


def _wedge_angle(w, p):
    v = vsub(p, w["P0"])
    a = datan2(vdot(v, w["n0"]), vdot(v, w["t0"]))
    return a + 2 * math.pi if float(val(a)) < 0 else a


def path_amplitudes(md: _Model, key, s, r, th, ph, ant_mode: int, freqs: Sequence[float]):
    """Amplitudes a_f of one path (duals) and its unfolded length L."""
    typ = int(key[2])
    pts = _points(md, key, s, r)
    amps = []
    if typ in (0, 1):
        P = [s, *pts, r]
        kk, L = [], 0.0
        for i in range(len(P) - 1):
            dv = vsub(P[i + 1], P[i])
            ln = vlen(dv)
            L = L + ln
            kk.append(vmul(dv, 1.0 / ln))
        for fz in freqs:
            lam = C0 / fz
            E = _antenna(ant_mode, kk[0], th, ph)
            for i in range(1, len(P) - 1):
                E = _reflect(md, E, kk[i - 1], kk[i], int(key[3 + i]))
            er = _antenna(0, kk[-1], 0.0, 0.0)
            amps.append(vdot(er, E) * _phase(L, lam) * (lam / (4 * math.pi)) / L)
        return amps, L
    rd, dr = typ == 3, typ == 4
    e = int(key[5]) if rd else int(key[4])
    fr = int(key[4]) if rd else (int(key[5]) if dr else -1)
    w = md.wedge(e)
    P = [s, *pts, r]
    kk, seg, L = [], [], 0.0
    for i in range(len(P) - 1):
        dv = vsub(P[i + 1], P[i])
        ln = vlen(dv)
        seg.append(ln)
        kk.append(vmul(dv, 1.0 / ln))
        L = L + ln
    iq = 1 if rd else 0  # segment arriving at the edge
    si, so = kk[iq], kk[iq + 1]
    sp = seg[0] + seg[1] if rd else seg[0]
    sd = seg[1] + seg[2] if dr else seg[iq + 1]
    cb = vdot(si, w["e"])
    cb = 1.0 if float(val(cb)) > 1 else (-1.0 if float(val(cb)) < -1 else cb)
    beta0 = dacos(cb)
    php, phw = _wedge_angle(w, P[iq]), _wedge_angle(w, P[iq + 2])
    Lp = sd * sp * dsin(beta0) * dsin(beta0) / (sd + sp)
    fp = vmul(vnorm(vcross(w["e"], si)), -1.0)
    bp = vcross(fp, si)
    fo = vnorm(vcross(w["e"], so))
    bo = vcross(fo, so)
    m0, mn = int(md.face_material[w["f0"]]), int(md.face_material[w["fn"]])
    for fz in freqs:
        lam = C0 / fz
        k = 2 * math.pi / lam
        Ds, Dh = _utd_D(md, w["n"], k, Lp, beta0, php, phw, m0, mn)
        E = _antenna(ant_mode, kk[0], th, ph)
        if rd:
            E = _reflect(md, E, kk[0], kk[1], fr)
        Ed = vadd(vmul(bo, -vdot(bp, E) * Ds), vmul(fo, -vdot(fp, E) * Dh))
        if dr:
            Ed = _reflect(md, Ed, kk[1], kk[2], fr)
        er = _antenna(0, kk[-1], 0.0, 0.0)
        spread = (1.0 / sp) * dsqrt(sp / (sd * (sd + sp)))
        amps.append(vdot(er, Ed) * _phase(L, lam) * spread * (lam / (4 * math.pi)))
    return amps, L


N_GEO = 5  # tangents: transmitter x, y, z, theta, phi


def evaluate_dual(os_: O.OracleScene, g: O.FrameGeom, frame, keys: np.ndarray, freqs: Sequence[float],
                  ant_mode: int = 0):
    """Amplitudes and lengths of fixed keys as duals.  Returns (a [n][nf]
    complex values, da [n][nf][5 + M] derivatives, L [n], dL [n][5]).
    Tangents 0..4 refer to the key's own transmitter; 5 + m to eps_m."""
    keys = O.check_keys(os_, keys, len(frame.tx_pos), len(frame.rx_pos))
    M = len(os_.materials)
    nt = N_GEO + M
    md = _Model(os_, g, nt, N_GEO)
    n, nf = len(keys), len(freqs)
    a = np.zeros((n, nf), np.complex128)
    da = np.zeros((n, nf, nt), np.complex128)
    L = np.zeros(n)
    dL = np.zeros((n, N_GEO))

    def seed(v, k):
        d = np.zeros(nt, np.complex128)
        d[k] = 1.0
        return Dual(float(v), d)

    for q, key in enumerate(keys):
        t, rx = int(key[0]), int(key[1])
        s = tuple(seed(frame.tx_pos[t][c], c) for c in range(3))
        r = tuple(float(x) for x in frame.rx_pos[rx])
        th, ph = seed(frame.tx_orient[t][0], 3), seed(frame.tx_orient[t][1], 4)
        amps, Lq = path_amplitudes(md, key, s, r, th, ph, ant_mode, freqs)
        for fi, x in enumerate(amps):
            a[q, fi] = complex(x.v)
            da[q, fi] = x.d
        L[q] = float(Lq.v)
        dL[q] = Lq.d[:N_GEO].real
    return a, da, L, dL


def grad_dual(os_: O.OracleScene, g: O.FrameGeom, frame, keys: np.ndarray, freqs: Sequence[float], G_H: np.ndarray,
              G_P: Optional[np.ndarray], n_rx: int, p_tx: float = O.P_TX_W, ant_mode: int = 0) -> Dict[str, np.ndarray]:
    """Gradients of ``oracle.channel_loss`` (same arguments, same outputs as
    ``oracle.grad_fd``) by forward-mode dual numbers, topology fixed."""
    keys = np.asarray(keys).reshape(-1, O.KEY_W)
    n_tx = len(frame.tx_pos)
    M = len(os_.materials)
    out = {"grad_tx_pos": np.zeros((n_tx, 3)), "grad_tx_orient": np.zeros((n_tx, 2)),
           "grad_eps": np.zeros(M, np.complex128)}
    if len(keys) == 0:
        return out
    a, da, _, _ = evaluate_dual(os_, g, frame, keys, freqs, ant_mode)
    link = keys[:, 0].astype(np.int64) * n_rx + keys[:, 1]
    for fi in range(len(freqs)):
        H = np.zeros(G_H.shape[1], np.complex128)
        np.add.at(H, link, a[:, fi])
        gl = G_H[fi] + (2.0 * p_tx * G_P[fi] * H if G_P is not None else 0.0)
        gq = gl[link]  # cotangent of each path's link
        geo = (np.conj(gq)[:, None] * da[:, fi, :N_GEO]).real
        np.add.at(out["grad_tx_pos"], keys[:, 0], geo[:, :3])
        if ant_mode == 1:
            np.add.at(out["grad_tx_orient"], keys[:, 0], geo[:, 3:5])
        out["grad_eps"] += (gq[:, None] * np.conj(da[:, fi, N_GEO:])).sum(0)
    return out
