"""Oracle: plain FP64 CPU reference of the dynamic SBR EM path search.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg import this module.  It drives the brute
force C routines in ``emrt_oracle.c`` (no acceleration structure, double
precision) and does the bookkeeping that the paper describes in words:

* path discovery from shooting and bouncing rays (Section II-A: direct,
  reflected and diffracted rays),
* the path cache, revalidated every frame and extended on discovery frames,
  invalid paths deleted (Section III-B, the "visibility hash table"),
* per-receiver channel sums: complex gain, received power, delay and Doppler
  with its power-weighted mean and RMS spread (Section III-C Eq (3) and
  Section V-D),
* gradients of a loss of those channels with respect to the permittivities,
  the transmitter positions and the dipole orientation, by central
  differences with the path topology held fixed (a reading: the paper has no
  gradients; ``grad_fd``); ``dual.py`` gives the same gradients by
  forward-mode dual numbers.

It shares no code with the GPU library (``paper_2303_10521_amd``) and never
imports it.  The only common dependency is the seeded input generator
(``synth``), which holds no arithmetic of the method.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "emrt_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

C0 = 299792458.0
P_TX_W = 100.0  # 50 dBm (Section IV)


# address and undefined-behaviour sanitizers (host code only): a build of the
# same source that the pin suite can run under, to show that no pin reads or
# writes outside the oracle's arrays
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(force: bool = False, sanitize: bool = False, out: Optional[str] = None) -> str:
    """Compile the C oracle with gcc (OpenMP, no floating-point contraction);
    with ``sanitize`` into ``out`` with the address and undefined-behaviour
    sanitizers."""
    target = out or _LIB
    if force or sanitize or not os.path.exists(target) or os.path.getmtime(target) < os.path.getmtime(_SRC):
        tmp = target + ".tmp"
        cmd = ["gcc", "-O1" if sanitize else "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", *(SANITIZE_FLAGS if sanitize else []), "-shared", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, target)
    return target


_lib = None


def lib():
    """The oracle's shared library: EMRT_ORACLE_LIB when set (e.g. the
    sanitized build), else the default build next to the source."""
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(os.environ.get("EMRT_ORACLE_LIB") or build())
        _lib.orc_num_threads.restype = ctypes.c_int32
        for name in ("orc_face_planes", "orc_edges", "orc_trace", "orc_validate", "orc_eval", "orc_image_points",
                     "orc_check_keys"):
            getattr(_lib, name).restype = ctypes.c_int32
    return _lib


def _p(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.c_void_p(0)
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ---------------------------------------------------------------------------
# thin wrappers over the C routines (exposed for the pins)
# ---------------------------------------------------------------------------

def fresnel_gamma(eps: complex, cos_theta: float) -> Tuple[complex, complex]:
    out = np.zeros(4)
    lib().orc_fresnel_gamma(ctypes.c_double(eps.real), ctypes.c_double(eps.imag), ctypes.c_double(cos_theta), _p(out))
    return complex(out[0], out[1]), complex(out[2], out[3])


def utd_F(X: float) -> complex:
    out = np.zeros(2)
    lib().orc_utd_F(ctypes.c_double(X), _p(out))
    return complex(out[0], out[1])


def erfcx_diag(v: float) -> complex:
    out = np.zeros(2)
    lib().orc_erfcx_diag(ctypes.c_double(v), _p(out))
    return complex(out[0], out[1])


def utd_D(n, k, L, beta0, php, ph, eps0: complex, epsn: complex) -> Tuple[complex, complex]:
    out = np.zeros(4)
    e0 = np.array([eps0.real, eps0.imag])
    en = np.array([epsn.real, epsn.imag])
    lib().orc_utd_D(*(ctypes.c_double(x) for x in (n, k, L, beta0, php, ph)), _p(e0), _p(en), _p(out))
    return complex(out[0], out[1]), complex(out[2], out[3])


def fib_dirs(N: int, ids: np.ndarray) -> np.ndarray:
    ids = _c(ids, np.int32)
    out = np.zeros((len(ids), 3), np.float32)
    lib().orc_fib_dirs(ctypes.c_int32(N), ctypes.c_int32(len(ids)), _p(ids), _p(out))
    return out


# ---------------------------------------------------------------------------
# scene state
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class FrameGeom:
    verts: np.ndarray  # f32 [V,3] world
    tv: np.ndarray  # f32 [T,9]
    plane: np.ndarray  # f64 [F,4]
    edge_p: np.ndarray  # f64 [E,6]
    sphere: np.ndarray  # f64 [4]


class OracleScene:
    """Static preprocessing of a ``synth.Scene`` (face planes, wedge edges)."""

    def __init__(self, sc) -> None:
        self.sc = sc
        self.verts = _c(sc.verts, np.float32)
        self.tris = _c(sc.tris, np.int32)
        self.tri_face = _c(sc.tri_face, np.int32)
        self.face_object = _c(sc.face_object, np.int32)
        self.face_material = _c(sc.face_material, np.int32)
        self.T = len(self.tris)
        self.F = len(self.face_object)
        dyn = np.asarray(sc.object_dynamic, np.int64)
        rank = np.cumsum(dyn) - 1
        obj_rank = np.where(dyn > 0, rank, -1).astype(np.int32)
        self.face_dyn = _c(obj_rank[self.face_object], np.int32)
        vdyn = np.full(len(self.verts), -1, np.int32)
        vdyn[self.tris.reshape(-1)] = np.repeat(self.face_dyn[self.tri_face], 3)
        self.vdyn = vdyn
        order = np.argsort(self.tri_face, kind="stable")
        self.face_tris = _c(order, np.int32)
        self.face_off = _c(np.concatenate([[0], np.cumsum(np.bincount(self.tri_face, minlength=self.F))]), np.int32)
        cap = 16 * self.F + 16
        out = np.zeros((cap, 6), np.int32)
        wn = np.zeros(cap)
        ne = lib().orc_edges(ctypes.c_int32(len(self.verts)), _p(self.verts), ctypes.c_int32(self.T), _p(self.tris),
                             _p(self.tri_face), ctypes.c_int32(self.F), _p(self.face_object), ctypes.c_int32(cap),
                             _p(out), _p(wn))
        assert 0 <= ne <= cap
        self.edges = out[:ne].copy()
        self.edge_n = wn[:ne].copy()
        self.materials = _c(np.stack([sc.materials.real, sc.materials.imag], 1), np.float64)
        refl = getattr(sc, "material_refl", None)
        self.material_refl = _c(np.zeros(len(sc.materials)) if refl is None else refl, np.float64)

    @property
    def E(self) -> int:
        return len(self.edges)

    def geometry(self, xform: np.ndarray) -> FrameGeom:
        xf = _c(xform if xform.size else np.zeros((1, 3, 4)), np.float64)
        w = np.zeros_like(self.verts)
        lib().orc_world_verts(ctypes.c_int32(len(self.verts)), _p(self.verts), _p(self.vdyn), _p(xf), _p(w))
        tv = _c(w[self.tris].reshape(-1, 9), np.float32)
        plane = np.zeros((self.F, 4))
        rc = lib().orc_face_planes(ctypes.c_int32(self.T), _p(tv), _p(self.tri_face), ctypes.c_int32(self.F), _p(plane))
        assert rc == 0, rc
        ep = np.zeros((self.E, 6))
        if self.E:
            ep[:, :3] = w[self.edges[:, 0]]
            ep[:, 3:] = w[self.edges[:, 1]]
        lo, hi = w.min(0).astype(np.float64), w.max(0).astype(np.float64)
        sph = np.concatenate([(lo + hi) / 2, [np.linalg.norm(hi - lo) / 2 + 1.0]])
        return FrameGeom(w, tv, plane, _c(ep, np.float64), sph)


# ---------------------------------------------------------------------------
# discovery, validation, evaluation, reduction
# ---------------------------------------------------------------------------

def f32(a: np.ndarray) -> np.ndarray:
    """Discovery-side positions: float64 values rounded to float32 and back."""
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass
class TraceResult:
    ray_ids: np.ndarray  # [n]
    hit_tri: np.ndarray  # [n, K+1]
    robust: np.ndarray  # [n] bool
    captures: np.ndarray  # [m, 3] (ray index into ray_ids, bounce, rx)
    edge_hits: np.ndarray  # [q, 3] (ray index, edge, segment: 0 direct, 1 after one reflection)


def trace(os_: OracleScene, g: FrameGeom, tx_pos: np.ndarray, N: int, ray_ids: np.ndarray, K: int,
          rx_pos: np.ndarray, k_rx: float = 1.0, diffraction: int = 0, want_robust: bool = True) -> TraceResult:
    """Bounce loop for one transmitter over the launch directions ``ray_ids`` of N
    (diffraction: 0 off, 1 edge capture on the first segment, 2 on the first two)."""
    ray_ids = _c(ray_ids, np.int32)
    n = len(ray_ids)
    txf = _c(f32(tx_pos), np.float64)
    rxf = _c(f32(rx_pos), np.float64)
    hit = np.zeros((n, K + 1), np.int32)
    rob = np.zeros(n, np.uint8)
    cap = max(1024, 8 * n)
    ecap = max(1024, 4 * n) if diffraction else 1
    while True:
        caps = np.zeros((cap, 3), np.int32)
        edges = np.zeros((ecap, 3), np.int32)
        ncap = ctypes.c_int64(0)
        nedge = ctypes.c_int64(0)
        lib().orc_trace(
            ctypes.c_int32(os_.T), _p(g.tv), _p(os_.tri_face), _p(g.plane), _p(txf), ctypes.c_int32(N),
            ctypes.c_int32(n), _p(ray_ids), ctypes.c_int32(K), ctypes.c_int32(len(rxf)), _p(rxf),
            ctypes.c_double(k_rx), ctypes.c_int32(os_.E if diffraction else 0), _p(g.edge_p),
            ctypes.c_int32(int(diffraction)), ctypes.c_int32(1 if want_robust else 0), _p(g.sphere),
            _p(hit), _p(rob), ctypes.c_int64(cap), _p(caps), ctypes.byref(ncap), ctypes.c_int64(ecap), _p(edges),
            ctypes.byref(nedge))
        if ncap.value <= cap and nedge.value <= ecap:
            break
        cap = max(cap, int(ncap.value) + 16)
        ecap = max(ecap, int(nedge.value) + 16)
    return TraceResult(ray_ids, hit, rob.astype(bool), caps[: ncap.value].copy(), edges[: nedge.value].copy())


KEY_W = 9  # tx, rx, type, order, id0..id4
LOS, SPEC, DIFF, REFL_DIFF, DIFF_REFL = 0, 1, 2, 3, 4


def spec_keys(os_: OracleScene, tr: TraceResult, tx: int) -> Dict[tuple, bool]:
    """Unique (tx, rx, face sequence) keys from captures, with 'robustly discovered'."""
    out: Dict[tuple, bool] = {}
    faces = np.where(tr.hit_tri >= 0, os_.tri_face[np.maximum(tr.hit_tri, 0)], -1)
    for ri, b, rx in tr.captures:
        seq = tuple(int(f) for f in faces[ri, :b])
        ids = seq + (-1,) * (5 - len(seq))
        key = (tx, int(rx), SPEC, int(b)) + ids
        out[key] = out.get(key, False) or bool(tr.robust[ri])
    return out


def spec_keys_from_receiver(os_: OracleScene, tr: TraceResult, rx: int) -> Dict[tuple, bool]:
    """Keys from a launch at receiver ``rx`` whose spheres sit on the
    transmitters: a capture at transmitter t after b reflections off faces
    f_1..f_b (in launch order) is the path from t to rx over f_b..f_1."""
    out: Dict[tuple, bool] = {}
    faces = np.where(tr.hit_tri >= 0, os_.tri_face[np.maximum(tr.hit_tri, 0)], -1)
    for ri, b, t in tr.captures:
        seq = tuple(int(f) for f in faces[ri, :b][::-1])
        ids = seq + (-1,) * (5 - len(seq))
        key = (int(t), rx, SPEC, int(b)) + ids
        out[key] = out.get(key, False) or bool(tr.robust[ri])
    return out


def reflected_edges(os_: OracleScene, tr: TraceResult) -> Dict[Tuple[int, int], bool]:
    """(face, edge) pairs lit by second segments: the ray reflected off the
    face of its first hit and then passed the edge."""
    out: Dict[Tuple[int, int], bool] = {}
    for ri, e, b in tr.edge_hits:
        if b != 1:
            continue
        f = int(os_.tri_face[tr.hit_tri[ri, 0]])
        out[(f, int(e))] = out.get((f, int(e)), False) or bool(tr.robust[ri])
    return out


def illuminated_edges(tr: TraceResult) -> Dict[int, bool]:
    out: Dict[int, bool] = {}
    for ri, e in tr.edge_hits[tr.edge_hits[:, 2] == 0, :2]:
        out[int(e)] = out.get(int(e), False) or bool(tr.robust[ri])
    return out


class MalformedKey(ValueError):
    """A key row outside the scene's index ranges (see ``check_keys``)."""


def check_keys(os_: OracleScene, keys: np.ndarray, n_tx: int, n_rx: int) -> np.ndarray:
    """Raise MalformedKey naming the first key row that is not well formed:
    tx in [0, n_tx), rx in [0, n_rx), type 0 with order 0, type 1 with order
    1..5 and face ids in [0, F), type 2 with order 1 and an edge id in [0, E),
    types 3 / 4 with order 2 and (face, edge) / (edge, face).  The C routines
    make the same check and never index with a malformed key."""
    keys = _c(np.asarray(keys).reshape(-1, KEY_W), np.int32)
    bad = np.zeros(len(keys), np.uint8)
    nb = lib().orc_check_keys(ctypes.c_int32(len(keys)), _p(keys), ctypes.c_int32(n_tx), ctypes.c_int32(n_rx),
                              ctypes.c_int32(os_.F), ctypes.c_int32(os_.E), _p(bad))
    if nb:
        i = int(np.nonzero(bad)[0][0])
        raise MalformedKey(f"{nb} malformed key(s); first: row {i} = {keys[i].tolist()} "
                           f"(n_tx {n_tx}, n_rx {n_rx}, faces {os_.F}, edges {os_.E})")
    return keys


def validate(os_: OracleScene, g: FrameGeom, keys: np.ndarray, tx_pos: np.ndarray, rx_pos: np.ndarray,
             diff_max_leg: float = 250.0):
    keys = check_keys(os_, keys, len(tx_pos), len(rx_pos))
    n = len(keys)
    valid = np.zeros(n, np.uint8)
    amb = np.zeros(n, np.uint8)
    tri = np.zeros((n, 5), np.int32)
    pts = np.zeros((n, 5, 3))
    edges = os_.edges if os_.E else np.zeros((1, 6), np.int32)
    en = os_.edge_n if os_.E else np.zeros(1)
    nb = lib().orc_validate(ctypes.c_int32(os_.T), _p(g.tv), _p(os_.tri_face), _p(g.plane), ctypes.c_int32(os_.F),
                            ctypes.c_int32(os_.E), ctypes.c_int32(len(tx_pos)), ctypes.c_int32(len(rx_pos)),
                            _p(os_.face_off), _p(os_.face_tris), _p(g.verts), _p(_c(edges, np.int32)),
                            _p(_c(en, np.float64)), _p(_c(tx_pos, np.float64)), _p(_c(rx_pos, np.float64)),
                            ctypes.c_double(diff_max_leg), ctypes.c_int32(n), _p(keys), _p(valid), _p(amb), _p(tri),
                            _p(pts))
    assert nb == 0, nb
    return valid.astype(bool), amb.astype(bool), tri, pts


def evaluate(os_: OracleScene, g: FrameGeom, keys: np.ndarray, pts: np.ndarray, frame, freqs: Sequence[float],
             ant_mode: int = 0, obj_vel: Optional[np.ndarray] = None, materials: Optional[np.ndarray] = None):
    """Fields of validated keys at the given interaction points.  ``materials``
    (complex [M]) overrides the scene permittivities."""
    keys = check_keys(os_, keys, len(frame.tx_pos), len(frame.rx_pos))
    n = len(keys)
    nf = len(freqs)
    a = np.zeros((n, nf, 2))
    tau = np.zeros(n)
    fd = np.zeros((n, nf))
    aod = np.zeros((n, 2))
    aoa = np.zeros((n, 2))
    ov = obj_vel if obj_vel is not None else frame.obj_vel
    ov = _c(ov if ov.size else np.zeros((1, 3)), np.float64)
    edges = os_.edges if os_.E else np.zeros((1, 6), np.int32)
    en = os_.edge_n if os_.E else np.zeros(1)
    if materials is None:
        mats = os_.materials
    else:
        m = np.asarray(materials, np.complex128)
        mats = _c(np.stack([m.real, m.imag], 1), np.float64)
    nb = lib().orc_eval(ctypes.c_int32(n), _p(keys), ctypes.c_int32(os_.F), ctypes.c_int32(os_.E),
                   ctypes.c_int32(len(frame.tx_pos)), ctypes.c_int32(len(frame.rx_pos)),
                   _p(_c(pts, np.float64)), _p(g.plane), _p(os_.face_material),
                   _p(os_.face_dyn), _p(ov), _p(mats), _p(os_.material_refl), _p(g.verts), _p(_c(edges, np.int32)),
                   _p(_c(en, np.float64)), _p(_c(frame.tx_pos, np.float64)), _p(_c(frame.tx_vel, np.float64)),
                   _p(_c(frame.tx_orient, np.float64)), _p(_c(frame.rx_pos, np.float64)),
                   _p(_c(frame.rx_vel, np.float64)), ctypes.c_int32(ant_mode), ctypes.c_int32(nf),
                   _p(_c(np.asarray(freqs, np.float64), np.float64)), _p(a), _p(tau), _p(fd), _p(aod), _p(aoa))
    assert nb == 0, nb
    return a[..., 0] + 1j * a[..., 1], tau, fd, aod, aoa


def image_points(os_: OracleScene, g: FrameGeom, keys: np.ndarray, tx_pos: np.ndarray,
                 rx_pos: np.ndarray) -> np.ndarray:
    """Interaction points of fixed keys: image method / Keller point with no
    containment, range or occlusion test (the topology is held fixed)."""
    keys = check_keys(os_, keys, len(tx_pos), len(rx_pos))
    n = len(keys)
    pts = np.zeros((n, 5, 3))
    edges = os_.edges if os_.E else np.zeros((1, 6), np.int32)
    en = os_.edge_n if os_.E else np.zeros(1)
    nb = lib().orc_image_points(ctypes.c_int32(n), _p(keys), ctypes.c_int32(os_.F), ctypes.c_int32(os_.E),
                                ctypes.c_int32(len(tx_pos)), ctypes.c_int32(len(rx_pos)), _p(g.plane), _p(g.verts),
                                _p(_c(edges, np.int32)), _p(_c(en, np.float64)), _p(_c(tx_pos, np.float64)),
                                _p(_c(rx_pos, np.float64)), _p(pts))
    assert nb == 0, nb
    return pts


class _FrameView:
    """A frame with some fields replaced (for finite differences)."""

    def __init__(self, fr, **kw) -> None:
        for name in ("t", "obj_xform", "obj_vel", "tx_pos", "tx_vel", "rx_pos", "rx_vel", "tx_orient"):
            setattr(self, name, kw.get(name, getattr(fr, name)))


def channel_loss(os_: OracleScene, g: FrameGeom, frame, keys: np.ndarray, freqs: Sequence[float], G_H: np.ndarray,
                 G_P: Optional[np.ndarray], n_rx: int, p_tx: float = P_TX_W, ant_mode: int = 0,
                 materials: Optional[np.ndarray] = None) -> float:
    """L = sum_{f, link} Re(conj(G_H) H) + G_P P_tx |H|^2, with H the coherent
    sum of the fields of the fixed keys (points rebuilt from the frame).
    G_H complex [nf, n_links], G_P real [nf, n_links] or None."""
    keys = np.asarray(keys).reshape(-1, KEY_W)
    if len(keys) == 0:
        return 0.0
    pts = image_points(os_, g, keys, frame.tx_pos, frame.rx_pos)
    a, _, _, _, _ = evaluate(os_, g, keys, pts, frame, freqs, ant_mode, materials=materials)
    link = keys[:, 0].astype(np.int64) * n_rx + keys[:, 1]
    total = 0.0
    for fi in range(len(freqs)):
        H = np.zeros(G_H.shape[1], np.complex128)
        np.add.at(H, link, a[:, fi])
        total += float(np.sum((np.conj(G_H[fi]) * H).real))
        if G_P is not None:
            total += float(np.sum(G_P[fi] * p_tx * np.abs(H) ** 2))
    return total


def grad_fd(os_: OracleScene, g: FrameGeom, frame, keys: np.ndarray, freqs: Sequence[float], G_H: np.ndarray,
            G_P: Optional[np.ndarray], n_rx: int, p_tx: float = P_TX_W, ant_mode: int = 0, h_pos: float = 1e-6,
            h_ang: float = 1e-6, h_eps_rel: float = 1e-6) -> Dict[str, np.ndarray]:
    """Gradients of ``channel_loss`` by central differences with the topology
    fixed (the keys are not revalidated):
      grad_tx_pos [n_tx, 3]   dL/d(transmitter position), step h_pos metres;
      grad_tx_orient [n_tx, 2] dL/d(theta, phi) of the dipole, step h_ang rad
                               (zero for the vertical isotropic antenna);
      grad_eps [M] complex     dL/d Re(eps) + j dL/d Im(eps), steps
                               h_eps_rel |eps| on each part separately.
    Only the keys of transmitter t change with its position or orientation,
    and the loss is separable per link, so those differences use its keys."""
    keys = np.asarray(keys).reshape(-1, KEY_W)
    n_tx = len(frame.tx_pos)
    mats = os_.materials[:, 0] + 1j * os_.materials[:, 1]
    out = {"grad_tx_pos": np.zeros((n_tx, 3)), "grad_tx_orient": np.zeros((n_tx, 2)),
           "grad_eps": np.zeros(len(mats), np.complex128)}

    def L(fr, ks, m=None):
        return channel_loss(os_, g, fr, ks, freqs, G_H, G_P, n_rx, p_tx, ant_mode, m)

    for t in range(n_tx):
        kt = keys[keys[:, 0] == t]
        if len(kt) == 0:
            continue
        for c in range(3):
            tp, tm = frame.tx_pos.copy(), frame.tx_pos.copy()
            tp[t, c] += h_pos
            tm[t, c] -= h_pos
            out["grad_tx_pos"][t, c] = (L(_FrameView(frame, tx_pos=tp), kt) - L(_FrameView(frame, tx_pos=tm), kt)) / (
                2 * h_pos)
        if ant_mode == 1:
            for c in range(2):
                op, om = frame.tx_orient.copy(), frame.tx_orient.copy()
                op[t, c] += h_ang
                om[t, c] -= h_ang
                out["grad_tx_orient"][t, c] = (L(_FrameView(frame, tx_orient=op), kt)
                                               - L(_FrameView(frame, tx_orient=om), kt)) / (2 * h_ang)
    for m in range(len(mats)):
        h = h_eps_rel * abs(mats[m])
        parts = []
        for d in (h, 1j * h):
            mp, mm = mats.copy(), mats.copy()
            mp[m] += d
            mm[m] -= d
            parts.append((L(frame, keys, mp) - L(frame, keys, mm)) / (2 * h))
        out["grad_eps"][m] = parts[0] + 1j * parts[1]
    return out


def reduce_links(keys: np.ndarray, a: np.ndarray, tau: np.ndarray, fd: np.ndarray, n_tx: int, n_rx: int,
                 p_tx: float = P_TX_W) -> Dict[str, np.ndarray]:
    """Per-link channel sums (Section V-D: mean Doppler shift, RMS Doppler spread):
    H = sum a, P_coh = P_tx |H|^2, P_inc = P_tx sum |a|^2, power-weighted mean and
    RMS of delay and Doppler (weights |a|^2 at each frequency)."""
    nf = a.shape[1] if a.ndim == 2 else 1
    nl = n_tx * n_rx
    link = keys[:, 0].astype(np.int64) * n_rx + keys[:, 1] if len(keys) else np.zeros(0, np.int64)
    out = {
        "H": np.zeros((nf, nl), np.complex128), "P_coh": np.zeros((nf, nl)), "P_inc": np.zeros((nf, nl)),
        "tau_mean": np.zeros((nf, nl)), "tau_rms": np.zeros((nf, nl)), "fd_mean": np.zeros((nf, nl)),
        "fd_rms": np.zeros((nf, nl)), "n_paths": np.bincount(link, minlength=nl).astype(np.int32),
        "los": np.zeros(nl, bool),
    }
    if len(keys):
        out["los"][link[keys[:, 2] == LOS]] = True
    for fi in range(nf):
        af = a[:, fi]
        w = np.abs(af) ** 2
        H = np.zeros(nl, np.complex128)
        np.add.at(H, link, af)
        sw = np.bincount(link, weights=w, minlength=nl)
        out["H"][fi] = H
        out["P_coh"][fi] = p_tx * np.abs(H) ** 2
        out["P_inc"][fi] = p_tx * sw
        safe = np.where(sw > 0, sw, 1.0)
        for name, x in (("tau", tau), ("fd", fd[:, fi])):
            m = np.bincount(link, weights=w * x, minlength=nl) / safe
            var = np.bincount(link, weights=w * (x - m[link]) ** 2, minlength=nl) / safe
            out[name + "_mean"][fi] = np.where(sw > 0, m, 0.0)
            out[name + "_rms"][fi] = np.where(sw > 0, np.sqrt(np.maximum(var, 0.0)), 0.0)
    return out


@dataclasses.dataclass
class OracleFrame:
    keys: np.ndarray  # [n, 9] valid keys, sorted
    robust: np.ndarray  # [n] key robustly discovered (or LoS / cached)
    ambiguous: np.ndarray  # [n] validation within a margin
    tri_ids: np.ndarray
    points: np.ndarray
    a: np.ndarray
    tau: np.ndarray
    fd: np.ndarray
    aod: np.ndarray
    aoa: np.ndarray
    channels: Dict[str, np.ndarray]
    traces: List[TraceResult]
    candidates: np.ndarray  # all candidate keys that were validated
    cand_valid: np.ndarray
    cand_amb: np.ndarray


def los_keys(n_tx: int, n_rx: int) -> np.ndarray:
    k = np.full((n_tx * n_rx, KEY_W), -1, np.int32)
    k[:, 0] = np.repeat(np.arange(n_tx), n_rx)
    k[:, 1] = np.tile(np.arange(n_rx), n_tx)
    k[:, 2] = LOS
    k[:, 3] = 0
    return k


def diffraction_candidates(os_: OracleScene, g: FrameGeom, tx: int, illum: Dict[int, bool], rx_pos: np.ndarray,
                           diff_max_leg: float) -> Dict[tuple, bool]:
    """(tx, edge, rx) candidates for illuminated edges: every receiver within
    diff_max_leg of the edge segment (the Keller point lies on the segment)."""
    out: Dict[tuple, bool] = {}
    for e, rob in illum.items():
        p0 = g.edge_p[e, :3]
        p1 = g.edge_p[e, 3:]
        d = p1 - p0
        l2 = float(d @ d)
        s = np.clip(((rx_pos - p0) @ d) / l2, 0.0, 1.0)
        dist = np.linalg.norm(rx_pos - (p0 + s[:, None] * d), axis=1)
        for r in np.nonzero(dist <= diff_max_leg)[0]:
            out[(tx, int(r), DIFF, 1, e, -1, -1, -1, -1)] = rob
    return out


def diffraction_candidates_from_receiver(g: FrameGeom, rx: int, illum: Dict[int, bool], rx_pos: np.ndarray,
                                         n_tx: int, diff_max_leg: float) -> Dict[tuple, bool]:
    """(tx, edge, rx) candidates for edges lit from receiver ``rx``: every
    transmitter, when rx lies within diff_max_leg of the edge segment."""
    out: Dict[tuple, bool] = {}
    r = np.asarray(rx_pos[rx], np.float64)
    for e, rob in illum.items():
        p0 = g.edge_p[e, :3]
        d = g.edge_p[e, 3:] - p0
        s = float(np.clip(((r - p0) @ d) / float(d @ d), 0.0, 1.0))
        if np.linalg.norm(r - (p0 + s * d)) <= diff_max_leg:
            for tx in range(n_tx):
                out[(tx, rx, DIFF, 1, e, -1, -1, -1, -1)] = rob
    return out


def refl_diff_candidates(g: FrameGeom, tx: int, lit: Dict[Tuple[int, int], bool], rx_pos: np.ndarray,
                         diff_max_leg: float) -> Dict[tuple, bool]:
    """Reflection-then-diffraction candidates (tx, rx, face, edge) for (face,
    edge) pairs lit from transmitter tx: every receiver within diff_max_leg of
    the edge segment."""
    out: Dict[tuple, bool] = {}
    for (f, e), rob in lit.items():
        p0 = g.edge_p[e, :3]
        d = g.edge_p[e, 3:] - p0
        s = np.clip(((rx_pos - p0) @ d) / float(d @ d), 0.0, 1.0)
        dist = np.linalg.norm(rx_pos - (p0 + s[:, None] * d), axis=1)
        for r in np.nonzero(dist <= diff_max_leg)[0]:
            out[(tx, int(r), REFL_DIFF, 2, f, e, -1, -1, -1)] = rob
    return out


def sort_keys(keys: np.ndarray) -> np.ndarray:
    """Row-lexicographic order of (tx, rx, type, order, id0..id4)."""
    if len(keys) == 0:
        return np.zeros(0, np.int64)
    return np.lexsort([keys[:, c] for c in reversed(range(KEY_W))])


def run_frame(os_: OracleScene, frame, N: int, K: int, freqs: Sequence[float], ray_ids: Optional[np.ndarray] = None,
              diffraction: int = 0, discover: bool = True, cache: Optional[np.ndarray] = None,
              k_rx: float = 1.0, diff_max_leg: float = 250.0, want_robust: bool = True, ant_mode: int = 0,
              p_tx: float = P_TX_W, rx_sources: Optional[Sequence[int]] = None) -> OracleFrame:
    """One frame of the method: discovery (optional) on the given launch
    directions of every transmitter, union with the cache, exact validation of
    every candidate plus line of sight for every link, field evaluation and
    per-link reduction (Sections II-A, III-B, III-C).

    With ``rx_sources`` the discovery launches from those receivers instead
    (the backward launch of Section II-A): the same lattice of N directions
    from each listed receiver, spheres k_rx sqrt(4 pi / N) (L + s) around the
    transmitters, keys reversed into transmitter-to-receiver order, and edges
    lit by the first segments proposing every transmitter.

    diffraction: 0 off; 1 first-order edge diffraction; 2 also one reflection
    combined with one diffraction -- from the transmitters, (face, edge) pairs
    lit by second segments propose reflection-then-diffraction paths to every
    receiver within diff_max_leg of the edge; from receivers, the same pairs
    seen from the receiver propose the reverse, diffraction-then-reflection
    paths, from every transmitter."""
    g = os_.geometry(frame.obj_xform)
    n_tx, n_rx = len(frame.tx_pos), len(frame.rx_pos)
    cand: Dict[tuple, bool] = {}
    traces: List[TraceResult] = []
    if discover and rx_sources is not None:
        ids = np.arange(N, dtype=np.int32) if ray_ids is None else _c(ray_ids, np.int32)
        for r in sorted({int(x) for x in rx_sources}):
            tr = trace(os_, g, frame.rx_pos[r], N, ids, K, frame.tx_pos, k_rx, diffraction, want_robust)
            traces.append(tr)
            for k, v in spec_keys_from_receiver(os_, tr, r).items():
                cand[k] = cand.get(k, False) or v
            if diffraction:
                for k, v in diffraction_candidates_from_receiver(g, r, illuminated_edges(tr), frame.rx_pos, n_tx,
                                                                 diff_max_leg).items():
                    cand[k] = cand.get(k, False) or v
            if diffraction == 2:
                for (f, e), v in reflected_edges(os_, tr).items():
                    for t in range(n_tx):
                        k = (t, r, DIFF_REFL, 2, e, f, -1, -1, -1)
                        cand[k] = cand.get(k, False) or v
    elif discover:
        ids = np.arange(N, dtype=np.int32) if ray_ids is None else _c(ray_ids, np.int32)
        for tx in range(n_tx):
            tr = trace(os_, g, frame.tx_pos[tx], N, ids, K, frame.rx_pos, k_rx, diffraction, want_robust)
            traces.append(tr)
            for k, v in spec_keys(os_, tr, tx).items():
                cand[k] = cand.get(k, False) or v
            if diffraction:
                for k, v in diffraction_candidates(os_, g, tx, illuminated_edges(tr), frame.rx_pos,
                                                   diff_max_leg).items():
                    cand[k] = cand.get(k, False) or v
            if diffraction == 2:
                for k, v in refl_diff_candidates(g, tx, reflected_edges(os_, tr), frame.rx_pos,
                                                 diff_max_leg).items():
                    cand[k] = cand.get(k, False) or v
    if cache is not None:
        for row in np.asarray(cache).reshape(-1, KEY_W):
            k = tuple(int(x) for x in row)
            cand[k] = True
    ck = np.array(list(cand.keys()), np.int32).reshape(-1, KEY_W)
    cr = np.array(list(cand.values()), bool)
    allk = np.concatenate([los_keys(n_tx, n_rx), ck])
    allr = np.concatenate([np.ones(n_tx * n_rx, bool), cr])
    valid, amb, tri, pts = validate(os_, g, allk, frame.tx_pos, frame.rx_pos, diff_max_leg)
    vk, vr, va, vt, vp = allk[valid], allr[valid], amb[valid], tri[valid], pts[valid]
    o = sort_keys(vk)
    vk, vr, va, vt, vp = vk[o], vr[o], va[o], vt[o], vp[o]
    a, tau, fd, aod, aoa = evaluate(os_, g, vk, vp, frame, freqs, ant_mode)
    ch = reduce_links(vk, a, tau, fd, n_tx, n_rx, p_tx)
    return OracleFrame(vk, vr, va, vt, vp, a, tau, fd, aod, aoa, ch, traces, allk, valid, amb)


def cache_of(fr: OracleFrame) -> np.ndarray:
    """The cache after a frame: every valid non-LoS key (LoS is re-tested each frame)."""
    return fr.keys[fr.keys[:, 2] != LOS].copy()
