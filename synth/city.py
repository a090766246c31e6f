"""Synthetic Manhattan-grid cities, vehicles, transmitters and receivers.

The paper evaluates on its own 2x2 km city model with SUMO traffic (Section IV),
neither of which is available; these seeded generators stand in for them with
the shapes the workloads name: box buildings on a regular block grid, metal
box vehicles moving along lanes, rooftop transmitters, pedestrian and
vehicle-mounted receivers.

Conventions (x east, y north, z up, origin at the city centre):
  * block pitch 50 m = 30 m building footprint + 20 m street;
  * the ground is one face at z = 0, tiled into one 2-triangle quad per block
    so that no triangle spans the whole city;
  * buildings are closed-on-top boxes (four walls + roof, no bottom) wound
    counter-clockwise seen from outside; walls are split into
    ``wall_cols x wall_rows`` panels and the roof into ``roof_div^2`` cells;
    vertices are shared inside one building, never across objects;
  * every vertex coordinate is rounded to float32 at generation, so
    axis-aligned faces are exactly planar;
  * vehicles are 4.5 x 1.8 x 1.5 m boxes (12 triangles, z in [0.3, 1.8]),
    driving in lanes at +-3.5 m from the street centre line with periodic wrap
    at the city edge (no collision model);
  * pedestrian receivers stand at z = 1.5 m on sidewalks at +-8.5 m from the
    street centre line; vehicle receivers sit 0.2 m above the roof centre line.

Random draw order (numpy default_rng(seed)): building heights, then per
vehicle (axis, line, side, position, speed), then receivers per vehicle, then
per pedestrian (axis, line, side, position, speed, direction), then street
receivers (workloads that place receivers on centre lines).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

PITCH = 50.0
FOOT = 30.0
LANE = 3.5
SIDEWALK = 8.5
VEH_L, VEH_W, VEH_Z0, VEH_Z1 = 4.5, 1.8, 0.3, 1.8
RX_PED_Z = 1.5
RX_VEH_DZ = 0.2

EPS_GROUND = 15.0 - 1.5j
EPS_CONCRETE = 5.3 - 0.2j
EPS_METAL = 1.0 - 1.0e6j
# Table I's reflection coefficients (magnitudes) of walls and of metal
REFL_WALL = 0.8
REFL_METAL = 0.9


@dataclasses.dataclass
class Frame:
    """Per-frame motion state (all float64)."""

    t: float
    obj_xform: np.ndarray  # [O_d, 3, 4] rigid transform of each dynamic object
    obj_vel: np.ndarray  # [O_d, 3] translational velocity, m/s
    tx_pos: np.ndarray  # [N_tx, 3]
    tx_vel: np.ndarray  # [N_tx, 3]
    rx_pos: np.ndarray  # [N_rx, 3]
    rx_vel: np.ndarray  # [N_rx, 3]
    tx_orient: np.ndarray  # [N_tx, 2] dipole (theta, phi), rad


@dataclasses.dataclass
class Scene:
    verts: np.ndarray  # f32 [V, 3]; local coordinates for vertices of dynamic objects
    tris: np.ndarray  # i32 [T, 3]
    tri_face: np.ndarray  # i32 [T]
    face_object: np.ndarray  # i32 [F]
    face_material: np.ndarray  # i32 [F]
    object_dynamic: np.ndarray  # u8 [O]
    materials: np.ndarray  # c128 [M], eps_r = eps' - j eps''
    extent: float  # half width of the ground square, m
    # motion model
    tx_pos: np.ndarray  # f64 [N_tx, 3]
    veh: Dict[str, np.ndarray]  # per vehicle: axis, coord, sign, s0, speed, obj
    rx_kind: np.ndarray  # i32 [N_rx]: 0 static/pedestrian, 1 vehicle-mounted
    rx_veh: np.ndarray  # i32 [N_rx]: vehicle index (kind 1)
    rx_off: np.ndarray  # f64 [N_rx]: offset along the vehicle length (kind 1)
    rx_ped: Dict[str, np.ndarray]  # per receiver (kind 0): axis, coord, s0, vel, z
    building_heights: Optional[np.ndarray] = None
    name: str = ""
    # per material: 0 = Fresnel from the permittivity, g > 0 = constant reflection coefficient magnitude
    material_refl: Optional[np.ndarray] = None

    @property
    def n_tx(self) -> int:
        return int(self.tx_pos.shape[0])

    @property
    def n_rx(self) -> int:
        return int(self.rx_kind.shape[0])

    @property
    def n_dynamic(self) -> int:
        return int(self.object_dynamic.sum())

    def frame(self, t: float) -> Frame:
        w = self.extent
        nv = len(self.veh["axis"])
        xf = np.zeros((nv, 3, 4))
        vel = np.zeros((nv, 3))
        vpos = np.zeros((nv, 3))
        rot = np.zeros((nv, 3, 3))
        for i in range(nv):
            axis = int(self.veh["axis"][i])
            sign = float(self.veh["sign"][i])
            s = _wrap(self.veh["s0"][i] + sign * self.veh["speed"][i] * t, w)
            r = _heading(axis, sign)
            p = np.zeros(3)
            p[axis] = s
            p[1 - axis] = self.veh["coord"][i]
            xf[i, :, :3] = r
            xf[i, :, 3] = p
            v = np.zeros(3)
            v[axis] = sign * self.veh["speed"][i]
            vel[i] = v
            vpos[i] = p
            rot[i] = r
        nrx = self.n_rx
        rx = np.zeros((nrx, 3))
        rv = np.zeros((nrx, 3))
        ped = self.rx_ped
        for j in range(nrx):
            if self.rx_kind[j] == 1:
                i = int(self.rx_veh[j])
                local = np.array([self.rx_off[j], 0.0, VEH_Z1 + RX_VEH_DZ])
                rx[j] = rot[i] @ local + vpos[i]
                rv[j] = vel[i]
            else:
                axis = int(ped["axis"][j])
                sp = float(ped["vel"][j])
                s = _wrap(ped["s0"][j] + sp * t, w) if sp != 0.0 else ped["s0"][j]
                rx[j, axis] = s
                rx[j, 1 - axis] = ped["coord"][j]
                rx[j, 2] = ped["z"][j]
                rv[j, axis] = sp
        ntx = self.n_tx
        return Frame(
            t=float(t),
            obj_xform=xf,
            obj_vel=vel,
            tx_pos=self.tx_pos.copy(),
            tx_vel=np.zeros((ntx, 3)),
            rx_pos=rx,
            rx_vel=rv,
            tx_orient=np.zeros((ntx, 2)),
        )


def _wrap(s: float, w: float) -> float:
    return float((s + w) % (2.0 * w) - w)


def _heading(axis: int, sign: float) -> np.ndarray:
    """Exact rotation taking the vehicle's local +x to the driving direction."""
    if axis == 0:
        return np.diag([sign, sign, 1.0])
    return np.array([[0.0, -sign, 0.0], [sign, 0.0, 0.0], [0.0, 0.0, 1.0]])


class _MeshBuilder:
    def __init__(self) -> None:
        self.verts: List[np.ndarray] = []
        self.tris: List[np.ndarray] = []
        self.tri_face: List[np.ndarray] = []
        self.face_object: List[int] = []
        self.face_material: List[int] = []
        self.object_dynamic: List[int] = []
        self.nv = 0

    def new_object(self, dynamic: bool) -> int:
        self.object_dynamic.append(1 if dynamic else 0)
        return len(self.object_dynamic) - 1

    def add(self, verts: np.ndarray, tris: np.ndarray, tri_local_face: np.ndarray,
            obj: int, face_mats: Sequence[int]) -> None:
        f0 = len(self.face_object)
        for m in face_mats:
            self.face_object.append(obj)
            self.face_material.append(int(m))
        self.verts.append(np.asarray(verts, np.float32))
        self.tris.append(np.asarray(tris, np.int64) + self.nv)
        self.tri_face.append(np.asarray(tri_local_face, np.int64) + f0)
        self.nv += len(verts)

    def finish(self) -> Tuple[np.ndarray, ...]:
        return (
            np.concatenate(self.verts).astype(np.float32),
            np.concatenate(self.tris).astype(np.int32),
            np.concatenate(self.tri_face).astype(np.int32),
            np.asarray(self.face_object, np.int32),
            np.asarray(self.face_material, np.int32),
            np.asarray(self.object_dynamic, np.uint8),
        )


def _grid_quads(nu: int, nv: int, idx) -> List[Tuple[int, int, int]]:
    """Two triangles per grid cell; idx(i, j) gives vertex ids; CCW order assumed."""
    out = []
    for i in range(nu):
        for j in range(nv):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            out.append((a, b, c))
            out.append((a, c, d))
    return out


def box_template(cols: int, rows: int, roof: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Unit-box building mesh (walls + roof, no bottom) in grid coordinates.

    Returns integer-lattice vertex coordinates (gx/cols, gy/cols, gz/rows as
    fractions), triangles and local face ids (0 south, 1 east, 2 north, 3 west,
    4 roof).  The roof is split ``roof x roof``; wall tops are split ``cols``;
    when ``roof != cols`` the roof border meets wall tops in T-junctions whose
    vertices lie exactly on the shared edge line.
    """
    key: Dict[Tuple[float, float, float], int] = {}
    verts: List[Tuple[float, float, float]] = []

    def vid(x: float, y: float, z: float) -> int:
        k = (x, y, z)
        if k not in key:
            key[k] = len(verts)
            verts.append(k)
        return key[k]

    tris: List[Tuple[int, int, int]] = []
    faces: List[int] = []
    u = [i / cols for i in range(cols + 1)]
    h = [k / rows for k in range(rows + 1)]
    # south wall y=0, outward -y: CCW seen from -y means (x right, z up)
    walls = [
        (0, lambda a, z: (a, 0.0, z)),  # south, x increasing
        (1, lambda a, z: (1.0, a, z)),  # east, y increasing
        (2, lambda a, z: (1.0 - a, 1.0, z)),  # north, x decreasing
        (3, lambda a, z: (0.0, 1.0 - a, z)),  # west, y decreasing
    ]
    for fid, pt in walls:
        quads = _grid_quads(cols, rows, lambda i, j, pt=pt: vid(*pt(u[i], h[j])))
        tris += quads
        faces += [fid] * len(quads)
    r = [i / roof for i in range(roof + 1)]
    quads = _grid_quads(roof, roof, lambda i, j: vid(r[i], r[j], 1.0))
    tris += quads
    faces += [4] * len(quads)
    return np.array(verts, np.float64), np.array(tris, np.int64), np.array(faces, np.int64)


def vehicle_template() -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Local vehicle box, length along +x, centred on x and y; 6 faces, 12 triangles."""
    x0, x1 = -VEH_L / 2, VEH_L / 2
    y0, y1 = -VEH_W / 2, VEH_W / 2
    z0, z1 = VEH_Z0, VEH_Z1
    v = np.array([
        [x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
        [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1],
    ])
    quads = [
        (0, 3, 2, 1),  # bottom, -z
        (4, 5, 6, 7),  # top, +z
        (0, 1, 5, 4),  # -y
        (1, 2, 6, 5),  # +x
        (2, 3, 7, 6),  # +y
        (3, 0, 4, 7),  # -x
    ]
    tris, faces = [], []
    for f, (a, b, c, d) in enumerate(quads):
        tris += [(a, b, c), (a, c, d)]
        faces += [f, f]
    return v, np.array(tris, np.int64), np.array(faces, np.int64)


def _ground(mb: _MeshBuilder, n: int, w: float, mat: int) -> None:
    obj = mb.new_object(False)
    xs = [-w + i * PITCH for i in range(n + 1)]
    verts = np.array([(x, y, 0.0) for y in xs for x in xs])
    idx = lambda i, j: j * (n + 1) + i  # noqa: E731
    tris = _grid_quads(n, n, idx)
    mb.add(verts, np.array(tris), np.zeros(len(tris), np.int64), obj, [mat])


@dataclasses.dataclass
class CityParams:
    n_blocks: int
    heights: str  # "uniform" (10..40 m) or "lognormal" (median 25, sigma 0.5, clip 5..150)
    wall_cols: int
    wall_rows: int
    roof_div: int
    n_vehicles: int
    n_tx: int
    tx_sites: Optional[np.ndarray]  # [n_tx, 2] or None (explicit tx_fixed)
    tx_fixed: Optional[np.ndarray]
    n_rx_vehicle: int
    n_rx_ped: int
    ped_moving: bool
    n_rx_street: int
    facade_classes: int  # 0: one concrete material; k>0: k facade materials
    seed: int


def make_city(p: CityParams, name: str = "") -> Scene:
    rng = np.random.default_rng(p.seed)
    n = p.n_blocks
    w = n * PITCH / 2.0
    nb = n * n
    if p.heights == "uniform":
        hts = rng.uniform(10.0, 40.0, nb)
    else:
        hts = np.clip(np.exp(rng.normal(math.log(25.0), 0.5, nb)), 5.0, 150.0)
    hts = hts.astype(np.float32).astype(np.float64)

    if p.facade_classes:
        mats = [EPS_GROUND, EPS_METAL] + [complex(4.0 + k, -(0.1 + 0.05 * k)) for k in range(p.facade_classes)]
        m_ground, m_metal = 0, 1
        m_facade = lambda b: 2 + (b % p.facade_classes)  # noqa: E731
    else:
        mats = [EPS_GROUND, EPS_CONCRETE, EPS_METAL]
        m_ground, m_metal = 0, 2
        m_facade = lambda b: 1  # noqa: E731

    mb = _MeshBuilder()
    _ground(mb, n, w, m_ground)
    tv, tt, tf = box_template(p.wall_cols, p.wall_rows, p.roof_div)
    for b in range(nb):
        bi, bj = b % n, b // n
        x0 = -w + bi * PITCH + (PITCH - FOOT) / 2
        y0 = -w + bj * PITCH + (PITCH - FOOT) / 2
        v = np.empty_like(tv)
        v[:, 0] = x0 + tv[:, 0] * FOOT
        v[:, 1] = y0 + tv[:, 1] * FOOT
        v[:, 2] = tv[:, 2] * hts[b]
        obj = mb.new_object(False)
        mb.add(v, tt, tf, obj, [m_facade(b)] * 5)

    # vehicles
    lines = np.array([-w + k * PITCH for k in range(1, n)])
    nveh = p.n_vehicles
    veh = {k: np.zeros(nveh) for k in ("axis", "coord", "sign", "s0", "speed", "obj")}
    vv, vt, vf = vehicle_template()
    for i in range(nveh):
        axis = int(rng.integers(0, 2))
        line = float(lines[int(rng.integers(0, len(lines)))])
        side = int(rng.integers(0, 2))
        s0 = float(rng.uniform(-w, w))
        speed = float(rng.uniform(5.0, 20.0))
        sign = 1.0 if side == 0 else -1.0
        # +x traffic south of an x-street, +y traffic east of a y-street
        off = -LANE if (axis == 0) == (side == 0) else LANE
        if axis == 1:
            off = LANE if side == 0 else -LANE
        veh["axis"][i], veh["coord"][i], veh["sign"][i] = axis, line + off, sign
        veh["s0"][i], veh["speed"][i] = s0, speed
        obj = mb.new_object(True)
        veh["obj"][i] = obj
        mb.add(vv, vt, vf, obj, [m_metal] * 6)

    verts, tris, tri_face, face_object, face_material, object_dynamic = mb.finish()

    # receivers
    kind, rveh, roff = [], [], []
    if p.n_rx_vehicle and nveh:
        base = p.n_rx_vehicle // nveh
        extra = p.n_rx_vehicle - base * nveh
        per = np.full(nveh, base)
        per[rng.permutation(nveh)[:extra]] += 1
        for i in range(nveh):
            offs = {1: [0.0], 2: [-1.5, 1.5], 3: [-1.5, 0.0, 1.5]}.get(int(per[i]), list(np.linspace(-1.5, 1.5, int(per[i]))))
            for o in offs:
                kind.append(1)
                rveh.append(i)
                roff.append(float(o))
    nped = p.n_rx_ped
    ped = {k: np.zeros(len(kind) + nped + p.n_rx_street) for k in ("axis", "coord", "s0", "vel", "z")}
    for j in range(nped):
        axis = int(rng.integers(0, 2))
        line = float(lines[int(rng.integers(0, len(lines)))])
        side = -1.0 if int(rng.integers(0, 2)) == 0 else 1.0
        s0 = float(rng.uniform(-w, w))
        sp = float(rng.uniform(0.5, 1.5))
        dirn = -1.0 if int(rng.integers(0, 2)) == 0 else 1.0
        k = len(kind)
        kind.append(0)
        rveh.append(-1)
        roff.append(0.0)
        ped["axis"][k], ped["coord"][k], ped["s0"][k] = axis, line + side * SIDEWALK, s0
        ped["vel"][k] = dirn * sp if p.ped_moving else 0.0
        ped["z"][k] = RX_PED_Z
    for j in range(p.n_rx_street):
        axis = int(rng.integers(0, 2))
        line = float(lines[int(rng.integers(0, len(lines)))])
        s0 = float(rng.uniform(-w, w))
        k = len(kind)
        kind.append(0)
        rveh.append(-1)
        roff.append(0.0)
        ped["axis"][k], ped["coord"][k], ped["s0"][k] = axis, line, s0
        ped["z"][k] = RX_PED_Z

    # transmitters: roof + 5 m on the building nearest each site
    if p.tx_fixed is not None:
        txp = np.asarray(p.tx_fixed, np.float64).reshape(-1, 3)
    else:
        centres = np.array([(-w + (b % n) * PITCH + PITCH / 2, -w + (b // n) * PITCH + PITCH / 2) for b in range(nb)])
        txp = np.zeros((p.n_tx, 3))
        for i, site in enumerate(p.tx_sites):
            b = int(np.argmin(((centres - site[None, :]) ** 2).sum(1)))
            txp[i] = (centres[b, 0], centres[b, 1], hts[b] + 5.0)

    return Scene(
        verts=verts, tris=tris, tri_face=tri_face, face_object=face_object,
        face_material=face_material, object_dynamic=object_dynamic,
        materials=np.asarray(mats, np.complex128), extent=w, tx_pos=txp, veh=veh,
        rx_kind=np.asarray(kind, np.int32), rx_veh=np.asarray(rveh, np.int32),
        rx_off=np.asarray(roff, np.float64), rx_ped=ped, building_heights=hts, name=name,
    )


@dataclasses.dataclass
class WorkloadConfig:
    name: str
    scene: Scene
    rays_per_tx: int
    max_reflections: int
    diffraction: bool
    freqs_hz: Tuple[float, ...]
    n_frames: int
    frame_dt: float = 0.01
    discover_every: int = 10
    diff_max_leg: float = 250.0


def _lattice(vals: Sequence[float]) -> np.ndarray:
    return np.array([(x, y) for y in vals for x in vals], np.float64)


def workload(name: str) -> WorkloadConfig:
    """The named workloads: toy, district, city, adjoint (batched cities via ``batch_city``)."""
    if name == "toy":  # 200x200 m static toy city, 1 Tx, 16 Rx, 10k rays, K=3
        p = CityParams(4, "uniform", 1, 1, 1, 0, 1, None, np.array([[0.0, 0.0, 25.0]]), 0, 0, False, 16, 0, 1)
        return WorkloadConfig(name, make_city(p, name), 10_000, 3, False, (28e9,), 1)
    if name == "district":  # 1x1 km, 200 vehicles, 4 Tx, 1000 Rx, 1M rays/Tx, K=4 + diffraction
        p = CityParams(20, "uniform", 3, 1, 1, 200, 4, _lattice([-250.0, 250.0]), None, 500, 500, False, 0, 0, 2)
        return WorkloadConfig(name, make_city(p, name), 1_000_000, 4, True, (28e9,), 100)
    if name == "city":  # 2x2 km, 2000 vehicles, 16 Tx, 10k Rx, 16M rays, K=5 + diffraction
        p = CityParams(40, "lognormal", 3, 2, 3, 2000, 16, _lattice([-750.0, -250.0, 250.0, 750.0]), None,
                       5000, 5000, True, 0, 0, 3)
        return WorkloadConfig(name, make_city(p, name), 1_000_000, 5, True, (3.5e9, 28e9), 60)
    if name == "adjoint":  # district scene with 8 material classes
        p = CityParams(20, "uniform", 3, 1, 1, 200, 4, _lattice([-250.0, 250.0]), None, 500, 500, False, 0, 6, 2)
        return WorkloadConfig(name, make_city(p, name), 1_000_000, 4, True, (28e9,), 10)
    raise KeyError(name)


WORKLOADS = ("toy", "district", "city", "adjoint")


def batch_city(i: int) -> WorkloadConfig:
    """City ``i`` (seed i) of the 64-city batched workload: uneven sizes."""
    rng = np.random.default_rng(1000 + i)
    nbld = int(rng.integers(100, 2001))
    nveh = int(rng.integers(0, 2001))
    nrx = int(rng.integers(50, 5001))
    rays = int(round(math.exp(rng.uniform(math.log(65536), math.log(4 * 1048576))) / 1024.0)) * 1024
    ntx = 1 + (i % 4)
    n = int(math.ceil(math.sqrt(nbld)))
    nrv = nrx // 2 if nveh else 0
    sites = np.array([[(-1) ** k * n * PITCH / 4, (-1) ** (k // 2) * n * PITCH / 4] for k in range(ntx)])
    p = CityParams(n, "uniform", 3, 1, 1, nveh, ntx, sites, None, nrv, nrx - nrv, False, 0, 0, i)
    sc = make_city(p, f"batch{i}")
    return WorkloadConfig(f"batch{i}", sc, max(1024, rays // ntx), 4, False, (28e9,), 20)


def table3_street(distance: float, speed: float, rays_per_tx: int = 1_000_000, n_blocks: int = 16,
                  seed: int = 7) -> WorkloadConfig:
    """Table III's scenario: one vehicle carrying a receiver drives along a
    street at ``speed`` m/s past a roadside transmitter that is ``distance``
    metres away at t = 0; 30 GHz; Table I's constant reflection coefficients
    (0.8 for the buildings and the ground, 0.9 for the metal vehicle).

    The paper gives only the speeds, the distances and the carrier; the
    street is this generator's: an east-west street 20 m wide between two
    rows of ``n_blocks`` box buildings (30 m footprints, 20 m cross streets,
    heights uniform in 15..35 m), the transmitter at (20, 8, 2) on the north
    kerb, the vehicle in the south lane (y = -2) heading east with its
    receiver 2 m above the road.  At distance 10 the vehicle is abeam the
    transmitter (line of sight perpendicular to the motion); otherwise it
    starts sqrt(distance^2 - 100) m west of it, approaching.
    """
    rng = np.random.default_rng(seed)
    w = n_blocks * PITCH / 2.0
    hts = rng.uniform(15.0, 35.0, 2 * n_blocks).astype(np.float32).astype(np.float64)
    mb = _MeshBuilder()
    m_wall, m_metal = 0, 1
    _ground(mb, n_blocks, w, m_wall)
    tv, tt, tf = box_template(1, 1, 1)
    for side in range(2):
        y0 = 10.0 if side == 0 else -10.0 - FOOT
        for i in range(n_blocks):
            x0 = -w + i * PITCH + (PITCH - FOOT) / 2
            v = np.empty_like(tv)
            v[:, 0] = x0 + tv[:, 0] * FOOT
            v[:, 1] = y0 + tv[:, 1] * FOOT
            v[:, 2] = tv[:, 2] * hts[side * n_blocks + i]
            mb.add(v, tt, tf, mb.new_object(False), [m_wall] * 5)
    vv, vt, vf = vehicle_template()
    obj = mb.new_object(True)
    mb.add(vv, vt, vf, obj, [m_metal] * 6)
    verts, tris, tri_face, face_object, face_material, object_dynamic = mb.finish()
    lane = -2.0
    tx = np.array([[20.0, 8.0, VEH_Z1 + RX_VEH_DZ]])
    lateral = tx[0, 1] - lane
    s0 = tx[0, 0] - math.sqrt(max(distance * distance - lateral * lateral, 0.0))
    veh = {"axis": np.zeros(1), "coord": np.array([lane]), "sign": np.ones(1), "s0": np.array([s0]),
           "speed": np.array([float(speed)]), "obj": np.array([float(obj)])}
    sc = Scene(
        verts=verts, tris=tris, tri_face=tri_face, face_object=face_object, face_material=face_material,
        object_dynamic=object_dynamic, materials=np.asarray([EPS_CONCRETE, EPS_METAL], np.complex128),
        extent=w, tx_pos=tx, veh=veh, rx_kind=np.ones(1, np.int32), rx_veh=np.zeros(1, np.int32),
        rx_off=np.zeros(1), rx_ped={k: np.zeros(1) for k in ("axis", "coord", "s0", "vel", "z")},
        building_heights=hts, name=f"table3_v{speed:g}_d{distance:g}",
        material_refl=np.array([REFL_WALL, REFL_METAL]),
    )
    return WorkloadConfig(sc.name, sc, rays_per_tx, 4, True, (30e9,), 1)


# ---------------------------------------------------------------------------
# tiny scenes with closed-form answers (used by the oracle's pins)
# ---------------------------------------------------------------------------

def _static_scene(verts, tris, tri_face, face_object, n_obj, mats, tx, extent, face_mat=None) -> Scene:
    nf = int(max(tri_face) + 1)
    return Scene(
        verts=np.asarray(verts, np.float32), tris=np.asarray(tris, np.int32),
        tri_face=np.asarray(tri_face, np.int32), face_object=np.asarray(face_object, np.int32),
        face_material=np.asarray(face_mat if face_mat is not None else [0] * nf, np.int32),
        object_dynamic=np.zeros(n_obj, np.uint8), materials=np.asarray(mats, np.complex128),
        extent=extent, tx_pos=np.asarray(tx, np.float64).reshape(-1, 3),
        veh={k: np.zeros(0) for k in ("axis", "coord", "sign", "s0", "speed", "obj")},
        rx_kind=np.zeros(0, np.int32), rx_veh=np.zeros(0, np.int32), rx_off=np.zeros(0),
        rx_ped={k: np.zeros(0) for k in ("axis", "coord", "s0", "vel", "z")},
    )


def with_static_rx(sc: Scene, rx: np.ndarray) -> Scene:
    """Copy of ``sc`` with explicit static receivers at ``rx`` [N, 3]."""
    rx = np.asarray(rx, np.float64).reshape(-1, 3)
    n = len(rx)
    axis = np.zeros(n)
    ped = {"axis": axis, "coord": rx[:, 1].copy(), "s0": rx[:, 0].copy(), "vel": np.zeros(n), "z": rx[:, 2].copy()}
    return dataclasses.replace(sc, rx_kind=np.zeros(n, np.int32), rx_veh=np.full(n, -1, np.int32),
                               rx_off=np.zeros(n), rx_ped=ped, extent=max(sc.extent, float(np.abs(rx[:, :2]).max()) + 1.0))


def tiny_ground(half: float = 500.0, eps: complex = EPS_GROUND) -> Scene:
    """A single ground face (2 triangles) at z = 0."""
    v = [(-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0)]
    return _static_scene(v, [(0, 1, 2), (0, 2, 3)], [0, 0], [0], 1, [eps], [0, 0, 10], half)


def tiny_ground_wall(half: float = 500.0, wall_x: float = 50.0, wall_h: float = 400.0,
                     eps_g: complex = EPS_GROUND, eps_w: complex = EPS_CONCRETE) -> Scene:
    """Ground at z = 0 plus one large vertical wall in the plane x = wall_x."""
    v = [(-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0),
         (wall_x, -half, 0), (wall_x, half, 0), (wall_x, half, wall_h), (wall_x, -half, wall_h)]
    tris = [(0, 1, 2), (0, 2, 3), (4, 5, 6), (4, 6, 7)]
    return _static_scene(v, tris, [0, 0, 1, 1], [0, 1], 2, [eps_g, eps_w], [0, 0, 10], half, face_mat=[0, 1])


def tiny_canyon(gap: float = 20.0, length: float = 4000.0, height: float = 4000.0,
                eps: complex = EPS_CONCRETE) -> Scene:
    """Two tall parallel walls at y = -gap/2 and y = +gap/2, no ground."""
    h, y0, y1 = length / 2, -gap / 2, gap / 2
    v = [(-h, y0, -height / 2), (h, y0, -height / 2), (h, y0, height / 2), (-h, y0, height / 2),
         (-h, y1, -height / 2), (h, y1, -height / 2), (h, y1, height / 2), (-h, y1, height / 2)]
    tris = [(0, 1, 2), (0, 2, 3), (4, 6, 5), (4, 7, 6)]
    return _static_scene(v, tris, [0, 0, 1, 1], [0, 1], 2, [eps], [0, 0, 0], h)


def tiny_box_ground(size: float = 40.0, height: float = 30.0, half: float = 500.0, refl=(1.0, 1.0)) -> Scene:
    """One box building [0,size]^2 x [0,height] (walls + roof, object 1) on a
    ground face at z = 0 (object 0); materials 0 ground, 1 building, with
    constant reflection coefficients ``refl``."""
    tv, tt, tf = box_template(1, 1, 1)
    v = np.empty_like(tv)
    v[:, 0] = tv[:, 0] * size
    v[:, 1] = tv[:, 1] * size
    v[:, 2] = tv[:, 2] * height
    g = [(-half, -half, 0), (half, -half, 0), (half, half, 0), (-half, half, 0)]
    verts = np.concatenate([np.asarray(g, np.float64), v])
    tris = np.concatenate([np.array([(0, 1, 2), (0, 2, 3)]), np.asarray(tt) + 4])
    faces = np.concatenate([[0, 0], np.asarray(tf) + 1])
    sc = _static_scene(verts, tris, faces, [0] + [1] * 5, 2, [EPS_GROUND, EPS_CONCRETE], [-50, size / 2, 10], half,
                       face_mat=[0] + [1] * 5)
    return dataclasses.replace(sc, material_refl=np.asarray(refl, np.float64))


def tiny_wedge(size: float = 40.0, height: float = 30.0, eps: complex = EPS_METAL,
               cols: int = 1, rows: int = 1) -> Scene:
    """One box building [0,size]^2 x [0,height] (walls + roof), no ground."""
    tv, tt, tf = box_template(cols, rows, cols)
    v = np.empty_like(tv)
    v[:, 0] = tv[:, 0] * size
    v[:, 1] = tv[:, 1] * size
    v[:, 2] = tv[:, 2] * height
    return _static_scene(v, tt, tf, [0] * 5, 1, [eps], [-50, size / 2, 10], 4 * size)
