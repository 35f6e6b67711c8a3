"""Seeded synthetic inputs: room surface meshes, wall admittances, sources, receivers.

This module generates *inputs only*.  It holds no boundary-integral arithmetic
(no centroids, normals, areas, kernels or quadrature): both the HIP path and the
CPU oracle compute their own geometry from the vertex/triangle arrays made here.

Rooms follow the problem statement of the paper (Section 2: a room bounded by a
closed surface S with a locally reacting impedance wall, normals pointing out of
the room, a unit monopole source inside).  Meshing recipe: every planar
rectangle a x b gets ceil(a/h) x ceil(b/h) cells, each split along the same
diagonal into two flat triangles, ordered so that (v1-v0)x(v2-v0) points out of
the fluid.  Admittance beta = 1/zeta (Eq. sp3/sp4; rigid is beta = 0) is real,
one value per planar face, drawn from U[0.05, 0.3] in face order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SOUND_SPEED = 343.0  # m/s

SEED_MESH, SEED_BETA, SEED_SOURCE, SEED_RECEIVERS = 0, 1, 2, 3


@dataclass
class Rect:
    """Planar rectangle o + s*u + t*v, s,t in [0,1]; `out` is the unit normal out of the fluid."""
    o: tuple
    u: tuple
    v: tuple
    out: tuple
    face: int          # planar-face id (one admittance draw per face)
    fixed_beta: complex | None = None   # e.g. an open doorway modelled as beta = 1


@dataclass
class Room:
    name: str
    rects: list
    nfaces: int
    boxes: list                      # fluid = union(boxes) minus solids
    solids: list = field(default_factory=list)
    vertices: np.ndarray = None      # (nv, 3) float64
    triangles: np.ndarray = None     # (nt, 3) int64
    tri_face: np.ndarray = None      # (nt,) int32 planar-face id
    tri_rect: np.ndarray = None      # (nt,) int32 rectangle id
    beta: np.ndarray = None          # (nt,) complex128 admittance per triangle
    h: float = 0.0

    @property
    def n(self) -> int:
        return int(self.triangles.shape[0])


def _mesh_rect(r: Rect, h: float):
    o, u, v = (np.asarray(a, float) for a in (r.o, r.u, r.v))
    na = max(1, math.ceil(np.linalg.norm(u) / h - 1e-9))
    nb = max(1, math.ceil(np.linalg.norm(v) / h - 1e-9))
    s = np.linspace(0.0, 1.0, na + 1)
    t = np.linspace(0.0, 1.0, nb + 1)
    S, T = np.meshgrid(s, t, indexing="ij")
    V = o[None, :] + S.reshape(-1, 1) * u[None, :] + T.reshape(-1, 1) * v[None, :]
    vid = lambda i, j: i * (nb + 1) + j
    I, J = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
    I, J = I.ravel(), J.ravel()
    p00, p10, p01, p11 = vid(I, J), vid(I + 1, J), vid(I, J + 1), vid(I + 1, J + 1)
    t1 = np.stack([p00, p10, p11], 1)
    t2 = np.stack([p00, p11, p01], 1)
    tri = np.stack([t1, t2], 1).reshape(-1, 3)
    if np.dot(np.cross(u, v), np.asarray(r.out, float)) < 0:
        tri = tri[:, [0, 2, 1]]
    return V, tri


def _build(room: Room, h: float, seed_beta: int = SEED_BETA) -> Room:
    Vs, Ts, F, R = [], [], [], []
    off = 0
    for ir, r in enumerate(room.rects):
        V, T = _mesh_rect(r, h)
        Vs.append(V)
        Ts.append(T + off)
        off += V.shape[0]
        F.append(np.full(T.shape[0], r.face, np.int32))
        R.append(np.full(T.shape[0], ir, np.int32))
    room.vertices = np.concatenate(Vs)
    room.triangles = np.concatenate(Ts).astype(np.int64)
    room.tri_face = np.concatenate(F)
    room.tri_rect = np.concatenate(R)
    rng = np.random.default_rng(seed_beta)
    face_beta = rng.uniform(0.05, 0.3, size=room.nfaces)
    beta = face_beta[room.tri_face].astype(np.complex128)
    for ir, r in enumerate(room.rects):
        if r.fixed_beta is not None:
            beta[room.tri_rect == ir] = r.fixed_beta
    room.beta = beta
    room.h = h
    return room


def _box_rects(x0, x1, y0, y1, z0, z1, face0, inward=False):
    """Six faces of an axis-aligned box.  Normals point out of the box, or into it if `inward`."""
    s = -1.0 if inward else 1.0
    dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
    return [
        Rect((x0, y0, z0), (dx, 0, 0), (0, dy, 0), (0, 0, -s), face0 + 0),  # z = z0
        Rect((x0, y0, z1), (dx, 0, 0), (0, dy, 0), (0, 0, s), face0 + 1),   # z = z1
        Rect((x0, y0, z0), (dx, 0, 0), (0, 0, dz), (0, -s, 0), face0 + 2),  # y = y0
        Rect((x0, y1, z0), (dx, 0, 0), (0, 0, dz), (0, s, 0), face0 + 3),   # y = y1
        Rect((x0, y0, z0), (0, dy, 0), (0, 0, dz), (-s, 0, 0), face0 + 4),  # x = x0
        Rect((x1, y0, z0), (0, dy, 0), (0, 0, dz), (s, 0, 0), face0 + 5),   # x = x1
    ]


def shoebox(lx: float, ly: float, lz: float, h: float, seed_beta: int = SEED_BETA) -> Room:
    room = Room("shoebox", _box_rects(0, lx, 0, ly, 0, lz, 0), 6, [(0, lx, 0, ly, 0, lz)])
    return _build(room, h, seed_beta)


def lroom(h: float, baffle: bool = True, doorway: bool = True, seed_beta: int = SEED_BETA) -> Room:
    """L-shaped room: box A [0,6]x[0,5]x[0,3] union box B [6,10]x[0,3]x[0,3]; optional
    7 cm thick baffle slab [3.00,3.07]x[1.5,3.5]x[0.5,2.5] and a 1x2 m doorway patch
    (beta = 1) on the wall x = 0, y in [2,3], z in [0,2]."""
    R = []
    # floor (face 0) and ceiling (face 1), each two rectangles
    R += [Rect((0, 0, 0), (6, 0, 0), (0, 5, 0), (0, 0, -1), 0), Rect((6, 0, 0), (4, 0, 0), (0, 3, 0), (0, 0, -1), 0)]
    R += [Rect((0, 0, 3), (6, 0, 0), (0, 5, 0), (0, 0, 1), 1), Rect((6, 0, 3), (4, 0, 0), (0, 3, 0), (0, 0, 1), 1)]
    R += [Rect((0, 0, 0), (10, 0, 0), (0, 0, 3), (0, -1, 0), 2)]   # y = 0
    R += [Rect((10, 0, 0), (0, 3, 0), (0, 0, 3), (1, 0, 0), 3)]    # x = 10
    R += [Rect((6, 3, 0), (4, 0, 0), (0, 0, 3), (0, 1, 0), 4)]     # y = 3 (x in [6,10])
    R += [Rect((6, 3, 0), (0, 2, 0), (0, 0, 3), (1, 0, 0), 5)]     # x = 6 (y in [3,5])
    R += [Rect((0, 5, 0), (6, 0, 0), (0, 0, 3), (0, 1, 0), 6)]     # y = 5
    if doorway:
        R += [Rect((0, 0, 0), (0, 2, 0), (0, 0, 3), (-1, 0, 0), 7),
              Rect((0, 3, 0), (0, 2, 0), (0, 0, 3), (-1, 0, 0), 7),
              Rect((0, 2, 2), (0, 1, 0), (0, 0, 1), (-1, 0, 0), 7),
              Rect((0, 2, 0), (0, 1, 0), (0, 0, 2), (-1, 0, 0), 7, fixed_beta=1.0 + 0j)]
    else:
        R += [Rect((0, 0, 0), (0, 5, 0), (0, 0, 3), (-1, 0, 0), 7)]
    nfaces = 8
    solids = []
    if baffle:
        R += _box_rects(3.00, 3.07, 1.5, 3.5, 0.5, 2.5, nfaces, inward=True)
        nfaces += 6
        solids.append((3.00, 3.07, 1.5, 3.5, 0.5, 2.5))
    room = Room("lroom", R, nfaces, [(0, 6, 0, 5, 0, 3), (6, 10, 0, 3, 0, 3)], solids)
    return _build(room, h, seed_beta)


def icosphere(radius: float, subdiv: int, beta: complex = 0.0) -> Room:
    """Sphere of radius `radius` (fluid inside, normals outward) from a subdivided icosahedron."""
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(subdiv):
        cache, F2 = {}, []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            F2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = F2
    Vt = np.array(V) * radius
    T = np.array(F, np.int64)
    # orient outward
    c = Vt[T].mean(1)
    nrm = np.cross(Vt[T[:, 1]] - Vt[T[:, 0]], Vt[T[:, 2]] - Vt[T[:, 0]])
    flip = (nrm * c).sum(1) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    room = Room("sphere", [], 1, [])
    room.vertices, room.triangles = Vt, T
    room.tri_face = np.zeros(T.shape[0], np.int32)
    room.tri_rect = np.zeros(T.shape[0], np.int32)
    room.beta = np.full(T.shape[0], beta, np.complex128)
    room.h = float(np.linalg.norm(Vt[T[:, 1]] - Vt[T[:, 0]], axis=1).mean())
    return room


# ----------------------------------------------------------------------------- points
def _rect_dist(p, r: Rect):
    o, u, v = (np.asarray(a, float) for a in (r.o, r.u, r.v))
    d = p - o
    s = np.clip(d @ u / (u @ u), 0, 1)
    t = np.clip(d @ v / (v @ v), 0, 1)
    q = o + s * u + t * v
    return float(np.linalg.norm(p - q))


def _inside(p, room: Room):
    ins = any(b[0] < p[0] < b[1] and b[2] < p[1] < b[3] and b[4] < p[2] < b[5] for b in room.boxes)
    if not ins:
        return False
    return not any(b[0] <= p[0] <= b[1] and b[2] <= p[1] <= b[3] and b[4] <= p[2] <= b[5] for b in room.solids)


def sample_points(room: Room, count: int, seed: int, min_wall: float = 0.3, avoid=None, min_avoid: float = 0.3):
    """Uniform points inside the fluid, >= min_wall from every face (rejection sampling)."""
    rng = np.random.default_rng(seed)
    lo = np.min([[b[0], b[2], b[4]] for b in room.boxes], 0)
    hi = np.max([[b[1], b[3], b[5]] for b in room.boxes], 0)
    out = []
    while len(out) < count:
        p = rng.uniform(lo, hi)
        if not _inside(p, room):
            continue
        if min(_rect_dist(p, r) for r in room.rects) < min_wall:
            continue
        if avoid is not None and np.min(np.linalg.norm(np.atleast_2d(avoid) - p, axis=1)) < min_avoid:
            continue
        out.append(p)
    return np.array(out)


def source_and_receivers(room: Room, nrec: int, nsrc: int = 1):
    src = sample_points(room, nsrc, SEED_SOURCE)
    rec = sample_points(room, nrec, SEED_RECEIVERS, avoid=src)
    return src, rec


def complex_normal(n: int, seed: int, count: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = (n,) if count is None else (count, n)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def wavenumber(f_hz: float) -> float:
    return 2.0 * math.pi * f_hz / SOUND_SPEED


# ----------------------------------------------------------------------------- named workloads
def config_room(cfg: int) -> tuple[Room, float]:
    """Room and wavenumber for the five named workloads (small shoebox at 250 Hz, 6x5x3 m
    shoebox at 1 kHz, L-room with baffle+doorway at 2.5 kHz, ...)."""
    if cfg == 1:
        return shoebox(3.0, 2.5, 2.0, 0.17), wavenumber(250.0)
    if cfg == 2:
        lam = SOUND_SPEED / 1000.0
        return shoebox(6.0, 5.0, 3.0, lam / 6.5), wavenumber(1000.0)
    if cfg == 3:
        return lroom(0.01908), wavenumber(2500.0)
    if cfg == 5:
        return lroom(0.00779), wavenumber(5000.0)
    raise ValueError(cfg)
