"""Procedural, watertight triangle meshes and rigid placement (all FP64, rounded
once to fp32 by the caller).

Shapes
  * icosphere: regular icosahedron refined by edge-midpoint subdivision with
    welded midpoints, pushed onto the unit sphere; vertices in creation order.
  * cube_sphere: an n x n grid on each face of the cube [-1, 1]^3, welded along
    cube edges (V = 6 n^2 + 2, T = 12 n^2), every quad split on one diagonal.
  * superquadric: each cube-sphere direction v is pushed to the surface of Barr's
    superquadric F(x, y, z) = 1 with
        F = (|x|^(2/e2) + |y|^(2/e2))^(e2/e1) + |z|^(2/e1),
    i.e. p = v * F(v)^(-e1/2) (F is homogeneous of degree 2/e1), then scaled per
    axis and optionally perturbed radially.
  * torus: an n_u x n_v grid with wrap-around (V = n_u n_v, T = 2 n_u n_v).

Every mesh is oriented with outward-facing counter-clockwise triangles, so the
area-weighted vertex normals point outwards.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    positions: np.ndarray  # [V, 3] float64 (rounded to fp32 by the scene builder)
    triangles: np.ndarray  # [T, 3] uint32

    @property
    def num_vertices(self) -> int:
        return int(self.positions.shape[0])

    @property
    def num_triangles(self) -> int:
        return int(self.triangles.shape[0])


# --------------------------------------------------------------------------- shapes

_ICO_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_VERTS = [
    (-1, _ICO_T, 0), (1, _ICO_T, 0), (-1, -_ICO_T, 0), (1, -_ICO_T, 0),
    (0, -1, _ICO_T), (0, 1, _ICO_T), (0, -1, -_ICO_T), (0, 1, -_ICO_T),
    (_ICO_T, 0, -1), (_ICO_T, 0, 1), (-_ICO_T, 0, -1), (-_ICO_T, 0, 1),
]
_ICO_FACES = [
    (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
    (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
    (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
    (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
]


def icosphere(subdivisions: int) -> Mesh:
    """Unit icosphere; subdivision s gives V = 10*4^s + 2, T = 20*4^s."""
    verts = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in _ICO_VERTS]
    faces = list(_ICO_FACES)
    for _ in range(subdivisions):
        midpoint: dict[tuple[int, int], int] = {}

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            idx = midpoint.get(key)
            if idx is None:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                idx = len(verts) - 1
                midpoint[key] = idx
            return idx

        new_faces = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    return Mesh(np.array(verts, dtype=np.float64), np.array(faces, dtype=np.uint32))


# (normal axis, sign, tangent axis a, tangent axis b) with e_a x e_b = sign * e_axis
_CUBE_FACES = [
    (0, +1, 1, 2), (0, -1, 2, 1),
    (1, +1, 2, 0), (1, -1, 0, 2),
    (2, +1, 0, 1), (2, -1, 1, 0),
]


def cube_sphere(n: int) -> tuple[np.ndarray, np.ndarray]:
    """Welded n x n-per-face cube grid: returns (unit directions [V,3], tris [T,3])."""
    if n < 1:
        raise ValueError("n >= 1 required")
    keys = []
    tris = []
    for axis, sign, a, b in _CUBE_FACES:
        base = len(keys)
        for j in range(n + 1):
            for i in range(n + 1):
                k = [0, 0, 0]
                k[axis] = sign * n
                k[a] = -n + 2 * i
                k[b] = -n + 2 * j
                keys.append(tuple(k))
        for j in range(n):
            for i in range(n):
                v00 = base + j * (n + 1) + i
                v10 = v00 + 1
                v01 = v00 + (n + 1)
                v11 = v01 + 1
                tris.append((v00, v10, v11))
                tris.append((v00, v11, v01))
    keys_arr = np.array(keys, dtype=np.int64)
    uniq, first, inverse = np.unique(keys_arr, axis=0, return_index=True, return_inverse=True)
    # renumber in order of first appearance so the vertex order is deterministic
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    remap = rank[inverse.reshape(-1)]
    pts = uniq[order].astype(np.float64)
    dirs = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    tri = remap[np.array(tris, dtype=np.int64)]
    return dirs, tri.astype(np.uint32)


def superquadric(n: int, e1: float, e2: float, scales=(1.0, 1.0, 1.0),
                 noise: float = 0.0, rng: np.random.Generator | None = None) -> Mesh:
    """Superquadric surface sampled on an n x n-per-face cube-sphere grid."""
    dirs, tris = cube_sphere(n)
    x, y, z = np.abs(dirs[:, 0]), np.abs(dirs[:, 1]), np.abs(dirs[:, 2])
    f = (x ** (2.0 / e2) + y ** (2.0 / e2)) ** (e2 / e1) + z ** (2.0 / e1)
    p = dirs * (f ** (-e1 / 2.0))[:, None]
    p = p * np.asarray(scales, dtype=np.float64)[None, :]
    if noise > 0.0:
        if rng is None:
            raise ValueError("noise needs an rng")
        p = p * (1.0 + rng.uniform(-noise, noise, size=(p.shape[0], 1)))
    return Mesh(p, tris)


def torus(n_u: int, n_v: int, major: float, minor: float) -> Mesh:
    """Torus around the z axis: major radius `major`, tube radius `minor`."""
    if n_u < 3 or n_v < 3:
        raise ValueError("torus grid needs n_u, n_v >= 3")
    th = 2.0 * np.pi * np.arange(n_u) / n_u
    ph = 2.0 * np.pi * np.arange(n_v) / n_v
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    ring = major + minor * np.cos(PH)
    p = np.stack([ring * np.cos(TH), ring * np.sin(TH), minor * np.sin(PH)], axis=-1)
    p = p.reshape(-1, 3)
    i = np.arange(n_u)[:, None]
    j = np.arange(n_v)[None, :]
    v00 = i * n_v + j
    v10 = ((i + 1) % n_u) * n_v + j
    v01 = i * n_v + (j + 1) % n_v
    v11 = ((i + 1) % n_u) * n_v + (j + 1) % n_v
    t1 = np.stack([v00, v10, v11], axis=-1).reshape(-1, 3)
    t2 = np.stack([v00, v11, v01], axis=-1).reshape(-1, 3)
    tris = np.empty((2 * n_u * n_v, 3), dtype=np.int64)
    tris[0::2] = t1
    tris[1::2] = t2
    return Mesh(p, tris.astype(np.uint32))


# ----------------------------------------------------------------- placement / normals

def vertex_normals(positions: np.ndarray, triangles: np.ndarray) -> np.ndarray:
    """Area-weighted vertex normals: sum over incident faces (in face order, FP64)
    of (p_b - p_a) x (p_c - p_a), normalised in FP64, rounded once to fp32.
    A vertex with no incident area gets the zero vector."""
    p = np.asarray(positions, dtype=np.float64)
    t = np.asarray(triangles, dtype=np.int64)
    a, b, c = p[t[:, 0]], p[t[:, 1]], p[t[:, 2]]
    fn = np.cross(b - a, c - a)
    acc = np.zeros_like(p)
    for k in range(3):
        np.add.at(acc, t[:, k], fn)
    norm = np.linalg.norm(acc, axis=1, keepdims=True)
    out = np.divide(acc, norm, out=np.zeros_like(acc), where=norm > 0)
    return out.astype(np.float32)


def normalize_to_unit_sphere(positions: np.ndarray) -> np.ndarray:
    """Centre of the bounding box to the origin, then scale so max |p| = 1."""
    p = np.asarray(positions, dtype=np.float64)
    centre = 0.5 * (p.min(axis=0) + p.max(axis=0))
    q = p - centre
    r = np.linalg.norm(q, axis=1).max()
    return q / r if r > 0 else q


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly distributed rotation from a uniform unit quaternion (Shoemake)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, size=3)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    qx, qy = a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2)
    qz, qw = b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)],
        [2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)],
        [2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)],
    ])


def transform(positions: np.ndarray, rotation=None, translation=None, scale: float = 1.0) -> np.ndarray:
    p = np.asarray(positions, dtype=np.float64) * scale
    if rotation is not None:
        p = p @ np.asarray(rotation, dtype=np.float64).T
    if translation is not None:
        p = p + np.asarray(translation, dtype=np.float64)[None, :]
    return p


def concat(meshes: list[Mesh]) -> Mesh:
    pos, tri, off = [], [], 0
    for m in meshes:
        pos.append(np.asarray(m.positions, dtype=np.float64))
        tri.append(np.asarray(m.triangles, dtype=np.int64) + off)
        off += m.num_vertices
    return Mesh(np.concatenate(pos, axis=0), np.concatenate(tri, axis=0).astype(np.uint32))


def sample_surface(positions: np.ndarray, triangles: np.ndarray, rng: np.random.Generator,
                   per_triangle: float = 10.0) -> np.ndarray:
    """Uniform random point samples of a mesh surface, fp32 [S, 3] with
    S = round(per_triangle * T): each sample picks a triangle with probability
    proportional to its area, then a uniform point in it (barycentric
    coordinates 1 - sqrt(r1), sqrt(r1) (1 - r2), sqrt(r1) r2).  The point cloud
    that Spin Images are built from."""
    p = np.asarray(positions, dtype=np.float64)
    t = np.asarray(triangles, dtype=np.int64)
    if t.shape[0] == 0:
        return np.zeros((0, 3), dtype=np.float32)
    a, b, c = p[t[:, 0]], p[t[:, 1]], p[t[:, 2]]
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    total = area.sum()
    n = int(round(per_triangle * t.shape[0]))
    if n == 0 or total <= 0.0:
        return np.zeros((0, 3), dtype=np.float32)
    pick = rng.choice(t.shape[0], size=n, p=area / total)
    r1 = np.sqrt(rng.random(n))
    r2 = rng.random(n)
    w0, w1, w2 = 1.0 - r1, r1 * (1.0 - r2), r1 * r2
    pts = w0[:, None] * a[pick] + w1[:, None] * b[pick] + w2[:, None] * c[pick]
    return pts.astype(np.float32)
