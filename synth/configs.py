"""The five synthetic workloads, built deterministically from a seed.

Shapes and placement follow the clutterbox set-up of the paper's evaluation
(objects normalised into a unit sphere, dropped into a cube of side 3, support
radius 0.3, 64x64 images; Sec. 4.1-4.2).  The paper's object collection is
not available, so seeded superquadrics, tori and a jittered icosphere stand in
for it.

Every scene is returned with fp32 positions, u32 triangle indices and fp32
area-weighted normals computed from the rounded positions; needles, haystack
and the true-match map are explicit arrays.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import (Mesh, concat, icosphere, normalize_to_unit_sphere,
                     random_rotation, superquadric, torus, transform,
                     vertex_normals)


@dataclass
class Scene:
    """One describe-and-match workload.

    haystack: mesh (positions/triangles) whose every vertex is an oriented point.
    needles : mesh of the needle object and its oriented points (may be the same
              arrays as the haystack), plus true_index[i] = haystack image that
              is the correct match of needle i.
    """
    name: str
    support_radius: float
    positions: np.ndarray
    triangles: np.ndarray
    op_positions: np.ndarray
    op_normals: np.ndarray
    needle_positions: np.ndarray
    needle_triangles: np.ndarray
    needle_op_positions: np.ndarray
    needle_op_normals: np.ndarray
    true_index: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def num_haystack(self) -> int:
        return int(self.op_positions.shape[0])

    @property
    def num_needles(self) -> int:
        return int(self.needle_op_positions.shape[0])

    @property
    def needles_are_haystack(self) -> bool:
        return self.needle_op_positions is self.op_positions


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _self_scene(name: str, mesh: Mesh, radius: float, meta: dict) -> Scene:
    pos = _f32(mesh.positions)
    tri = np.ascontiguousarray(mesh.triangles.astype(np.uint32))
    nrm = vertex_normals(pos, tri)
    idx = np.arange(pos.shape[0], dtype=np.uint32)
    meta = dict(meta, V=int(pos.shape[0]), T=int(tri.shape[0]))
    return Scene(name, float(radius), pos, tri, pos, nrm, pos, tri, pos, nrm, idx, meta)


# ------------------------------------------------------------------------ objects

def random_object(rng: np.random.Generator, target_tris: int, kinds=("superquadric", "torus")) -> tuple[Mesh, dict]:
    """A seeded superquadric or torus with about `target_tris` triangles,
    normalised into the unit sphere (its canonical pose)."""
    kind = kinds[int(rng.integers(len(kinds)))]
    if kind == "superquadric":
        n = max(1, int(round(np.sqrt(target_tris / 12.0))))
        e1, e2 = rng.uniform(0.3, 3.0, size=2)
        scales = rng.uniform(0.5, 1.0, size=3)
        m = superquadric(n, e1, e2, scales, noise=0.02, rng=rng)
        info = dict(kind=kind, n=n, e1=float(e1), e2=float(e2))
    else:
        n_v = max(3, int(round(np.sqrt(target_tris / 4.0))))
        n_u = 2 * n_v
        major = rng.uniform(0.5, 0.8)
        minor = rng.uniform(0.1, 0.3)
        m = torus(n_u, n_v, major, minor)
        info = dict(kind=kind, n_u=n_u, n_v=n_v, major=float(major), minor=float(minor))
    return Mesh(normalize_to_unit_sphere(m.positions), m.triangles), info


def clutter_scene(rng: np.random.Generator, n_objects: int, tri_lo: int, tri_hi: int,
                  log_uniform: bool = False):
    """Objects in canonical pose, then each rotated at random and translated by
    U(-0.5, 0.5)^3 so its unit bounding sphere stays inside the cube of side 3.
    Returns (scene mesh, canonical object meshes, vertex offsets, info)."""
    canon, placed, infos, offsets, off = [], [], [], [], 0
    for _ in range(n_objects):
        if log_uniform:
            t = int(round(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi)))))
        else:
            t = int(rng.integers(tri_lo, tri_hi + 1))
        m, info = random_object(rng, t)
        rot = random_rotation(rng)
        shift = rng.uniform(-0.5, 0.5, size=3)
        canon.append(m)
        placed.append(Mesh(transform(m.positions, rot, shift), m.triangles))
        infos.append(info)
        offsets.append(off)
        off += m.num_vertices
    return concat(placed), canon, offsets, infos


# ------------------------------------------------------------------------ configs

def config1_icosphere(seed: int = 1) -> Scene:
    """Icosphere (subdivision 2: V = 162, T = 320), vertex radius jittered by
    1 + U(-0.05, 0.05), support radius 1.0; all-vs-all with t(i) = i."""
    rng = np.random.default_rng(seed)
    m = icosphere(2)
    jitter = 1.0 + rng.uniform(-0.05, 0.05, size=(m.num_vertices, 1))
    return _self_scene("icosphere", Mesh(m.positions * jitter, m.triangles), 1.0,
                       dict(seed=seed, config=1))


def config2_union12(seed: int = 2, n: int = 18, shapes: int = 12) -> Scene:
    """Union of 12 noisy superquadrics (n = 18 per cube face: 3 888 triangles and
    1 946 vertices each) posed at random in one frame and scaled into the unit
    sphere; support radius 0.3; all-vs-all with t(i) = i."""
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(shapes):
        e1, e2 = rng.uniform(0.3, 3.0, size=2)
        scales = rng.uniform(0.5, 1.0, size=3)
        m = superquadric(n, e1, e2, scales, noise=0.02, rng=rng)
        p = normalize_to_unit_sphere(m.positions)
        p = transform(p, random_rotation(rng), rng.uniform(-1.0, 1.0, size=3))
        parts.append(Mesh(p, m.triangles))
    u = concat(parts)
    return _self_scene("union12", Mesh(normalize_to_unit_sphere(u.positions), u.triangles), 0.3,
                       dict(seed=seed, config=2, shapes=shapes, n=n))


def config3_clutter(seed: int = 3, n_objects: int = 10, tri_lo: int = 20_000,
                    tri_hi: int = 100_000) -> Scene:
    """Clutter scene: 10 seeded superquadric/torus objects of U[20k, 100k]
    triangles in the side-3 box.  Needles: object 0 alone in canonical pose.
    Haystack: every vertex of the combined scene; t(i) = i (object 0 first)."""
    rng = np.random.default_rng(seed)
    scene, canon, offsets, infos = clutter_scene(rng, n_objects, tri_lo, tri_hi)
    pos = _f32(scene.positions)
    tri = np.ascontiguousarray(scene.triangles)
    nrm = vertex_normals(pos, tri)
    npos = _f32(canon[0].positions)
    ntri = np.ascontiguousarray(canon[0].triangles)
    nnrm = vertex_normals(npos, ntri)
    true_index = (offsets[0] + np.arange(npos.shape[0])).astype(np.uint32)
    meta = dict(seed=seed, config=3, objects=infos, V=int(pos.shape[0]), T=int(tri.shape[0]),
                needle_V=int(npos.shape[0]), needle_T=int(ntri.shape[0]))
    return Scene("clutter", 0.3, pos, tri, pos, nrm, npos, ntri, npos, nnrm, true_index, meta)


def config4_batch(seed: int = 4, meshes: int = 256, tri_lo: int = 1_000,
                  tri_hi: int = 200_000) -> list[Scene]:
    """256 meshes with log-uniform triangle counts in [1k, 200k], each in its own
    frame (unit sphere); per mesh all-vs-all with t(i) = i; support radius 0.3."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(meshes):
        t = int(round(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi)))))
        m, info = random_object(rng, t)
        out.append(_self_scene(f"batch{k}", m, 0.3, dict(seed=seed, config=4, index=k, **info)))
    return out


def config5_database(seed: int = 5, target_images: int = 1_000_000, objects_per_scene: int = 4,
                     tri_lo: int = 1_000, tri_hi: int = 100_000):
    """Descriptor database source: clutter scenes of 4 objects each (log-uniform
    1k-100k triangles) until `target_images` vertices are reached.  Returns a
    list of (scene mesh, canonical objects, vertex offsets) and the total count."""
    rng = np.random.default_rng(seed)
    scenes, total = [], 0
    while total < target_images:
        mesh, canon, offsets, _ = clutter_scene(rng, objects_per_scene, tri_lo, tri_hi, log_uniform=True)
        scenes.append((mesh, canon, offsets))
        total += mesh.num_vertices
    return scenes, total


def config5_request(db_scenes, rng: np.random.Generator, max_queries: int = 1024):
    """One serving request: a seeded object of a database scene in canonical pose
    (its mesh to describe) and up to `max_queries` of its vertices as needles.
    Returns (needle mesh arrays, needle vertex ids, database offset of the
    object's vertex 0 counting from the start of the database)."""
    s = int(rng.integers(len(db_scenes)))
    _, canon, offsets = db_scenes[s]
    o = int(rng.integers(len(canon)))
    base = sum(db_scenes[i][0].num_vertices for i in range(s)) + offsets[o]
    m = canon[o]
    pos = _f32(m.positions)
    tri = np.ascontiguousarray(m.triangles)
    nrm = vertex_normals(pos, tri)
    q = min(pos.shape[0], max_queries)
    ids = np.sort(rng.choice(pos.shape[0], size=q, replace=False)).astype(np.uint32)
    return pos, tri, nrm, ids, base


CONFIG_BUILDERS = {
    1: config1_icosphere,
    2: config2_union12,
    3: config3_clutter,
}
