"""Synthetic clutterbox experiment (Sec. 4.1) on the GPU path.

One trial:
  1. draw n objects (seeded superquadrics / tori), each scaled into the unit
     sphere (their canonical pose);
  2. the first object is the reference: its RICIs, one per vertex, are the
     reference set {RD};
  3. place the objects one by one in a cube of side s, the reference first,
     each at a random orientation and a position that keeps its bounding sphere
     inside the cube;
  4. at each requested clutter level k (objects placed so far) compute the
     cluttered set {CD}, one RICI per vertex of the combined mesh, and rank
     every reference RICI against all of {CD}; its correct match is the same
     vertex of the placed reference, which comes first in the combined mesh;
  5. the histogram of those ranks is the trial's result for level k;
  6. with each rank, the clutter around the reference vertex (Eq. 8): the
     share of the surface inside its support volume that is not the
     reference object's, (A_all - A_object) / A_all (rici_clutter_areas).

The paper reports, per level, the fraction of searches whose correct match is
at rank 0; `summarise` does the same over many trials, and splits it by the
clutter around each searched vertex.  Objects here are synthetic stand-ins for
a mesh collection (no dataset is used).
"""

from __future__ import annotations

import time

import numpy as np


def _torch():
    import torch
    return torch


def run_trial(ctx, rng: np.random.Generator, levels=(1, 5, 10), tri_lo: int = 1000, tri_hi: int = 20000,
              support_radius: float = 0.3, box_side: float = 3.0, keep: bool = False) -> dict:
    """One clutterbox trial; returns {level: {"ranks": np.ndarray, ...}}.  With
    keep, each level also holds its scene mesh and host copies of both image
    sets ("scene", "rd", "cd"), and the reference mesh is under key 0."""
    from synth.configs import random_object
    from synth.meshes import Mesh, concat, random_rotation, transform, vertex_normals

    torch = _torch()
    dev = torch.device("cuda", ctx.device)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)
    i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(dev)

    levels = sorted(set(int(k) for k in levels))
    n = levels[-1]
    objects = []
    for _ in range(n):
        t = int(round(np.exp(rng.uniform(np.log(tri_lo), np.log(tri_hi)))))
        m, _ = random_object(rng, t)
        objects.append(m)
    ref = objects[0]
    ref_pos = ref.positions.astype(np.float32)
    ref_nrm = vertex_normals(ref_pos, ref.triangles)
    rd = ctx.generate(f32(ref_pos), i32(ref.triangles), f32(ref_pos), f32(ref_nrm), support_radius)

    # placements: the bounding sphere (radius 1 around the origin) stays inside
    # the cube [-s/2, s/2]^3
    half = box_side / 2.0 - 1.0
    if half < 0:
        raise ValueError("the clutterbox must be at least 2 units wide")
    placed = []
    for m in objects:
        rot = random_rotation(rng)
        shift = rng.uniform(-half, half, size=3)
        placed.append(Mesh(transform(m.positions, rot, shift), m.triangles))

    v0 = ref.num_vertices
    true_index = i32(np.arange(v0, dtype=np.uint32))
    out = {}
    for k in levels:
        scene = concat(placed[:k])
        pos = scene.positions.astype(np.float32)
        nrm = vertex_normals(pos, scene.triangles)
        t0 = time.perf_counter()
        cd = ctx.generate(f32(pos), i32(scene.triangles), f32(pos), f32(nrm), support_radius)
        rank, dist = ctx.distance_rank(rd, cd, true_index)
        # Eq. 8 around each placed reference vertex; the reference's triangles
        # come first in the combined mesh
        d_pos, d_tri = f32(pos), i32(scene.triangles)
        a_all, a_obj = ctx.clutter_areas(d_pos, d_tri, 0, ref.triangles.shape[0], d_pos[:v0].contiguous(),
                                         f32(nrm[:v0]), support_radius)
        ctx.sync()
        wall = time.perf_counter() - t0
        ranks = rank.cpu().numpy().view(np.uint32).copy()
        A, O = a_all.cpu().numpy(), a_obj.cpu().numpy()
        clutter = np.where(A > 0, (A - O) / np.where(A > 0, A, 1.0), 0.0)
        out[k] = {"ranks": ranks, "clutter": clutter, "area_all": A, "area_object": O,
                  "reference_vertices": int(v0), "scene_vertices": int(pos.shape[0]),
                  "scene_triangles": int(scene.triangles.shape[0]), "gpu_s": wall}
        if keep:
            out[k].update(scene=(pos, scene.triangles, nrm), rd=rd.cpu().numpy().view(np.uint32).copy(),
                          cd=cd.cpu().numpy().view(np.uint32).copy())
    if keep:
        out[0] = {"reference": (ref_pos, ref.triangles, ref_nrm)}
    return out


def summarise(trials: list[dict]) -> dict:
    """Per clutter level: rank-0 fraction over all searches, its spread over
    trials (sorted per-trial fractions, as the paper plots them), and the
    histogram of the first ranks."""
    levels = sorted(k for k in trials[0].keys() if k > 0) if trials else []
    res = {}
    for k in levels:
        per_trial = np.array([float((t[k]["ranks"] == 0).mean()) for t in trials])
        allr = np.concatenate([t[k]["ranks"] for t in trials])
        hist = np.bincount(np.minimum(allr, 10).astype(np.int64), minlength=11)
        res[k] = {"searches": int(allr.size), "rank0_fraction": float((allr == 0).mean()),
                  "rank0_fraction_per_trial_sorted": np.sort(per_trial).round(4).tolist(),
                  "rank_histogram_0_to_10plus": hist.tolist(),
                  "median_rank": float(np.median(allr))}
        if all("clutter" in t[k] for t in trials):
            cl = np.concatenate([t[k]["clutter"] for t in trials])
            res[k]["clutter_mean"] = float(cl.mean())
            res[k]["rank0_fraction_by_clutter"] = by_clutter(allr, cl)
    return res


def by_clutter(ranks: np.ndarray, clutter: np.ndarray, edges=(0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9,
                                                                  1.0)) -> list:
    """Rank-0 fraction of the searches in each clutter bin [e_i, e_i+1)
    (the last bin closed): [(lower edge, searches, rank-0 fraction)]."""
    out = []
    for i in range(len(edges) - 1):
        lo, hi = edges[i], edges[i + 1]
        sel = (clutter >= lo) & ((clutter < hi) if i + 2 < len(edges) else (clutter <= hi))
        n = int(sel.sum())
        out.append((lo, n, float((ranks[sel] == 0).mean()) if n else None))
    return out
