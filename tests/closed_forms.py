"""Scenes with closed-form RICIs, shared by the oracle pins (CPU) and the GPU
parity tests.  Test infrastructure: the expected images are written from the
geometry of Sec. 3.1 (a circle of radius rho_c in the row plane beta_r crosses
a segment once if exactly one end lies outside it, twice if both ends lie
outside and the segment's closest point to the axis lies inside)."""

from __future__ import annotations

import numpy as np


def bin_radius_boundaries(R: float = 1.0, delta: float = 1e-4, b0: float = -0.31, b1: float = 0.23):
    """Ranges starting `delta` bins inside and outside each of the 64 bin
    radii, for the oriented point at the origin with normal +z.  Each radius r
    gets a radial rectangle (inner edge at r, outer edge at 2R: one crossing
    for every bin radius above r) and a chord rectangle (a segment at distance
    r from the axis, both ends at about 2R: two crossings for every bin radius
    above r), both spanning heights b0 .. b1, at golden-angle azimuths.

    Returns (positions float32 [V, 3], triangles uint32 [T, 3], expected
    image int64 [64, 64]) with the expectation computed in float64 from the
    float32 coordinates."""
    verts, tris = [], []

    def rect(p0, p1):
        k = len(verts)
        verts.extend([(p0[0], p0[1], b0), (p1[0], p1[1], b0), (p1[0], p1[1], b1), (p0[0], p0[1], b1)])
        tris.extend([(k, k + 1, k + 2), (k, k + 2, k + 3)])

    n = 0
    for c in range(64):
        for d in (-delta, delta):
            r = (c + 0.5 + d) * R / 64
            phi = 2.399963 * n
            u = np.array([np.cos(phi), np.sin(phi)])
            w = np.array([-u[1], u[0]])
            rect(r * u, 2.0 * R * u)
            rect(r * w - 2.0 * R * u, r * w + 2.0 * R * u)
            n += 1
    v = np.array(verts, np.float32)
    t = np.array(tris, np.uint32)
    V = v.astype(np.float64)
    rho = (np.arange(64) + 0.5) * R / 64
    beta = -R / 2 + (np.arange(64) + 0.5) * R / 64
    rows = (beta > np.float64(np.float32(b0))) & (beta < np.float64(np.float32(b1)))
    per_col = np.zeros(64, np.int64)
    for k in range(0, len(V), 8):
        per_col += rho > np.hypot(V[k, 0], V[k, 1])       # radial rectangle: its inner edge
        p, q = V[k + 4, :2], V[k + 5, :2]                 # chord: distance of its line from the axis
        per_col += 2 * (rho > abs(p[0] * q[1] - p[1] * q[0]) / np.hypot(*(q - p)))
    return v, t, rows[:, None] * per_col[None, :]


def row_plane_boundaries(R: float = 1.0, delta: float = 1e-4):
    """Radial rectangles whose lower and upper edges lie `delta` bins above or
    below row planes, for the oriented point at the origin with normal +z.
    Rectangle (r, s) has its lower edge at beta_r + s * delta (s = -1, +1) and
    its upper edge at beta_{r+3} - s * delta (or above the image near the top),
    its inner edge between two bin radii and its outer edge at 2R.  A row plane
    beta cuts a rectangle spanning z_lo .. z_hi iff z_lo < beta <= z_hi (a
    vertex at z >= beta counts as above it), and then adds one crossing for
    each bin radius beyond the inner edge.

    Returns (positions float32 [V, 3], triangles uint32 [T, 3], expected
    image int64 [64, 64])."""
    b = R / 64
    beta = -R / 2 + (np.arange(64) + 0.5) * b
    rho = (np.arange(64) + 0.5) * b
    verts, tris, rects = [], [], []
    n = 0
    for r in range(64):
        for s in (-1.0, 1.0):
            lo = beta[r] + s * delta * b
            hi = beta[r + 3] - s * delta * b if r + 3 < 64 else R / 2 + 0.3 * b
            rin = ((7 * n) % 60 + 0.75) * b
            phi = 2.399963 * n
            u = np.array([np.cos(phi), np.sin(phi)])
            k = len(verts)
            p0, p1 = rin * u, 2.0 * R * u
            verts.extend([(p0[0], p0[1], lo), (p1[0], p1[1], lo), (p1[0], p1[1], hi), (p0[0], p0[1], hi)])
            tris.extend([(k, k + 1, k + 2), (k, k + 2, k + 3)])
            n += 1
    v = np.array(verts, np.float32)
    t = np.array(tris, np.uint32)
    V = v.astype(np.float64)
    exp = np.zeros((64, 64), np.int64)
    for k in range(0, len(V), 4):
        z_lo, z_hi = V[k, 2], V[k + 2, 2]
        rows = (beta > z_lo) & (beta <= z_hi)
        cols = rho > np.hypot(V[k, 0], V[k, 1])
        exp += rows[:, None] * cols[None, :]
    return v, t, exp


def degenerate_triangles():
    """Degenerate and boundary triangles near the origin (support radius 1,
    normal +z): a point, a vertical and a slanted segment, a triangle lying in
    a row plane, one with an edge in a row plane, one with vertices on two
    row planes, and one with an edge on the axis.  (No closed form: used to
    compare the row-range algorithm with the brute-force definition and the
    GPU with the oracle.)"""
    b = 1.0 / 64
    beta = lambda r: -0.5 + (r + 0.5) * b
    V, T = [], []

    def tri(p, q, s):
        k = len(V)
        V.extend([p, q, s])
        T.append((k, k + 1, k + 2))

    tri((0.2, 0.1, 0.05), (0.2, 0.1, 0.05), (0.2, 0.1, 0.05))
    tri((0.1, -0.2, -0.3), (0.1, -0.2, 0.0), (0.1, -0.2, 0.3))
    tri((-0.3, 0.0, -0.2), (0.0, 0.1, 0.0), (0.3, 0.2, 0.2))
    tri((-0.4, -0.4, beta(40)), (0.4, -0.3, beta(40)), (0.0, 0.5, beta(40)))
    tri((-0.3, 0.25, beta(20)), (0.3, 0.25, beta(20)), (0.0, 0.25, beta(28)))
    tri((0.15, 0.0, beta(10)), (0.15, 0.0, beta(30)), (0.45, 0.0, beta(10)))
    tri((0.0, 0.0, -0.45), (0.0, 0.0, 0.45), (0.3, 0.0, 0.0))
    return np.array(V, np.float32), np.array(T, np.uint32)
