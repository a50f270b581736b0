"""Pins of the oracle's RICI generation.

* The row-range algorithm (Sec. 3.1.2) against the plain definition of a bin
  (the number of points where the bin's circle meets the surface, Sec. 3.1) on
  random tiny scenes, outside flagged pixels.
* Closed forms: a planar square whose plane contains the Central Axis, and an
  off-axis sphere.
* Invariants: even counts on closed surfaces, rigid motions, power-of-two
  scaling, additivity over triangles, empty scenes.
"""

import numpy as np
import pytest

import closed_forms
import oracle
import synth

NB = 64


def _grid(R):
    d = np.float64(np.float32(R)) / NB
    rho = (np.arange(NB) + 0.5) * d
    beta = -0.5 * np.float64(np.float32(R)) + (np.arange(NB) + 0.5) * d
    return rho, beta


def _random_scene(rng, ntri, npts, spread=1.0):
    pts = rng.uniform(-spread, spread, size=(3 * ntri, 3)).astype(np.float32)
    tri = np.arange(3 * ntri, dtype=np.uint32).reshape(ntri, 3)
    op = rng.uniform(-0.5 * spread, 0.5 * spread, size=(npts, 3)).astype(np.float32)
    nrm = rng.normal(size=(npts, 3)).astype(np.float32)
    return pts, tri, op, nrm


@pytest.mark.parametrize("seed", range(8))
def test_rowrange_equals_brute_force_on_tiny_scenes(seed):
    rng = np.random.default_rng(100 + seed)
    ntri = int(rng.integers(1, 40))
    pts, tri, op, nrm = _random_scene(rng, ntri, 6)
    R = float(rng.uniform(0.4, 2.0))
    im, fl, wk = oracle.rici_rowrange(pts, tri, op, nrm, R)
    ib, fb = oracle.rici_brute(pts, tri, op, nrm, R)
    ok = ~(fl | fb)
    assert ok.mean() > 0.99
    assert np.array_equal(im[ok], ib[ok])
    assert (wk[:, 0] == ntri).all()
    assert im.sum() > 0


def test_single_triangle_counts_at_most_two():
    rng = np.random.default_rng(42)
    for _ in range(20):
        pts, tri, op, nrm = _random_scene(rng, 1, 4)
        im, fl, _ = oracle.rici_rowrange(pts, tri, op, nrm, 1.5)
        assert im.max() <= 2
        ib, fb = oracle.rici_brute(pts, tri, op, nrm, 1.5)
        ok = ~(fl | fb)
        assert np.array_equal(im[ok], ib[ok])


def test_config1_rowrange_equals_brute_force():
    s = synth.config1_icosphere()
    sel = np.arange(0, s.num_haystack, 9)
    im, fl, _ = oracle.rici_rowrange(s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], 1.0)
    ib, fb = oracle.rici_brute(s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], 1.0)
    ok = ~(fl | fb)
    assert np.array_equal(im[ok], ib[ok])
    assert im.max() > 0


# ----------------------------------------------------------------- closed forms

def _square(L1, L2, b0, b1):
    v = np.array([[-L1, 0, b0], [L2, 0, b0], [L2, 0, b1], [-L1, 0, b1]], dtype=np.float64)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.uint32)
    return v, t


def _square_expected(R, L1, L2, b0, b1):
    rho, beta = _grid(R)
    inside = ((beta > b0) & (beta < b1))[:, None]
    return (inside * ((rho < L1).astype(int) + (rho < L2).astype(int))[None, :]).astype(np.uint32)


def _square_margins(R, L1, L2, b0, b1):
    """smallest distance of any sample radius / height from a place where the
    closed form changes or the diagonal's crossing sits."""
    rho, beta = _grid(R)
    m = min(np.abs(rho - L1).min(), np.abs(rho - L2).min(), np.abs(beta - b0).min(), np.abs(beta - b1).min())
    for b in beta[(beta > b0) & (beta < b1)]:
        xd = -L1 + (b - b0) / (b1 - b0) * (L1 + L2)
        m = min(m, np.abs(rho - abs(xd)).min(), abs(xd))
    return m


@pytest.mark.parametrize("params", [(0.7, 0.45, -0.31, 0.23), (0.2, 0.9, -0.47, 0.41), (0.333, 0.6, 0.05, 0.37)])
def test_planar_square_containing_axis(params):
    L1, L2, b0, b1 = params
    R = 1.0
    assert _square_margins(R, L1, L2, b0, b1) > 1e-4
    v, t = _square(L1, L2, b0, b1)
    im, fl, _ = oracle.rici_rowrange(v.astype(np.float32), t, np.zeros((1, 3), np.float32),
                                     np.array([[0, 0, 1]], np.float32), R)
    exp = _square_expected(R, np.float32(L1), np.float32(L2), np.float32(b0), np.float32(b1))
    assert not fl.any()
    assert np.array_equal(im[0], exp)
    assert exp.max() == 2 and exp.sum() > 0


@pytest.mark.parametrize("seed", range(4))
def test_planar_square_rotated_and_moved(seed):
    rng = np.random.default_rng(seed)
    L1, L2, b0, b1 = 0.7, 0.45, -0.31, 0.23
    v, t = _square(L1, L2, b0, b1)
    rot = synth.random_rotation(rng)
    shift = rng.uniform(-1, 1, 3)
    sv = shift.astype(np.float32)[None, :]
    sn = (rot @ np.array([0, 0, 1.0])).astype(np.float32)[None, :]
    vv = (v @ rot.T + shift).astype(np.float32)
    im, fl, _ = oracle.rici_rowrange(vv, t, sv, sn, 1.0)
    exp = _square_expected(1.0, L1, L2, b0, b1)
    assert np.array_equal(im[0][~fl[0]], exp[~fl[0]])
    assert fl.sum() == 0


@pytest.mark.parametrize("case", [(0.3, 0.1, 0.02, 1.0), (0.45, 0.25, -0.1, 1.0), (0.12, 0.08, 0.03, 0.5)])
def test_off_axis_sphere(case):
    """Sphere of radius a whose centre sits at axial height q and axis distance
    d: the row plane at beta cuts it in a circle of radius
    s = sqrt(a^2 - (beta - q)^2) centred d away from the axis, which meets the
    bin circle twice iff |rho - s| < d < rho + s (0 times otherwise)."""
    a, d, q, R = case
    m = synth.icosphere(5)
    sag = 1.0 - np.cos(np.deg2rad(63.43) / 32 / np.sqrt(3) * 2)  # circumradius angle bound
    chord = 4 * a * sag + 1e-6
    rng = np.random.default_rng(1)
    rot = synth.random_rotation(rng)
    n = rot @ np.array([0, 0, 1.0])
    u = rot @ np.array([1.0, 0, 0])
    sv = np.array([0.1, -0.2, 0.3])
    centre = sv + q * n + d * u
    pos = (m.positions * a + centre).astype(np.float32)
    im, fl, _ = oracle.rici_rowrange(pos, m.triangles, sv.astype(np.float32)[None, :],
                                     n.astype(np.float32)[None, :], R)
    rho, beta = _grid(R)
    B, P = np.meshgrid(beta, rho, indexing="ij")
    h2 = a * a - (B - q) ** 2
    s = np.sqrt(np.maximum(h2, 0))
    exp = np.where((h2 > 0) & (np.abs(P - s) < d) & (d < P + s), 2, 0)
    margin = np.minimum.reduce([np.abs(np.abs(B - q) - a), np.abs(np.abs(P - s) - d), np.abs(P + s - d)])
    ok = (margin > chord) & ~fl[0]
    assert ok.mean() > 0.8
    assert (exp[ok] == 2).sum() > 20
    assert np.array_equal(im[0][ok], exp[ok])


# ------------------------------------------------------------------- invariants

def test_columns_next_to_every_bin_radius():
    """Single ranges (radial rectangles) and double ranges (chords) that start
    1e-4 bins inside and outside each of the 64 bin radii: the oracle's image
    equals the closed form exactly and flags nothing (the margin is far above
    the degenerate-case tolerance)."""
    v, t, exp = closed_forms.bin_radius_boundaries()
    o, fl, _ = oracle.rici_rowrange(v, t, np.zeros((1, 3), np.float32), np.array([[0, 0, 1]], np.float32), 1.0)
    assert not fl.any()
    assert np.array_equal(o[0].astype(np.int64), exp)
    # column c lies above 2c + 1 of the 128 radii: 3 (2c + 1) crossings on the
    # rows inside the rectangles' height, none elsewhere
    inside = exp.any(axis=1)
    assert inside.sum() == 35   # rows 12 .. 46: beta_r in (-0.31, 0.23)
    assert (exp[inside] == 3 * (2 * np.arange(64) + 1)).all() and (exp[~inside] == 0).all()


def test_rows_next_to_every_row_plane():
    """Rectangles whose lower and upper edges lie 1e-4 bins above or below
    the row planes: the oracle includes exactly the rows with z_lo < beta <=
    z_hi, flags nothing, and a plane just below an edge cuts the rectangle
    while one just above it does not."""
    v, t, exp = closed_forms.row_plane_boundaries()
    o, fl, _ = oracle.rici_rowrange(v, t, np.zeros((1, 3), np.float32), np.array([[0, 0, 1]], np.float32), 1.0)
    assert not fl.any()
    assert np.array_equal(o[0].astype(np.int64), exp)
    assert exp[0].sum() > 0 and exp[63].sum() > 0


def test_degenerate_triangles_rowrange_equals_brute_force():
    """Points, segments, a triangle in a row plane, edges and vertices on row
    planes and an edge on the axis: the row-range algorithm equals the
    brute-force definition wherever neither flags a pixel, and each triangle
    flags exactly the pixels its contact with a row plane makes ambiguous, in
    that row: the triangle lying in row plane 40 the radii it covers (its
    farthest vertex is at 0.566, so columns 0..35); the edge in row plane 20
    the radii of that edge (0.25 .. 0.39: columns 16..24); the edge in row
    plane 10 the radii 0.15 .. 0.45 (columns 10..28).  A lone vertex on row
    plane 30 flags nothing: both sides of it give the same slice."""
    v, t = closed_forms.degenerate_triangles()
    sv, sn = np.zeros((1, 3), np.float32), np.array([[0, 0, 1]], np.float32)
    o, fl, _ = oracle.rici_rowrange(v, t, sv, sn, 1.0)
    ob, flb = oracle.rici_brute(v, t, sv, sn, 1.0)
    assert o.sum() > 0
    m = ~(fl | flb)
    assert np.array_equal(o[m], ob[m])
    expected = np.zeros((NB, NB), bool)
    expected[40, 0:36] = True
    expected[20, 16:25] = True
    expected[10, 10:29] = True
    assert np.array_equal(fl[0], expected)
    for k, (row, cols) in enumerate([(None, None), (None, None), (None, None), (40, range(0, 36)),
                                     (20, range(16, 25)), (10, range(10, 29)), (None, None)]):
        _, f1, _ = oracle.rici_rowrange(v, t[k:k + 1], sv, sn, 1.0)
        want = np.zeros((NB, NB), bool)
        if row is not None:
            want[row, list(cols)] = True
        assert np.array_equal(f1[0], want), k


def test_closed_surface_counts_are_even():
    s = synth.config2_union12()
    sel = np.random.default_rng(0).choice(s.num_haystack, 64, replace=False)
    im, fl, _ = oracle.rici_rowrange(s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], 0.3)
    assert im.max() > 2
    assert ((im % 2) == 0)[~fl].all()


def _dyadic_scene(rng):
    m = synth.superquadric(6, 0.7, 1.8, (1.0, 0.8, 0.6))
    pos = np.round(m.positions * 2 ** 20) / 2 ** 20
    pos = pos.astype(np.float32)
    assert np.array_equal(pos.astype(np.float64) * 2 ** 20, np.round(pos.astype(np.float64) * 2 ** 20))
    nrm = synth.vertex_normals(pos, m.triangles)
    return pos, m.triangles, nrm


@pytest.mark.parametrize("seed", range(3))
def test_signed_permutation_and_dyadic_translation(seed):
    rng = np.random.default_rng(seed)
    pos, tri, nrm = _dyadic_scene(rng)
    perm = rng.permutation(3)
    signs = rng.choice([-1.0, 1.0], size=3)
    Q = np.zeros((3, 3))
    Q[np.arange(3), perm] = signs
    shift = np.round(rng.uniform(-1, 1, 3) * 2 ** 20) / 2 ** 20
    pos2 = (pos.astype(np.float64) @ Q.T + shift).astype(np.float32)
    nrm2 = (nrm.astype(np.float64) @ Q.T).astype(np.float32)
    assert np.array_equal(pos2.astype(np.float64), pos.astype(np.float64) @ Q.T + shift)
    sel = np.arange(0, pos.shape[0], 7)
    a, fa, _ = oracle.rici_rowrange(pos, tri, pos[sel], nrm[sel], 0.6)
    b, fb, _ = oracle.rici_rowrange(pos2, tri, pos2[sel], nrm2[sel], 0.6)
    ok = ~(fa | fb)
    assert np.array_equal(a[ok], b[ok])
    assert a.max() > 0


@pytest.mark.parametrize("k", [-3, 2, 5])
def test_power_of_two_scaling_is_bit_identical(k):
    s = synth.config1_icosphere()
    f = np.float32(2.0 ** k)
    sel = np.arange(0, s.num_haystack, 5)
    a, _, _ = oracle.rici_rowrange(s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], 1.0)
    b, _, _ = oracle.rici_rowrange(s.positions * f, s.triangles, s.op_positions[sel] * f, s.op_normals[sel],
                                   float(f))
    assert np.array_equal(a, b)


def test_additivity_over_triangle_sets():
    s = synth.config2_union12()
    sel = np.arange(0, s.num_haystack, 997)
    T = s.triangles.shape[0]
    cut = T // 3
    a, _, _ = oracle.rici_rowrange(s.positions, s.triangles[:cut], s.op_positions[sel], s.op_normals[sel], 0.3)
    b, _, _ = oracle.rici_rowrange(s.positions, s.triangles[cut:], s.op_positions[sel], s.op_normals[sel], 0.3)
    c, _, _ = oracle.rici_rowrange(s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], 0.3)
    assert np.array_equal(a + b, c)


def test_empty_scene_and_zero_normal():
    op = np.array([[0, 0, 0], [1, 1, 1]], dtype=np.float32)
    nrm = np.array([[0, 0, 1], [0, 0, 0]], dtype=np.float32)
    im, fl, wk = oracle.rici_rowrange(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.uint32), op, nrm, 0.3)
    assert (im == 0).all() and (wk == 0).all()
    assert fl[1].all() and not fl[0].any()


def test_zero_normal_uses_plus_z_axis():
    s = synth.config1_icosphere()
    op = s.op_positions[:4]
    a, _, _ = oracle.rici_rowrange(s.positions, s.triangles, op, np.zeros_like(op), 1.0)
    b, _, _ = oracle.rici_rowrange(s.positions, s.triangles, op, np.tile(np.float32([0, 0, 1]), (4, 1)), 1.0)
    assert np.array_equal(a, b)


def test_bad_index_is_rejected():
    with pytest.raises(ValueError):
        oracle.rici_rowrange(np.zeros((3, 3), np.float32), np.array([[0, 1, 3]], np.uint32),
                             np.zeros((1, 3), np.float32), np.ones((1, 3), np.float32), 1.0)


def test_mesh_generators_are_watertight():
    for m in [synth.icosphere(2), synth.superquadric(5, 0.5, 2.0), synth.torus(9, 5, 0.7, 0.2)]:
        t = m.triangles.astype(np.int64)
        edges = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
        fwd = {tuple(e) for e in edges}
        assert len(fwd) == edges.shape[0]
        assert all((b, a) in fwd for a, b in fwd)
