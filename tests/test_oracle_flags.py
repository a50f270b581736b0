"""Pins of the oracle's degeneracy flags and work counters.

A pixel is flagged when a decision that sets its count lies within 1e-9 (plus
the FP64 rounding bound of the compared quantity) of its threshold: (i) a
slice end at a bin radius, (ii) the foot point of a double range at a bin
radius, or a double range whose presence is uncertain, (iii) a vertex on the
row plane whose side changes the slice, (iv) an edge or a whole triangle in
the row plane.  Each rule is pinned by a constructed case that must flag its
own pixel, in its own row and nowhere else, and by the contrasting case just
outside its band, whose count the geometry then fixes.  The soundness of the
bands is pinned by an invariant: an FP64 rigid motion of a degenerate scene
changes the rounding of every quantity but not the exact counts, so the
counts of every pixel unflagged before and after must agree.

The work counters (slices S and pixel updates U, and the triangles and slices
that come closer to the axis than the support radius, which set the generation
kernel's algorithmic work) are pinned by closed forms.

Canonical frame throughout: oriented point at the origin with normal +z and
support radius 1, so rho_c = (c + 1/2) / 64 and beta_r = -1/2 + (r + 1/2) / 64.
"""

import numpy as np
import pytest

import closed_forms
import oracle
import synth

NB = 64
B = 1.0 / NB


def rho(c):
    return (c + 0.5) * B


def beta(r):
    return -0.5 + (r + 0.5) * B


def _run(pos, f64=False, tri=None, op=((0, 0, 0),), nrm=((0, 0, 1),), R=1.0):
    pos = np.asarray(pos, np.float64 if f64 else np.float32).reshape(-1, 3)
    if tri is None:
        tri = np.arange(pos.shape[0], dtype=np.uint32).reshape(-1, 3)
    return oracle.rici_rowrange(pos, tri, np.asarray(op), np.asarray(nrm), R, f64=f64)


def _only(flags, pixels):
    want = np.zeros((NB, NB), bool)
    for r, c in pixels:
        want[r, c] = True
    return np.array_equal(flags, want)


# --------------------------------------------------------------- (i) slice ends

def test_rule_i_slice_end_on_a_bin_radius():
    """A vertical edge at radius rho_20 crossing only row 40: the slice's end
    on it lies exactly on the bin circle, so (40, 20) is flagged and nothing
    else (the other end, at radius 0.354, is 0.17 bins from any circle)."""
    p = [(rho(20), 0, beta(40) - 0.004), (rho(20), 0, beta(40) + 0.004), (rho(20) + 0.05, 0.03, beta(40) + 0.002)]
    im, fl, _ = _run(p)
    assert _only(fl[0], [(40, 20)])
    assert (im[0, 40, 21:23] == 1).all() and im[0].sum() == 2


@pytest.mark.parametrize("off,count", [(1e-8, 0), (-1e-8, 1)])
def test_rule_i_band_is_narrow(off, count):
    """The same edge 1e-8 outside or inside the circle (ten times the
    tolerance): nothing is flagged, and column 20 is counted exactly when the
    circle lies inside the single range."""
    p = [(rho(20) + off, 0, beta(40) - 0.004), (rho(20) + off, 0, beta(40) + 0.004),
         (rho(20) + 0.05, 0.03, beta(40) + 0.002)]
    im, fl, _ = _run(p, f64=True)
    assert not fl.any()
    assert im[0, 40, 20] == count and (im[0, 40, 21:23] == 1).all()


@pytest.mark.parametrize("off", [5e-10, -5e-10])
def test_rule_i_band_inside_tolerance(off):
    p = [(rho(20) + off, 0, beta(40) - 0.004), (rho(20) + off, 0, beta(40) + 0.004),
         (rho(20) + 0.05, 0.03, beta(40) + 0.002)]
    _, fl, _ = _run(p, f64=True)
    assert _only(fl[0], [(40, 20)])


# ------------------------------------------------------ (ii) foot of the slice

def test_rule_ii_tangent_chord():
    """A triangle in the plane x = rho_30 crossing only row 40: its slice is a
    chord whose closest point to the axis lies exactly on the circle of column
    30 (tangency), so (40, 30) is flagged and nothing else."""
    x = rho(30)
    p = [(x, -0.2, beta(40) - 0.004), (x, 0.2, beta(40) - 0.004), (x, 0.0, beta(40) + 0.004)]
    im, fl, _ = _run(p)
    assert _only(fl[0], [(40, 30)])
    assert im[0].sum() == 0 or im[0, 40, 30] in (0, 2)


@pytest.mark.parametrize("off,count", [(1e-8, 0), (-1e-8, 2)])
def test_rule_ii_band_is_narrow(off, count):
    """The chord 1e-8 beyond or inside the circle: nothing is flagged, and the
    circle crosses the chord twice exactly when it reaches past it."""
    x = rho(30) + off
    p = [(x, -0.2, beta(40) - 0.004), (x, 0.2, beta(40) - 0.004), (x, 0.0, beta(40) + 0.004)]
    im, fl, _ = _run(p, f64=True)
    assert not fl.any()
    assert im[0, 40, 30] == count and im[0].sum() == count


@pytest.mark.parametrize("off,flagged", [(2e-8, True), (1e-7, False)])
def test_rule_ii_short_slice(off, flagged):
    """A sharp tip 2e-9 above row plane 20 gives a slice 4e-8 long at radius
    about rho_25 + off.  Its foot point is only known to within the slice's
    length, so a circle that close is flagged at (20, 25) -- and one 1e-7 away
    is not.  Either way no circle meets such a short slice (count 0)."""
    tip = np.array([rho(25) + off - 2e-8, 0.0, beta(20) + 2e-9])
    p = [tip, tip + (0.1, 0.1, -0.01 - 2e-9), tip + (0.1, -0.1, -0.01 - 2e-9)]
    im, fl, wk = _run(p, f64=True)
    assert wk[0, 1] == 1                       # one slice: row 20 only
    assert im[0].sum() == 0
    assert _only(fl[0], [(20, 25)] if flagged else [])


# ------------------------------------------------ (iii) a vertex on the plane

def test_rule_iii_vertex_on_row_plane_at_a_bin_radius():
    """A vertex exactly on row plane 10 at radius rho_15, the triangle's other
    vertices above and below it: (10, 15) is flagged, and no other pixel --
    in particular none in row 20."""
    k = np.array([rho(15), 0.0, beta(10)])
    p = [k, k + (0.1, 0.05, 0.01), k + (0.1, -0.05, -0.01)]
    _, fl, _ = _run(p)
    assert _only(fl[0], [(10, 15)])


def test_rule_iii_vertex_on_row_plane_between_radii():
    """The vertex 1e-7 beyond the circle instead: taking it on either side of
    the plane moves the slice's end by at most 1e-8, so nothing is flagged and
    the count is certain (0 at column 15, 1 from 16 to 21)."""
    k = np.array([rho(15) + 1e-7, 0.0, beta(10)])
    p = [k, k + (0.1, 0.05, 0.01), k + (0.1, -0.05, -0.01)]
    im, fl, _ = _run(p, f64=True)
    assert not fl.any()
    assert im[0, 10, 15] == 0 and (im[0, 10, 16:22] == 1).all() and im[0].sum() == 6


@pytest.mark.parametrize("rise,flagged", [(1e-6, True), (0.01, False)])
def test_rule_iii_flat_neighbour_widens_the_band(rise, flagged):
    """A vertex on row plane 10, 1.5e-9 beyond the circle of column 15, with a
    neighbour that rises by `rise` over 0.11.  Taken below the plane, the
    vertex makes the slice end on the edge to that neighbour, whose crossing
    moves by ~2e-9 per ulp of height error when the edge rises by only 1e-6:
    the circle 1.5e-9 away is then flagged.  A steep neighbour leaves the
    band at 1e-9, and the circle is not."""
    k = np.array([rho(15) + 1.5e-9, 0.0, beta(10)])
    p = [k, k + (0.1, 0.05, rise), k + (0.1, -0.05, -0.01)]
    im, fl, _ = _run(p, f64=True)
    assert _only(fl[0], [(10, 15)] if flagged else [])
    assert im[0, 10, 15] == 0


# ------------------------------------------- (iv) edges and triangles in a plane

@pytest.mark.parametrize("r", [3, 20, 50])
def test_rule_iv_triangle_in_row_plane(r):
    """A triangle lying in row plane r around the axis flags every radius it
    covers (its farthest vertex is at 0.566: columns 0..35) in row r only."""
    p = [(-0.4, -0.4, beta(r)), (0.4, -0.3, beta(r)), (0.0, 0.5, beta(r))]
    _, fl, _ = _run(p)
    assert _only(fl[0], [(r, c) for c in range(36)])


@pytest.mark.parametrize("r", [5, 40])
def test_rule_iv_edge_in_row_plane(r):
    """An edge in row plane r at distance 0.25 from the axis, out to radius
    0.39: columns 16..24 of row r, and nothing else."""
    p = [(-0.3, 0.25, beta(r)), (0.3, 0.25, beta(r)), (0.0, 0.25, beta(r) + 0.1)]
    _, fl, _ = _run(p)
    assert _only(fl[0], [(r, c) for c in range(16, 25)])


# ------------------------------------------- flat edges (rounding-bound widening)

@pytest.mark.parametrize("rise,flagged", [(4e-9, True), (0.01, False)])
def test_flat_edge_widens_the_band_of_its_crossing(rise, flagged):
    """An edge of length 0.3 crossing row plane 20 at its middle, 1e-6 beyond
    the circle of column 22.  When the edge rises by only 4e-9 (its ends stay
    2e-9 from the plane, outside the 1e-9 band), an ulp of height error moves
    the crossing by ~1e-6, so the circle is flagged, in row 20 only.  A steep
    edge leaves the band at 1e-9: nothing is flagged, and the circle lies
    inside the single range, whose ends are the crossing (0.3516) and the
    middle of the edge to the third vertex (0.2945)."""
    x = rho(22) + 1e-6
    p = [(x - 0.15, 0.0, beta(20) - rise / 2), (x + 0.15, 0.0, beta(20) + rise / 2),
         (x, 0.2, beta(20) + 0.005)]
    im, fl, _ = _run(p, f64=True)
    assert _only(fl[0], [(20, 22)] if flagged else [])
    if not flagged:
        assert (im[0, 20, 19:23] == 1).all() and im[0].sum() == 4


def test_flat_edge_within_the_band_is_an_edge_in_the_plane():
    """An edge rising by 1e-13 across row plane 20 lies within 1e-9 of it
    along its whole length: every radius it covers (0.2 .. 0.5, columns
    12..31) is flagged in row 20, and nothing elsewhere."""
    p = [(0.2, 0.0, beta(20) - 5e-14), (0.5, 0.0, beta(20) + 5e-14), (0.35, 0.2, beta(20) + 0.005)]
    _, fl, _ = _run(p, f64=True)
    rows, cols = np.nonzero(fl[0])
    assert set(rows.tolist()) == {20}
    assert set(range(12, 32)) <= set(cols.tolist()) and cols.max() == 31 and cols.min() >= 8


def test_fp32_flat_edge():
    """The flattest edge fp32 can hold (one ulp of height): flagged around its
    crossing in its own row."""
    z = np.float32(beta(20))
    z1 = np.nextafter(z, np.float32(1))
    p = np.array([(0.2, 0.0, z), (0.5, 0.0, z1), (0.35, 0.2, z + np.float32(0.005))], np.float32)
    _, fl, _ = _run(p)
    rows, _ = np.nonzero(fl[0])
    assert set(rows.tolist()) <= {20}


# ---------------------------------------------------- soundness of the bands

def _snapped_scene(rng, nt=30):
    z = beta(rng.integers(0, NB, size=(nt, 3)))
    z[::3, 1] = z[::3, 0]
    z[::7, :] = z[::7, :1]
    r = rho(rng.integers(0, NB, size=(nt, 3))) + rng.choice([0.0, 1e-12, -3e-10, 2e-9], size=(nt, 3))
    a = rng.uniform(0, 2 * np.pi, size=(nt, 3))
    return np.stack([r * np.cos(a), r * np.sin(a), z], -1).reshape(-1, 3)


def _flat_and_short(rng, n=24):
    """Flat edges (ends 1.5e-9 .. 1e-8 from a row plane, just outside the
    1e-9 band) crossing it within 3e-8 of a bin radius, where the crossing's
    actual rounding error (~1e-8) can move it across the circle, and sharp
    tips 1e-9 .. 1e-7 above a row plane within 5e-8 of a bin radius (short
    slices)."""
    out = []
    for _ in range(n):
        rr = int(rng.integers(2, 60))
        h = 10.0 ** rng.uniform(np.log10(1.5e-9), -8)
        x = rho(int(rng.integers(5, 50))) + rng.uniform(-3e-8, 3e-8)
        out += [(x - 0.15, 0.0, beta(rr) - h), (x + 0.15, 0.0, beta(rr) + h), (x, 0.2, beta(rr) + 0.004)]
        tip = np.array([rho(int(rng.integers(0, 60))) + rng.uniform(-5e-8, 5e-8), 0.0,
                        beta(rr) + 10.0 ** rng.uniform(-9, -7)])
        out += [tip, tip + (0.1, 0.1, -0.01), tip + (0.1, -0.1, -0.01)]
    return np.array(out)


def _moved(pos, rng):
    """Rigid motion in FP64: positions, oriented point and normal rotated by
    a uniform random rotation and translated by up to 0.5."""
    Q = synth.random_rotation(rng)
    t = rng.uniform(-0.5, 0.5, 3)
    return pos @ Q.T + t, Q @ np.zeros(3) + t, Q @ np.array([0.0, 0.0, 1.0])


@pytest.mark.parametrize("scene", ["degenerate", "snapped", "flat_and_short"])
def test_unflagged_counts_survive_rigid_motions(scene):
    rng = np.random.default_rng({"degenerate": 1, "snapped": 2, "flat_and_short": 3}[scene])
    if scene == "degenerate":
        v, t = closed_forms.degenerate_triangles()
        pos, tri = v.astype(np.float64), t
    elif scene == "snapped":
        pos = _snapped_scene(rng)
        tri = np.arange(len(pos), dtype=np.uint32).reshape(-1, 3)
    else:
        pos = _flat_and_short(rng)
        tri = np.arange(len(pos), dtype=np.uint32).reshape(-1, 3)
    a, fa, _ = oracle.rici_rowrange(pos, tri, np.zeros((1, 3)), np.array([[0.0, 0, 1]]), 1.0, f64=True)
    assert fa.any() and a.sum() > 0
    differ = 0
    for _ in range(12):
        p2, s2, n2 = _moved(pos, rng)
        b, fb, _ = oracle.rici_rowrange(p2, tri, s2[None], n2[None], 1.0, f64=True)
        ok = ~(fa | fb)
        assert np.array_equal(a[ok], b[ok])
        differ += int((a != b).sum())
    assert differ > 0 or scene == "degenerate"   # the motions do change flagged counts


# ----------------------------------------------------------- work counters

def _segment_updates(p, q, foot):
    """Pixels a slice from p to q changes.  `foot` is None when the axis's
    foot point lies outside the slice: then the radii strictly between the
    two ends.  Otherwise it is the foot's distance from the axis, and the
    slice changes every radius above it and below the far end (the double
    range up to the nearer end, then the single range)."""
    d0, d1 = np.hypot(*p), np.hypot(*q)
    lo, hi = min(d0, d1), max(d0, d1)
    rr = rho(np.arange(NB))
    if foot is None:
        return int(((rr > lo) & (rr < hi)).sum())
    return int(((rr > foot) & (rr < hi) & (rr != lo)).sum())


def test_work_counters_planar_square():
    """Square in the plane y = 0 spanning x in (-L1, L2) and heights (b0, b1),
    split on the diagonal from (-L1, b0) to (L2, b1).  Every row inside its
    height cuts both triangles: S = 2 per row.  At height beta the diagonal
    sits at xd; the lower-right triangle's slice runs from xd to L2 and the
    upper-left one's from -L1 to xd, each holding the axis's foot (x = 0)
    iff it straddles 0."""
    L1, L2, b0, b1 = (np.float64(np.float32(v)) for v in (0.7, 0.45, -0.31, 0.23))
    v = np.array([[-L1, 0, b0], [L2, 0, b0], [L2, 0, b1], [-L1, 0, b1]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    _, fl, wk = _run(v, tri=t)
    assert not fl.any()
    rows = [r for r in range(NB) if b0 < beta(r) < b1]
    U = 0
    per_add = 0
    for r in rows:
        f = (beta(r) - b0) / (b1 - b0)
        xd = -L1 + f * (L1 + L2)
        for (p, q) in (((xd, 0), (L2, 0)), ((-L1, 0), (xd, 0))):
            inside = min(p[0], q[0]) < 0 < max(p[0], q[0])
            u = _segment_updates(p, q, 0.0 if inside else None)
            U += u
            lo = min(abs(p[0]), abs(q[0]))
            per_add += u + (int((rho(np.arange(NB)) < lo).sum()) if inside else 0)
    assert wk[0, 0] == 2 and wk[0, 1] == 2 * len(rows)
    assert wk[0, 2] == U
    assert per_add > U          # counting each +2 twice would be caught
    # every slice lies within R = 1 of the axis
    assert wk[0, 3] == 2 and wk[0, 4] == 2 * len(rows)


@pytest.mark.parametrize("x0,x1", [(0.8, 1.4), (1.2, 1.5), (0.3, 0.9)])
def test_work_counters_inside_the_support_radius(x0, x1):
    """Square in the plane y = 0 with x in (x0, x1) > 0, heights (b0, b1),
    split on the diagonal from (x0, b0) to (x1, b1).  At height beta the
    diagonal sits at xd; the upper-left slice runs from x0 to xd (nearest
    point x0), the lower-right one from xd to x1 (nearest point xd).  A slice
    counts as inside when its nearest point is closer to the axis than R = 1;
    a triangle when any of its slices is."""
    b0, b1 = np.float64(np.float32(-0.31)), np.float64(np.float32(0.23))
    x0, x1 = np.float64(np.float32(x0)), np.float64(np.float32(x1))
    v = np.array([[x0, 0, b0], [x1, 0, b0], [x1, 0, b1], [x0, 0, b1]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    _, fl, wk = _run(v, tri=t)
    rows = [r for r in range(NB) if b0 < beta(r) < b1]
    xd = [x0 + (beta(r) - b0) / (b1 - b0) * (x1 - x0) for r in rows]
    s_in = sum(int(x0 < 1.0) + int(x < 1.0) for x in xd)
    t_in = int(x0 < 1.0) + int(any(x < 1.0 for x in xd))
    assert wk[0, 1] == 2 * len(rows)
    assert wk[0, 3] == t_in and wk[0, 4] == s_in
    if x0 >= 1.0:
        assert wk[0, 2] == 0 and s_in == 0
    assert 0 < s_in < 2 * len(rows) or x0 >= 1.0 or x1 < 1.0


@pytest.mark.parametrize("y,inside", [(0.9, True), (1.05, False), (0.99, True)])
def test_work_counters_chord_uses_its_foot_point(y, inside):
    """A square in the plane y = const spanning x in (-0.3, 0.3): every slice
    straddles the axis's foot point, so its nearest point is at distance y
    although both ends lie farther out (sqrt(y^2 + 0.09) > 1 for y >= 0.96)."""
    v = np.array([[-0.3, y, -0.31], [0.3, y, -0.31], [0.3, y, 0.23], [-0.3, y, 0.23]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.uint32)
    _, fl, wk = _run(v, tri=t)
    V = v.astype(np.float64)
    b0, b1, yy, xa = V[0, 2], V[2, 2], V[0, 1], V[1, 0]
    rows = [r for r in range(NB) if b0 < beta(r) < b1]
    # per row: the slice that straddles x = 0 comes as close as y; the other
    # one ends at the diagonal's crossing xd, its nearest point
    s_in = 0
    for r in rows:
        xd = -xa + (beta(r) - b0) / (b1 - b0) * 2 * xa
        s_in += int(yy < 1.0) + int(np.hypot(xd, yy) < 1.0)
    assert wk[0, 1] == 2 * len(rows)
    assert wk[0, 4] == s_in
    if inside:
        assert wk[0, 3] == 2 and s_in >= len(rows)
    else:
        assert wk[0, 3] == 0 and s_in == 0 and wk[0, 2] == 0


def test_work_counters_bin_radius_boundaries():
    """The radial rectangles and chords of the bin-radius scene span heights
    -0.31 .. 0.23: 35 rows, each cutting all 512 triangles, S = 17 920.  A
    rectangle from p0 to p1 (bottom) is split on its diagonal; at height
    fraction f the lower triangle's slice runs from p0 + f (p1 - p0) to p1 and
    the upper one's from p0 to that point.  Radial rectangles point away from
    the axis (no foot point inside); a chord's slice holds its foot point iff
    it straddles the chord's middle."""
    v, t, _ = closed_forms.bin_radius_boundaries()
    _, fl, wk = _run(v, tri=t)
    assert not fl.any()
    V = v.astype(np.float64)
    b0, b1 = V[0, 2], V[2, 2]
    rows = [r for r in range(NB) if b0 < beta(r) < b1]
    assert len(rows) == 35
    U = 0
    for k in range(0, len(V), 4):
        p0, p1 = V[k, :2], V[k + 1, :2]
        chord = (k // 4) % 2 == 1
        foot, dist = 2.0, None
        if chord:
            d = p1 - p0
            foot = -(p0 @ d) / (d @ d)            # parameter of the axis's foot along p0 -> p1
            dist = abs(p0[0] * p1[1] - p0[1] * p1[0]) / np.hypot(*d)
        for r in rows:
            f = (beta(r) - b0) / (b1 - b0)
            m = p0 + f * (p1 - p0)
            U += _segment_updates(m, p1, dist if f < foot else None)
            U += _segment_updates(p0, m, dist if chord and f > foot else None)
    assert wk[0, 0] == len(t) and wk[0, 1] == 35 * len(t)
    assert wk[0, 2] == U
