"""Pins of the clutter oracle (Eq. 8 with reading C1: areas inside the
support cylinder alpha <= R, |beta| <= R/2).

Closed forms in the frame of the axis (z) and the Spin Vertex (origin): a
horizontal plane inside the slab holds the disc pi R^2 and one outside it
nothing; a vertical plane at distance d from the axis holds the strip
2 sqrt(R^2 - d^2) x R; a plane through the origin tilted by theta holds the
part of the ellipse s^2 + (t cos theta)^2 <= R^2 with |t sin theta| <= R/2,
whose area is an elementary integral.  Planes within a hair of vertical are
checked against scipy's adaptive quadrature of the same cross-section length,
random triangles against Monte Carlo, and splitting a triangle must not
change its area.  Eq. 8 itself is pinned on two patches of known area."""

import numpy as np
import pytest

import oracle
import synth

R = 0.3


def _square(corners):
    a, b, c, d = (np.asarray(x, np.float64) for x in corners)
    return oracle.triangle_area_in_volume(a, b, c, R) + oracle.triangle_area_in_volume(a, c, d, R)


@pytest.mark.parametrize("z,want", [(0.0, np.pi * R * R), (0.1, np.pi * R * R), (-0.149, np.pi * R * R),
                                    (0.2, 0.0), (-0.16, 0.0)])
def test_horizontal_plane_holds_the_disc(z, want):
    got = _square([[-1, -1, z], [1, -1, z], [1, 1, z], [-1, 1, z]])
    assert got == pytest.approx(want, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("d", [0.0, 0.1, 0.29, 0.31])
def test_vertical_plane_holds_a_strip(d):
    got = _square([[-1, d, -1], [1, d, -1], [1, d, 1], [-1, d, 1]])
    want = 2.0 * np.sqrt(max(R * R - d * d, 0.0)) * R
    assert got == pytest.approx(want, rel=1e-13, abs=1e-15)


def _tilted(theta, extent=3.0):
    c, s = np.cos(theta), np.sin(theta)
    e1, e2 = np.array([1.0, 0, 0]), np.array([0.0, c, s])
    return [x * extent for x in (-e1 - e2, e1 - e2, e1 + e2, -e1 + e2)]


def _ellipse_in_slab(theta):
    c, s = np.cos(theta), np.sin(theta)
    T = min(R / (2 * s), R / c) if s > 0 else R / c
    d = c * T
    F = lambda x: 0.5 * (x * np.sqrt(max(R * R - x * x, 0.0)) + R * R * np.arcsin(np.clip(x / R, -1, 1)))
    return 2.0 * (F(d) - F(-d)) / c


@pytest.mark.parametrize("tan_theta", [0.0, 0.3, 0.5, 1.0, 3.0, 40.0])
def test_tilted_plane_holds_a_clipped_ellipse(tan_theta):
    theta = np.arctan(tan_theta)
    got = _square(_tilted(theta))
    want = _ellipse_in_slab(theta)
    assert got == pytest.approx(want, rel=1e-12)
    if tan_theta <= 0.5:
        assert got == pytest.approx(np.pi * R * R / np.cos(theta), rel=1e-12)   # the whole ellipse


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9, 1e-12])
def test_nearly_vertical_planes_against_quadrature(eps):
    """A plane tilted eps from vertical, offset 0.2 from the axis: the
    cross-section at in-plane height t is |s| <= sqrt(R^2 - (a2 + k t)^2)."""
    from scipy import integrate
    theta = np.pi / 2 - eps
    c, s = np.cos(theta), np.sin(theta)
    off = np.array([0.0, 0.2, 0.0])
    corners = [x + off for x in _tilted(theta, 1.0)]
    got = _square(corners)
    # in-plane coordinates: e1 = x, e2 = (0, c, s); a point (s, t) sits at
    # y = 0.2 + t c, z = t s; the slab bounds t by R / (2 s)
    T = 0.5 * R / s
    f = lambda t: 2.0 * np.sqrt(max(R * R - (0.2 + t * c) ** 2, 0.0))
    want, _ = integrate.quad(f, -T, T, epsabs=1e-15, epsrel=1e-13, limit=200)
    assert got == pytest.approx(want, rel=1e-11)


def test_random_triangles_against_monte_carlo():
    rng = np.random.default_rng(4)
    for _ in range(12):
        P = rng.uniform(-0.35, 0.35, size=(3, 3))
        got = oracle.triangle_area_in_volume(P[0], P[1], P[2], R)
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        n = 400_000
        r1, r2 = np.sqrt(rng.random(n)), rng.random(n)
        X = (1 - r1)[:, None] * P[0] + (r1 * (1 - r2))[:, None] * P[1] + (r1 * r2)[:, None] * P[2]
        inside = (X[:, 0] ** 2 + X[:, 1] ** 2 <= R * R) & (np.abs(X[:, 2]) <= R / 2)
        frac = inside.mean()
        sigma = np.sqrt(max(frac * (1 - frac), 1e-12) / n)
        assert abs(got / area - frac) < 5 * sigma + 1e-9, (got / area, frac)


def test_splitting_a_triangle_keeps_its_area():
    rng = np.random.default_rng(5)
    for _ in range(20):
        P = rng.uniform(-0.4, 0.4, size=(3, 3))
        m = 0.5 * (P[1] + P[2])
        whole = oracle.triangle_area_in_volume(P[0], P[1], P[2], R)
        parts = oracle.triangle_area_in_volume(P[0], P[1], m, R) + oracle.triangle_area_in_volume(P[0], m, P[2], R)
        assert parts == pytest.approx(whole, rel=1e-12, abs=1e-16)


def _patch(cx, cy, z, half):
    v = np.array([[cx - half, cy - half, z], [cx + half, cy - half, z], [cx + half, cy + half, z],
                  [cx - half, cy + half, z]], np.float32)
    return v, np.array([[0, 1, 2], [0, 2, 3]], np.uint32)


def test_eq8_on_two_patches():
    """Object: a 0.1 x 0.1 patch at the Spin Vertex; clutter: a 0.2 x 0.2
    patch 0.05 above it and one outside the volume.  A_all = 0.05,
    A_object = 0.01, clutter 0.8."""
    v0, t0 = _patch(0.0, 0.0, 0.0, 0.05)
    v1, t1 = _patch(0.0, 0.0, 0.05, 0.1)
    v2, t2 = _patch(0.0, 0.0, 0.4, 0.1)
    pos = np.concatenate([v0, v1, v2])
    tri = np.concatenate([t0, t1 + 4, t2 + 8])
    a_all, a_obj = oracle.clutter_areas(pos, tri, 0, 2, np.zeros((1, 3)), np.array([[0.0, 0, 1]]), R)
    # the patches are fp32: their sides are 0.1 and 0.2 to within 1e-8
    assert a_all[0] == pytest.approx(0.05, rel=1e-6)
    assert a_obj[0] == pytest.approx(0.01, rel=1e-6)
    assert (a_all[0] - a_obj[0]) / a_all[0] == pytest.approx(0.8, rel=1e-6)


def test_areas_follow_the_scene_under_rigid_motion():
    rng = np.random.default_rng(6)
    s = synth.config1_icosphere()
    idx = rng.choice(s.num_haystack, 8, replace=False)
    a, o = oracle.clutter_areas(s.positions, s.triangles, 0, 100, s.op_positions[idx], s.op_normals[idx], 0.6)
    rot = synth.random_rotation(rng)
    shift = rng.uniform(-1, 1, 3)
    p2 = (s.positions.astype(np.float64) @ rot.T + shift).astype(np.float32)
    a2, o2 = oracle.clutter_areas(p2, s.triangles, 0, 100, s.op_positions[idx].astype(np.float64) @ rot.T + shift,
                                  s.op_normals[idx].astype(np.float64) @ rot.T, 0.6)
    assert np.allclose(a, a2, rtol=1e-5) and np.allclose(o, o2, rtol=1e-5, atol=1e-9)
    assert (a > 0).all() and (o <= a + 1e-15).all()
    # the whole closed surface: every triangle counted once
    full, _ = oracle.clutter_areas(s.positions, s.triangles, 0, 0, np.zeros((1, 3)), np.array([[0.0, 0, 1]]), 100.0)
    v = s.positions.astype(np.float64)[s.triangles.astype(np.int64)]
    total = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1).sum()
    assert full[0] == pytest.approx(total, rel=1e-12)


def _xy_projection_reference(P, R):
    """The area inside the volume by an independent route: clip the triangle
    to the slab, project it onto the xy plane (areas scale by |m_z|), and
    integrate the length of (polygon cross-section) x (disc cross-section)
    over x with adaptive quadrature."""
    from scipy import integrate
    poly = [np.asarray(p, np.float64) for p in P]

    def clip(pl, f):
        out = []
        for a, b in zip(pl, pl[1:] + pl[:1]):
            fa, fb = f(a), f(b)
            if fa >= 0:
                out.append(a)
            if (fa >= 0) != (fb >= 0):
                out.append(a + fa / (fa - fb) * (b - a))
        return out
    poly = clip(clip(poly, lambda x: R / 2 - x[2]), lambda x: x[2] + R / 2)
    if len(poly) < 3:
        return 0.0
    n = np.cross(P[1] - P[0], P[2] - P[0])
    mz = abs(n[2]) / np.linalg.norm(n)
    xy = np.array([[p[0], p[1]] for p in poly])

    def length(x):
        ys = []
        for a, b in zip(xy, np.roll(xy, -1, axis=0)):
            if (a[0] - x) * (b[0] - x) <= 0 and a[0] != b[0]:
                ys.append(a[1] + (x - a[0]) / (b[0] - a[0]) * (b[1] - a[1]))
        if len(ys) < 2 or abs(x) >= R:
            return 0.0
        w = np.sqrt(R * R - x * x)
        return max(0.0, min(max(ys), w) - max(min(ys), -w))
    # the integrand has kinks at the polygon's vertices and where its edges
    # cross the circle: all are breakpoints of the quadrature
    pts = set(xy[:, 0].tolist())
    for a, b in zip(xy, np.roll(xy, -1, axis=0)):
        d = b - a
        A, B, C = d @ d, 2 * (a @ d), a @ a - R * R
        disc = B * B - 4 * A * C
        if A > 0 and disc >= 0:
            for r in ((-B - np.sqrt(disc)) / (2 * A), (-B + np.sqrt(disc)) / (2 * A)):
                if 0 < r < 1:
                    pts.add(float(a[0] + r * d[0]))
    val, _ = integrate.quad(length, -R, R, points=sorted(p for p in pts if -R < p < R), limit=1000,
                            epsabs=1e-16, epsrel=1e-14)
    return val / mz


def test_triangles_across_the_boundary_against_an_independent_route():
    """Triangles straddling the cylinder near tangency and the slab ends, in
    planes no steeper than 60 degrees (where the projection route is well
    conditioned): the piecewise closed form must match adaptive quadrature in
    the projection to 1e-13 of R^2 (a form of the root's integral that
    cancels near tangency is off by up to 1e-9)."""
    rng = np.random.default_rng(12)
    worst = 0.0
    for _ in range(300):
        c = rng.normal(size=2)
        c = c / np.linalg.norm(c) * rng.uniform(0.26, 0.32)
        P = np.concatenate([c + rng.normal(0, 0.04, (3, 2)), rng.uniform(-0.19, 0.19, (3, 1))], axis=1)
        n = np.cross(P[1] - P[0], P[2] - P[0])
        if abs(n[2]) < 0.5 * np.linalg.norm(n):
            continue
        got = oracle.triangle_area_in_volume(P[0], P[1], P[2], R)
        want = _xy_projection_reference(list(P), R)
        worst = max(worst, abs(got - want))
    assert worst < 1e-13 * R * R


def _scene_triangle_near_tangency():
    """A triangle of a seeded clutter scene, in the frame of one of the
    reference vertices, whose first piece starts at a tangency of the
    cylinder (found by search once; fixed by its seed and indices)."""
    rng = np.random.default_rng(21)
    mesh, canon, _, _ = synth.configs.clutter_scene(rng, 4, 2000, 6000)
    pos = mesh.positions.astype(np.float32).astype(np.float64)
    nrm = synth.vertex_normals(mesh.positions.astype(np.float32), mesh.triangles).astype(np.float64)
    sel = np.unique(np.linspace(0, canon[0].num_vertices - 1, 300).astype(int))
    i = sel[129]
    n = nrm[i] / np.linalg.norm(nrm[i])
    u = np.cross(n, [1.0, 0.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    q = pos[mesh.triangles[11637].astype(np.int64)] - pos[i]
    return np.stack([q @ u, q @ w, q @ n], axis=1)      # any frame with z along the normal


def test_area_is_well_conditioned_at_tangency():
    """Moving the vertices by a few units in the last place moves the area by
    about as much; a form of the root's integral whose two halves cancel near
    tangency moves it by 1e-4 of its value."""
    P = _scene_triangle_near_tangency()
    base = oracle.triangle_area_in_volume(P[0], P[1], P[2], R)
    assert base > 1e-4
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(400):
        Q = P.copy()
        steps = rng.integers(-3, 4, size=Q.shape)
        for _ in range(3):
            Q = np.where(steps > 0, np.nextafter(Q, np.inf), np.where(steps < 0, np.nextafter(Q, -np.inf), Q))
            steps = steps - np.sign(steps)
        worst = max(worst, abs(oracle.triangle_area_in_volume(Q[0], Q[1], Q[2], R) - base))
    assert worst < 1e-13 * base
