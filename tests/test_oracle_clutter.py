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
