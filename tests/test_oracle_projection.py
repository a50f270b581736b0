"""Pins of the oracle's projection (Sec. 3.1.1, Eq. 1-5) against the plain
geometric definition of the cylindrical coordinates (Sec. 2.1: alpha is the
distance to the Central Axis, beta the signed height along it from the Spin
Vertex)."""

import numpy as np
import pytest

import oracle


def _plain(sv, sn, pts):
    sv = np.asarray(sv, dtype=np.float64)
    n = np.asarray(sn, dtype=np.float64)
    n = n / np.linalg.norm(n)
    d = pts - sv
    beta = d @ n
    alpha = np.linalg.norm(d - beta[:, None] * n[None, :], axis=1)
    return alpha, beta


@pytest.mark.parametrize("seed", range(6))
def test_eq1_to_5_matches_axis_distance_and_height(seed):
    rng = np.random.default_rng(seed)
    sv = rng.uniform(-1, 1, 3).astype(np.float32)
    sn = rng.normal(size=3).astype(np.float32)
    pts = rng.uniform(-2, 2, size=(500, 3))
    a, b, _ = oracle.project(sv, sn, pts)
    a0, b0 = _plain(sv, sn, pts)
    assert np.max(np.abs(a - a0)) < 1e-12
    assert np.max(np.abs(b - b0)) < 1e-12


@pytest.mark.parametrize("sn", [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0, 1, 0), (0, -3, 0),
                                (0.6, -0.8, 0), (0, 2, 5), (1e-30, 0, 1)])
def test_special_normals(sn):
    rng = np.random.default_rng(7)
    sv = np.array([0.25, -0.5, 0.125], dtype=np.float32)
    pts = rng.uniform(-1, 1, size=(200, 3))
    a, b, _ = oracle.project(sv, sn, pts)
    a0, b0 = _plain(sv, sn, pts)
    assert np.allclose(a, a0, atol=1e-12) and np.allclose(b, b0, atol=1e-12)


def test_zero_normal_is_identity_frame():
    # Sec. 3.1.1: a rotation whose coefficients are both zero is the identity,
    # so the axis is +z and (T_x, T_y, T_z) = P - S_v.
    sv = np.array([0.5, 0.25, -0.75], dtype=np.float32)
    pts = np.random.default_rng(3).uniform(-1, 1, size=(50, 3))
    a, b, txy = oracle.project(sv, (0, 0, 0), pts)
    d = pts - sv.astype(np.float64)
    assert np.array_equal(b, d[:, 2])
    assert np.array_equal(txy, d[:, :2])


def test_spin_normal_maps_to_plus_z():
    rng = np.random.default_rng(11)
    for _ in range(20):
        sn = rng.normal(size=3).astype(np.float32)
        sv = np.zeros(3, dtype=np.float32)
        a, b, _ = oracle.project(sv, sn, sn.astype(np.float64)[None, :])
        assert abs(a[0]) < 1e-12 and abs(b[0] - np.linalg.norm(sn.astype(np.float64))) < 1e-12


def test_printed_eq1_is_not_an_alignment():
    """Reading R1: Eq. 1 as printed normalises (S_nx, S_nz) for the second
    rotation, which misplaces points whenever S_ny != 0; the corrected line
    (normalising the first rotation's output) agrees with the definition."""
    rng = np.random.default_rng(5)
    sv = np.zeros(3, dtype=np.float32)
    sn = np.array([0.3, 0.8, 0.52], dtype=np.float32)
    pts = rng.uniform(-1, 1, size=(1000, 3))
    a0, b0 = _plain(sv, sn, pts)
    a1, b1, _ = oracle.project(sv, sn, pts, printed_eq1=True)
    assert np.max(np.abs(b1 - b0)) > 0.1
    a2, b2, _ = oracle.project(sv, sn, pts, printed_eq1=False)
    assert np.max(np.abs(b2 - b0)) < 1e-12
    # with S_ny == 0 both readings coincide
    sn2 = np.array([0.3, 0.0, 0.52], dtype=np.float32)
    _, b3, _ = oracle.project(sv, sn2, pts, printed_eq1=True)
    _, b4, _ = oracle.project(sv, sn2, pts)
    assert np.max(np.abs(b3 - b4)) < 1e-15


def test_rotation_about_axis_keeps_alpha_beta():
    rng = np.random.default_rng(9)
    sv = np.array([0.1, 0.2, 0.3], dtype=np.float32)
    sn = np.array([0.0, 0.0, 1.0], dtype=np.float32)
    pts = rng.uniform(-1, 1, size=(100, 3))
    th = 0.7
    rot = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    moved = (pts - sv) @ rot.T + sv
    a, b, _ = oracle.project(sv, sn, pts)
    a2, b2, _ = oracle.project(sv, sn, moved)
    assert np.allclose(a, a2, atol=1e-12) and np.allclose(b, b2, atol=1e-12)
