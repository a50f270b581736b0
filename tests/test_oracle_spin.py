"""Pins of the Spin Image and Pearson oracle (Sec. 2.1 with the projection of
Sec. 3.1.1; readings S1-S4 of the oracle).

Closed forms in the canonical frame (oriented point at the origin, normal +z,
support radius 1: bin width d = 1/64, bin centres at alpha = (c + 1/2) d and
beta = -1/2 + (r + 1/2) d): a sample at a bin centre adds exactly 1 to that
bin; one between centres splits by the bilinear weights; samples in the outer
half bins lose the weight of the missing neighbour; samples outside the
support volume add nothing.  The projection and the spreading together are
pinned against an independent formulation (alpha and beta as distance from and
height along the normal axis, spread with numpy), which must agree on scenes
in random frames; the sum over an image counts the samples well inside the
volume; a rigid motion of the whole scene leaves images unchanged.  The
Pearson coefficient is pinned by its invariants and against numpy.corrcoef,
ranks by brute force."""

import numpy as np
import pytest

import oracle
import synth

NB = 64
D = 1.0 / NB


def _canon(points):
    pts = np.asarray(points, np.float32).reshape(-1, 3)
    return oracle.spin_images(pts, np.zeros((1, 3)), np.array([[0.0, 0.0, 1.0]]), 1.0)


def _beta(r):
    return -0.5 + (r + 0.5) * D


@pytest.mark.parametrize("r,c", [(0, 0), (31, 7), (40, 63), (63, 12)])
def test_sample_at_a_bin_centre(r, c):
    im, cnt, fl = _canon([[(c + 0.5) * D, 0.0, _beta(r)]])
    want = np.zeros((NB, NB))
    want[r, c] = 1.0
    assert np.array_equal(im[0], want)
    assert cnt[0, r, c] == 1 and cnt[0].sum() == 1
    assert not fl.any()


def test_bilinear_weights_between_centres():
    r, c = 20, 30
    im, cnt, _ = _canon([[0.0, (c + 0.75) * D, _beta(r) + 0.5 * D]])   # on the y axis: alpha = |y|
    want = np.zeros((NB, NB))
    want[r, c], want[r, c + 1], want[r + 1, c], want[r + 1, c + 1] = 0.375, 0.125, 0.375, 0.125
    assert np.array_equal(im[0], want)
    assert cnt[0].sum() == 4


def test_outer_half_bins_drop_the_missing_neighbour():
    r = 10
    im, _, _ = _canon([[0.25 * D, 0.0, _beta(r)], [0.0, -63.75 * D, _beta(r + 5)],
                       [0.5 * D, 0.0, -0.5 + 0.25 * D]])
    assert im[0, r, 0] == 0.75                  # u = -1/4: three quarters to column 0
    assert im[0, r + 5, 63] == 0.75             # u = 63.25: three quarters to column 63
    assert im[0, 0, 0] == 0.75                  # v = -1/4 at the bottom row
    assert np.isclose(im[0].sum(), 2.25, rtol=0, atol=1e-15)


def test_samples_outside_the_support_volume_add_nothing():
    pts = [[1.0, 0.0, 0.0], [0.0, 1.5, 0.1], [0.2, 0.0, 0.5], [0.2, 0.0, -0.50001], [0.75, 0.75, 0.0]]
    im, cnt, fl = _canon(pts)
    assert im.sum() == 0.0 and cnt.sum() == 0
    # alpha = 1 exactly and beta = 1/2 exactly sit on the boundary: their
    # pixels are flagged; the far ones flag nothing
    assert fl[0, :, 63].any() and fl[0, 63, :].any()
    far, _, ffar = _canon([[0.0, 1.5, 0.1], [0.75, 0.75, 0.0]])
    assert not ffar.any()


def _plain_definition(samples, sv, sn, R):
    """alpha = distance from the normal axis, beta = height along it; the
    bilinear spreading of reading S2 with numpy."""
    n = np.asarray(sn, np.float64) / np.linalg.norm(sn)
    q = samples.astype(np.float64) - np.asarray(sv, np.float64)
    beta = q @ n
    alpha = np.linalg.norm(q - beta[:, None] * n[None, :], axis=1)
    keep = (alpha < R) & (beta >= -R / 2) & (beta < R / 2)
    u = alpha[keep] / (R / NB) - 0.5
    v = (beta[keep] + R / 2) / (R / NB) - 0.5
    c0, r0 = np.floor(u).astype(int), np.floor(v).astype(int)
    fu, fv = u - c0, v - r0
    img = np.zeros((NB + 2, NB + 2))
    for dr, dc, w in ((0, 0, (1 - fu) * (1 - fv)), (0, 1, fu * (1 - fv)), (1, 0, (1 - fu) * fv), (1, 1, fu * fv)):
        np.add.at(img, (r0 + dr + 1, c0 + dc + 1), w)
    return img[1:-1, 1:-1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_projection_and_spreading_match_the_plain_definition(seed):
    rng = np.random.default_rng(seed)
    s = synth.config1_icosphere()
    samples = synth.sample_surface(s.positions, s.triangles, rng, per_triangle=20)
    idx = rng.choice(s.num_haystack, 6, replace=False)
    R = float(np.float32(rng.uniform(0.4, 1.5)))          # the support radius is an fp32 input
    im, _, fl = oracle.spin_images(samples, s.op_positions[idx], s.op_normals[idx], R)
    for k, i in enumerate(idx):
        ref = _plain_definition(samples, s.op_positions[i].astype(np.float64), s.op_normals[i].astype(np.float64), R)
        ok = ~fl[k]
        assert np.allclose(im[k][ok], ref[ok], rtol=0, atol=1e-9)
        assert im[k].sum() > 10


def test_image_sum_counts_the_samples_well_inside():
    rng = np.random.default_rng(7)
    n = 5000
    a = rng.uniform(1.0 * D, 1.0 - 1.0 * D, n)
    th = rng.uniform(0, 2 * np.pi, n)
    b = rng.uniform(-0.5 + 1.0 * D, 0.5 - 1.0 * D, n)
    pts = np.stack([a * np.cos(th), a * np.sin(th), b], axis=1)
    # three samples outside
    pts = np.concatenate([pts, [[1.2, 0, 0], [0, 0, 0.6], [0.3, 0.3, -0.7]]])
    im, _, fl = _canon(pts)
    assert not fl.any()
    assert abs(im.sum() - n) < 1e-9


def test_rigid_motion_leaves_images_unchanged():
    rng = np.random.default_rng(11)
    s = synth.config1_icosphere()
    samples = synth.sample_surface(s.positions, s.triangles, rng, per_triangle=10).astype(np.float64)
    idx = rng.choice(s.num_haystack, 5, replace=False)
    sv, sn = s.op_positions[idx].astype(np.float64), s.op_normals[idx].astype(np.float64)
    rot = synth.random_rotation(rng)
    shift = rng.uniform(-0.5, 0.5, 3)
    a, _, fa = oracle.spin_images(samples.astype(np.float32), sv, sn, 0.8)
    # the motion is applied in FP64 and rounded to fp32 once, as the inputs are
    b, _, fb = oracle.spin_images((samples @ rot.T + shift).astype(np.float32), sv @ rot.T + shift, sn @ rot.T, 0.8)
    ok = ~(fa | fb)
    # fp32 rounding of the moved samples shifts them by ~1e-7: bilinear weights move by that times 64 / R
    assert np.allclose(a[ok], b[ok], rtol=0, atol=1e-4)
    assert a.sum() > 50


def test_zero_normal_flags_the_image():
    im, _, fl = oracle.spin_images(np.array([[0.1, 0.0, 0.0]], np.float32), np.zeros((1, 3)), np.zeros((1, 3)), 1.0)
    assert fl.all()


# ---------------------------------------------------------------- Pearson

def test_pearson_invariants_and_numpy():
    rng = np.random.default_rng(3)
    x = rng.random((64, 64)).astype(np.float32)
    y = rng.random((64, 64)).astype(np.float32)
    assert oracle.pearson(x, 2.0 * x + 3.0) == pytest.approx(1.0, abs=1e-12)
    assert oracle.pearson(x, -0.5 * x + 1.0) == pytest.approx(-1.0, abs=1e-12)
    assert oracle.pearson(x, y) == pytest.approx(np.corrcoef(x.ravel().astype(np.float64),
                                                             y.ravel().astype(np.float64))[0, 1], abs=1e-13)
    assert oracle.pearson(x, y) == oracle.pearson(y, x)
    assert oracle.pearson(x, np.full((64, 64), 5.0, np.float32)) == 0.0     # S3: constant image
    assert oracle.pearson(np.zeros((64, 64), np.float32), np.zeros((64, 64), np.float32)) == 0.0


def test_pearson_matrix_and_rank_against_brute_force():
    rng = np.random.default_rng(5)
    hay = (rng.random((40, 64, 64)) ** 3).astype(np.float32)
    hay[7] = hay[3]                                       # a duplicate of a true match: a tie
    needles = hay[[3, 10, 20, 33]] + rng.normal(0, 0.05, (4, 64, 64)).astype(np.float32)
    needles[2] = 1.0                                      # a constant needle: every correlation 0
    t = np.array([3, 10, 20, 33], np.uint32)
    m = oracle.pearson_matrix(needles, hay)
    for i in range(4):
        for j in range(40):
            if i == 2:
                assert m[i, j] == 0.0
            else:
                assert m[i, j] == pytest.approx(np.corrcoef(needles[i].ravel().astype(np.float64),
                                                            hay[j].ravel().astype(np.float64))[0, 1], abs=1e-13)
    rk, lo, hi, rt = oracle.pearson_rank(needles, hay, t, band=1e-3)
    for i in range(4):
        ref = int((m[i] > m[i, t[i]]).sum())
        assert rk[i] == ref and rt[i] == m[i, t[i]]
        others = np.arange(40) != t[i]
        assert lo[i] == int((m[i][others] > m[i, t[i]] + 1e-3).sum())
        assert hi[i] == int((m[i][others] > m[i, t[i]] - 1e-3).sum())
        assert lo[i] <= rk[i] <= hi[i]
    assert rk[2] == 0 and hi[2] == 39      # constant needle: all tie at 0
    assert hi[0] >= 1                      # the duplicate ties with the true match
    with pytest.raises(ValueError):
        oracle.pearson_rank(needles, hay, np.array([0, 0, 0, 40], np.uint32))
