"""GPU parity of the Spin Image path (rici_spin_generate, rici_spin_rank,
rici_spin_correlation_matrix) against the FP64 oracle (Sec. 2.1 with the
projection of Sec. 3.1.1; readings S1-S4).

Tolerance of a Spin Image pixel: the GPU adds the pixel's n contributions as
fp32 in arbitrary order, each an FP64 weight rounded once; the sum is then
within (n + 1) 2^-24 of the exact pixel value times that value (first-order
bound of an fp32 sum of non-negative terms), plus 1e-12 per contribution for
the FP64 projection's own rounding.  Pixels that a sample on the support
boundary reaches are flagged by the oracle and excused.

Ranks: the GPU settles every pair near the true match's correlation in FP64,
so its ranks must lie in the oracle's range for a band of 1e-12 when both see
the same fp32 images.  End to end (each side builds its own images) the band
follows from the pixel bound: 1e-4."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_f32, dev_u32, host_u32, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context
    c = Context(0)
    yield c
    c.close()


def _check_images(g, o, n, fl, what):
    bound = (n + 1.0) * 2.0 ** -24 * np.abs(o) * 1.01 + 1e-12 * (n + 1)
    bad = (np.abs(g.astype(np.float64) - o) > bound) & ~fl
    if bad.any():
        i = tuple(np.argwhere(bad)[0])
        raise AssertionError(f"{what}: {int(bad.sum())} pixels outside the bound; first {i}: gpu {g[i]!r} "
                             f"oracle {o[i]!r} contributions {n[i]}")
    return int(fl.sum())


def _gpu_spin(ctx, samples, opp, opn, R):
    out = ctx.spin_generate(dev_f32(samples), dev_f32(opp), dev_f32(opn), R)
    ctx.sync()
    return out.cpu().numpy()


def test_icosphere_every_image(ctx):
    s = synth.config1_icosphere()
    smp = synth.sample_surface(s.positions, s.triangles, np.random.default_rng(1), per_triangle=10)
    g = _gpu_spin(ctx, smp, s.op_positions, s.op_normals, s.support_radius)
    o, n, fl = oracle.spin_images(smp, s.op_positions, s.op_normals, s.support_radius)
    flagged = _check_images(g, o, n, fl, "icosphere")
    say(f"  icosphere: {len(smp)} samples, {flagged} flagged pixels, max image sum {o.sum(axis=(1, 2)).max():.1f}")
    assert o.sum() > 1000


def test_union12_sampled_at_full_size(ctx):
    s = synth.config2_union12()
    smp = synth.sample_surface(s.positions, s.triangles, np.random.default_rng(2), per_triangle=10)
    g = _gpu_spin(ctx, smp, s.op_positions, s.op_normals, s.support_radius)
    n_img = s.num_haystack
    sel = np.unique(np.concatenate([[0, 1, 2, 3, n_img - 1], np.random.default_rng(3).choice(n_img, 60, False)]))
    o, n, fl = oracle.spin_images(smp, s.op_positions[sel], s.op_normals[sel], s.support_radius)
    _check_images(g[sel], o, n, fl, "union12")
    say(f"  union12: {len(smp)} samples x {n_img} images, {len(sel)} checked")


def test_edge_cases(ctx):
    import torch
    from paper_2007_02306_amd import RiciError
    # no samples: zero images; a zero normal selects +z; one oriented point
    opp = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]], np.float32)
    opn = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.0]], np.float32)
    z = ctx.spin_generate(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), dev_f32(opp), dev_f32(opn), 0.5)
    ctx.sync()
    assert float(z.abs().sum()) == 0.0
    smp = np.array([[0.2, 0.0, 0.01], [0.0, 0.3, -0.1], [0.05, 0.05, 0.2]], np.float32)
    g = _gpu_spin(ctx, smp, opp, opn, 0.5)
    o, n, fl = oracle.spin_images(smp, opp, opn, 0.5)
    _check_images(g[1:], o[1:], n[1:], fl[1:], "small")
    _check_images(g[:1], o[:1], n[:1], np.zeros_like(fl[:1]), "zero normal as +z")
    with pytest.raises(RiciError):
        ctx.spin_generate(dev_f32(smp), dev_f32(opp), dev_f32(opn), -1.0)


def _random_images(rng, n):
    im = (rng.random((n, 64, 64)) ** 4 * 20).astype(np.float32)
    im[rng.random((n, 64, 64)) < 0.6] = 0.0
    return im


@pytest.mark.parametrize("nn,nh", [(1, 1), (37, 300), (130, 257), (200, 129)])
def test_rank_on_the_same_images(ctx, nn, nh):
    rng = np.random.default_rng(nn * 1000 + nh)
    hay = _random_images(rng, nh)
    src = rng.integers(0, nh, nn)
    needles = hay[src] + (rng.random((nn, 64, 64)) < 0.05).astype(np.float32) * rng.random((nn, 64, 64)).astype(
        np.float32) * 5
    t = src.astype(np.uint32)
    t[::3] = rng.integers(0, nh, len(t[::3]))           # unrelated true matches: ranks in the middle
    if nh > 3:
        hay[2] = hay[src[0]]                            # a duplicate of a true match
        hay[3] = 7.0                                    # a constant image
    if nn > 2:
        needles[1] = 0.0                                # a constant needle
    rk, rt = ctx.spin_rank(dev_f32(needles), dev_f32(hay), dev_u32(t))
    ctx.sync()
    g_rk, g_rt = host_u32(rk), rt.cpu().numpy()
    o_rk, lo, hi, o_rt = oracle.pearson_rank(needles, hay, t, band=1e-12)
    assert np.allclose(g_rt, o_rt, rtol=0, atol=1e-12)
    bad = (g_rk < lo) | (g_rk > hi)
    assert not bad.any(), (np.argwhere(bad)[:5].ravel(), g_rk[bad][:5], lo[bad][:5], hi[bad][:5])
    say(f"  {nn} x {nh}: ranks exact {int((g_rk == o_rk).sum())}/{nn}, max {int(o_rk.max())}")
    # the correlation matrix from the same contraction, within its bound
    m = ctx.spin_correlation_matrix(dev_f32(needles), dev_f32(hay))
    ctx.sync()
    om = oracle.pearson_matrix(needles, hay)
    assert np.abs(m.cpu().numpy().astype(np.float64) - om).max() < 2.5e-4


def test_rank_self_and_bad_index(ctx):
    rng = np.random.default_rng(9)
    hay = _random_images(rng, 300)
    t = np.arange(300, dtype=np.uint32)
    t[5] = 300                                          # out of range: rank = haystack size
    rk, rt = ctx.spin_rank(dev_f32(hay), dev_f32(hay), dev_u32(t))
    ctx.sync()
    g = host_u32(rk)
    assert g[5] == 300 and np.isinf(rt.cpu().numpy()[5])
    ok = np.arange(300) != 5
    # every image correlates 1 with itself: nothing ranks above it
    assert (g[ok] == 0).all()


def test_end_to_end_describe_and_rank(ctx):
    """Needles and haystack are Spin Images of the same 768 union12 vertices
    from two independent samplings of the surface (the true match of needle i
    is haystack image i): the GPU builds both sets and ranks; the oracle does
    the same from the same samples."""
    s = synth.config2_union12()
    sel = np.sort(np.random.default_rng(4).choice(s.num_haystack, 768, replace=False))
    opp, opn = s.op_positions[sel], s.op_normals[sel]
    smp_h = synth.sample_surface(s.positions, s.triangles, np.random.default_rng(5), per_triangle=10)
    smp_n = synth.sample_surface(s.positions, s.triangles, np.random.default_rng(6), per_triangle=10)
    gh = ctx.spin_generate(dev_f32(smp_h), dev_f32(opp), dev_f32(opn), s.support_radius)
    gn = ctx.spin_generate(dev_f32(smp_n), dev_f32(opp), dev_f32(opn), s.support_radius)
    t = np.arange(len(sel), dtype=np.uint32)
    rk, _ = ctx.spin_rank(gn, gh, dev_u32(t))
    ctx.sync()
    g_rk = host_u32(rk)
    oh, _, flh = oracle.spin_images(smp_h, opp, opn, s.support_radius)
    on, _, fln = oracle.spin_images(smp_n, opp, opn, s.support_radius)
    o_rk, lo, hi, _ = oracle.pearson_rank(on.astype(np.float32), oh.astype(np.float32), t, band=1e-4)
    bad = (g_rk < lo) | (g_rk > hi)
    assert not bad.any(), (np.argwhere(bad)[:5].ravel(), g_rk[bad][:5], lo[bad][:5], hi[bad][:5])
    say(f"  768 needles: {int((g_rk == o_rk).sum())} ranks equal the oracle's, rank-0 share "
        f"{float((o_rk == 0).mean()):.3f}, flagged images {int(flh.any(axis=(1, 2)).sum() + fln.any(axis=(1, 2)).sum())}")
