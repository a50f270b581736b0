"""GPU parity of the clutter-resistant distance search (rici_distance_matrix,
rici_distance_rank) against the oracle: exact integers, always."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_u32, gpu_images, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context
    c = Context(0)
    yield c
    c.close()


def gpu_matrix(ctx, n, h):
    say(f"  gpu matrix: {len(n)} x {len(h)}")
    out = ctx.distance_matrix(dev_u32(n), dev_u32(h))
    ctx.sync()
    return out.cpu().numpy()


def gpu_rank(ctx, n, h, t):
    say(f"  gpu rank: {len(n)} needles x {len(h)} haystack")
    rk, ds = ctx.distance_rank(dev_u32(n), dev_u32(h), dev_u32(np.asarray(t, np.uint32)))
    ctx.sync()
    return rk.cpu().numpy().view(np.uint32), ds.cpu().numpy()


@pytest.mark.parametrize("nn,nh,scale", [(1, 1, 2), (37, 53, 2), (16, 256, 3), (257, 300, 2), (300, 17, 11)])
def test_matrix_small_deltas(ctx, nn, nh, scale):
    rng = np.random.default_rng(nn * 1000 + nh)
    n = synth.step_images(rng, nn, delta_scale=scale)
    h = synth.step_images(rng, nh, delta_scale=scale)
    assert np.array_equal(gpu_matrix(ctx, n, h), oracle.distance_matrix(n, h))


@pytest.mark.parametrize("nmax,hmax", [(11, 12), (11, 127), (127, 11), (127, 127), (128, 11), (11, 128), (300, 500),
                                       (15, 15), (15, 16), (16, 15)])
def test_matrix_delta_ranges(ctx, nmax, hmax):
    """Every arithmetic path: |D_h| <= 15 (two phases), 15 < |D_h| <= 127
    (three phases), |D| > 127 (int64 path) on either side."""
    rng = np.random.default_rng(nmax * 7 + hmax)
    n = synth.step_images(rng, 70, delta_scale=3)
    h = synth.step_images(rng, 90, delta_scale=3)
    n[5] = synth.step_images(rng, 1, max_delta=nmax, density=0.05)[0]
    n[5, 3, 10] += nmax          # force the extreme delta
    h[40] = synth.step_images(rng, 1, max_delta=hmax, density=0.05)[0]
    h[40, 60, 33] += hmax
    n[6] = h[40]
    got = gpu_matrix(ctx, n, h)
    assert np.array_equal(got, oracle.distance_matrix(n, h))


def _exact_step_images(rng, n, peak):
    """Sparse small steps plus one step of exactly `peak` (so max |D| = peak)
    per image; `peak` <= 2 keeps only the small steps."""
    im = synth.step_images(rng, n, density=0.05, delta_scale=2).astype(np.int64)
    if peak > 2:
        for k in range(n):
            r, c = rng.integers(0, 64), rng.integers(1, 64)
            im[k, r, c:] += peak - (im[k, r, c] - im[k, r, c - 1])   # that delta becomes exactly peak
    return im.astype(np.uint32)


@pytest.mark.parametrize("tile", [256, 128])
def test_extreme_deltas_at_the_accumulator_bound(tile):
    """Images whose 4 032 deltas are all +-127 (ramps up and down, zigzags),
    flat images (no mask) and their mixes: the largest distances the int8
    contraction can meet (4 032 * 254^2 between opposite ramps), exact
    against the oracle in the matrix and in the ranks."""
    from paper_2007_02306_amd import Context
    c = Context(0)
    c.set_tuning("search_tile_m", tile)
    col = np.arange(64, dtype=np.uint32)
    up = np.tile(col * 127, (64, 1))
    down = np.tile((63 - col) * 127, (64, 1))
    zig = np.tile((col % 2) * 127, (64, 1))
    zag = np.tile(((col + 1) % 2) * 127, (64, 1))
    flat = np.full((64, 64), 5000, np.uint32)
    mixed = np.where((np.arange(64) % 2)[:, None] == 0, up, zag).astype(np.uint32)
    base = np.stack([up, down, zig, zag, flat, mixed]).astype(np.uint32)
    rng = np.random.default_rng(tile)
    h = np.concatenate([base, base[rng.integers(0, 6, 300)]])
    n = np.concatenate([base, base[::-1]])
    o = oracle.distance_matrix(n, h)
    assert o.max() == 4032 * 254 * 254
    assert np.array_equal(gpu_matrix(c, n, h), o)
    t = rng.integers(0, len(h), len(n)).astype(np.uint32)
    rk, ds = gpu_rank(c, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)
    c.close()


@pytest.mark.parametrize("tile,exit_", [(256, 0), (128, 0), (256, 1)])
def test_delta_range_boundaries(tile, exit_):
    """Haystack and needle images whose largest delta sits exactly on each side
    of the two-phase limit (15), the int8 limit (127) and in between, mixed in
    one haystack: exact matrix and ranks against the oracle, for both tile
    heights and with the early exit."""
    from paper_2007_02306_amd import Context
    c = Context(0)
    c.set_tuning("search_tile_m", tile)
    c.set_tuning("search_early_exit", exit_)
    rng = np.random.default_rng(tile + exit_)
    peaks = [0, 11, 12, 15, 16, 17, 60, 127, 128]
    h = np.concatenate([_exact_step_images(rng, 40, p) for p in peaks])
    for i, p in zip(range(0, len(h), 40), peaks):
        d = np.abs(np.diff(h[i:i + 40].astype(np.int64), axis=2)).max(axis=(1, 2))
        assert (d >= p).all() and (p < 3 or (d == p).all())
    t = rng.integers(0, len(h), 200).astype(np.uint32)
    n = synth.perturb(rng, h[t], frac=0.01)
    n[:9] = np.stack([_exact_step_images(rng, 1, p)[0] for p in peaks])
    t[:9] = rng.integers(0, len(h), 9)
    if not exit_:
        assert np.array_equal(gpu_matrix(c, n, h), oracle.distance_matrix(n, h))
    rk, ds = gpu_rank(c, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)
    c.close()


@pytest.mark.parametrize("seed", range(3))
def test_rank_with_ties(ctx, seed):
    rng = np.random.default_rng(seed)
    nh, nn = 333, 129
    h = synth.step_images(rng, nh, density=0.03)
    h[10] = h[11]
    h[12] = h[11]
    t = rng.integers(0, nh, nn).astype(np.uint32)
    t[0] = 11
    n = synth.perturb(rng, h[t], frac=0.01)
    n[0] = h[11]
    rk, ds = gpu_rank(ctx, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods)
    assert np.array_equal(rk, ork)
    assert rk[0] == 0 and rk.max() <= nh - 1


def test_rank_mixed_ranges(ctx):
    rng = np.random.default_rng(9)
    h = synth.step_images(rng, 500, delta_scale=2)
    h[100:110] = synth.step_images(rng, 10, max_delta=60, density=0.04)
    h[200:203] = synth.step_images(rng, 3, max_delta=400, density=0.02)
    t = rng.integers(0, 500, 90).astype(np.uint32)
    t[:6] = [100, 101, 200, 201, 5, 6]
    n = synth.perturb(rng, h[t], frac=0.02)
    n[50] = synth.step_images(rng, 1, max_delta=200, density=0.03)[0]
    rk, ds = gpu_rank(ctx, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)


def test_rank_large_haystack_sampled(ctx):
    """70 000 haystack images (beyond 2^16), 600 needles; the oracle ranks a
    seeded sample of needles over the full haystack."""
    rng = np.random.default_rng(77)
    nh, nn = 70_000, 600
    h = synth.step_images(rng, nh, density=0.06)
    t = rng.integers(0, nh, nn).astype(np.uint32)
    n = synth.perturb(rng, h[t], frac=0.03)
    rk, ds = gpu_rank(ctx, n, h, t)
    sel = np.unique(np.concatenate([[0, nn - 1], rng.choice(nn, 10, replace=False)]))
    ork, ods = oracle.rank(n[sel], h, t[sel])
    assert np.array_equal(ds[sel], ods) and np.array_equal(rk[sel], ork)
    assert (rk < nh).all()


def test_config1_end_to_end(ctx):
    """Icosphere: GPU images -> GPU ranks versus oracle images -> oracle ranks,
    with a shuffled true-match map so that ranks are not trivially 0."""
    s = synth.config1_icosphere()
    g = gpu_images(ctx, s.positions, s.triangles, s.op_positions, s.op_normals, s.support_radius)
    o, fl, _ = oracle.rici_rowrange(s.positions, s.triangles, s.op_positions, s.op_normals, s.support_radius)
    assert not fl.any()
    rng = np.random.default_rng(1)
    t = rng.permutation(s.num_haystack).astype(np.uint32)
    rk, ds = gpu_rank(ctx, g, g, t)
    ork, ods = oracle.rank(o, o, t)
    assert np.array_equal(rk, ork) and np.array_equal(ds, ods)
    assert rk.max() > 0
    rk0, ds0 = gpu_rank(ctx, g, g, np.arange(s.num_haystack))
    assert (rk0 == 0).all() and (ds0 == 0).all()
    assert np.array_equal(gpu_matrix(ctx, g, g), oracle.distance_matrix(o, o))


def test_benchmark_sized_search_sampled(ctx):
    """Search at the benchmark's size (23 352 x 23 352) on seeded step images;
    a sample of needles is ranked by the oracle over the full haystack."""
    rng = np.random.default_rng(2)
    n_img = 23_352
    h = synth.step_images(rng, n_img, density=0.05)
    t = rng.permutation(n_img).astype(np.uint32)
    n = synth.perturb(rng, h[t], frac=0.01)
    rk, ds = gpu_rank(ctx, n, h, t)
    sel = np.unique(np.concatenate([[0, n_img - 1], rng.choice(n_img, 14, replace=False)]))
    ork, ods = oracle.rank(n[sel], h, t[sel])
    assert np.array_equal(ds[sel], ods) and np.array_equal(rk[sel], ork)


def test_bad_true_index_and_empty(ctx):
    rng = np.random.default_rng(3)
    h = synth.step_images(rng, 20)
    t = np.array([0, 25, 2], np.uint32)
    rk, ds = gpu_rank(ctx, h[:3], h, t)
    assert rk[1] == 20 and rk[0] == 0 and rk[2] == 0
    import torch
    from paper_2007_02306_amd import RiciError
    e_rk, e_ds = ctx.distance_rank(torch.zeros((0, 64, 64), dtype=torch.int32, device="cuda"), dev_u32(h),
                                   torch.zeros(0, dtype=torch.int32, device="cuda"))
    ctx.sync()
    assert e_rk.numel() == 0
    with pytest.raises(RiciError):
        ctx.distance_rank(dev_u32(h[:2]), torch.zeros((0, 64, 64), dtype=torch.int32, device="cuda"),
                          dev_u32(np.zeros(2, np.uint32)))


def test_misaligned_images_rejected(ctx):
    """Image arrays are read with 16-byte vector loads: a pointer off that
    boundary is an argument error reported before any work is enqueued."""
    import torch
    from paper_2007_02306_amd import RiciError
    rng = np.random.default_rng(5)
    h = dev_u32(synth.step_images(rng, 4))
    flat = torch.zeros(4 * 4096 + 1, dtype=torch.int32, device="cuda")
    flat[1:].copy_(h.reshape(-1))
    off = flat[1:].view(4, 64, 64)                 # 4 bytes past a 16-byte boundary
    t = dev_u32(np.arange(4, dtype=np.uint32))
    with pytest.raises(RiciError) as e:
        ctx.distance_rank(off, h, t)
    assert "16-byte" in str(e.value)
    with pytest.raises(RiciError):
        ctx.distance_rank(h, off, t)
    rk, _ = ctx.distance_rank(h, h, t)             # the handle stays usable
    ctx.sync()
    assert rk.cpu().numpy().tolist() == [0, 0, 0, 0]


@pytest.fixture()
def ctx128():
    from paper_2007_02306_amd import Context
    c = Context(0)
    c.set_tuning("search_tile_m", 128)
    assert c.get_tuning("search_tile_m") == 128
    yield c
    c.close()


@pytest.mark.parametrize("nn,nh", [(1, 5), (127, 300), (129, 257), (385, 700)])
def test_small_tile_matches_oracle(ctx128, nn, nh):
    """The 128-needle search tile: same exact matrix and ranks (ragged needle
    counts on both sides of a tile, every delta range)."""
    rng = np.random.default_rng(nn + 31 * nh)
    h = synth.step_images(rng, nh, delta_scale=3)
    h[nh // 2] = synth.step_images(rng, 1, max_delta=90, density=0.05)[0]
    h[nh - 1] = synth.step_images(rng, 1, max_delta=300, density=0.02)[0]
    t = rng.integers(0, nh, nn).astype(np.uint32)
    t[0] = nh // 2
    n = synth.perturb(rng, h[t], frac=0.02)
    assert np.array_equal(gpu_matrix(ctx128, n, h), oracle.distance_matrix(n, h))
    rk, ds = gpu_rank(ctx128, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)


def test_tuning_rejects_bad_values(ctx):
    from paper_2007_02306_amd import RiciError
    with pytest.raises(RiciError):
        ctx.set_tuning("search_tile_m", 64)
    with pytest.raises(RiciError):
        ctx.set_tuning("no_such_knob", 1)
    with pytest.raises(RiciError):
        ctx.set_tuning("gen_images_per_group", 3)
    with pytest.raises(RiciError):
        ctx.set_tuning("search_early_exit", 2)
    with pytest.raises(RiciError):
        ctx.set_tuning("gen_sort_triangles", 3)
    assert ctx.get_tuning("gen_sort_triangles") == 2
    assert ctx.get_tuning("search_tile_m") == 256
    assert ctx.get_tuning("gen_images_per_group") == 2


@pytest.fixture()
def ctx_exit():
    from paper_2007_02306_amd import Context
    c = Context(0)
    assert c.get_tuning("search_early_exit") == 0        # off unless asked for
    c.set_tuning("search_early_exit", 1)
    yield c
    c.close()


@pytest.mark.parametrize("tile", [256, 128])
def test_early_exit_ranks_equal(ctx_exit, tile):
    """Tiles that leave early (every partial distance of the last phase at or
    above the needle's threshold) change no rank: near-duplicate needles (small
    thresholds, most tiles leave) and far ones, every delta range."""
    ctx_exit.set_tuning("search_tile_m", tile)
    rng = np.random.default_rng(40 + tile)
    nh, nn = 1500, 300
    h = synth.step_images(rng, nh, density=0.04)
    h[100:140] = synth.step_images(rng, 40, max_delta=60, density=0.04)
    h[200:203] = synth.step_images(rng, 3, max_delta=300, density=0.02)
    t = rng.integers(0, nh, nn).astype(np.uint32)
    t[:4] = [100, 120, 200, 5]
    n = synth.perturb(rng, h[t], frac=0.002)
    # the second half are images of other haystack entries: large thresholds
    n[150:] = synth.perturb(rng, h[rng.integers(0, nh, nn - 150)], frac=0.01)
    rk, ds = gpu_rank(ctx_exit, n, h, t)
    ork, ods = oracle.rank(n, h, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)
    assert (rk == 0).sum() > 10 and rk.max() > 0


def test_early_exit_clutter_sampled(ctx_exit):
    """Clutter scene: GPU needle and haystack images, ranks with the early exit
    against the oracle's ranks of the same images for a sample of needles."""
    s = synth.config3_clutter()
    rng = np.random.default_rng(5)
    hsel = np.sort(rng.choice(s.num_haystack, 3000, replace=False))
    nsel = np.sort(rng.choice(s.num_needles, 64, replace=False))
    hay = gpu_images(ctx_exit, s.positions, s.triangles, s.op_positions[hsel], s.op_normals[hsel], s.support_radius)
    nd = gpu_images(ctx_exit, s.needle_positions, s.needle_triangles, s.needle_op_positions[nsel],
                    s.needle_op_normals[nsel], s.support_radius)
    # true matches: the needles' own vertices where sampled, else a seeded image
    t = rng.integers(0, len(hsel), len(nsel)).astype(np.uint32)
    rk, ds = gpu_rank(ctx_exit, nd, hay, t)
    ork, ods = oracle.rank(nd, hay, t)
    assert np.array_equal(ds, ods) and np.array_equal(rk, ork)
