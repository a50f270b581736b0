"""GPU parity of the paired search: a set of images ranked against itself
(rici_distance_rank with the same array as needles and haystack, and every
mesh of a batched plan) takes the tile-pair path, where the tile pair (I, J)
serves both directions and computes the cross term <D_a, D_b> once when all
its images have |D| <= 15.  Ranks and true-match distances (Sec. 4.1 step 6c,
ties to the best rank, distance of Sec. 3.2 Eq. 6-7) must equal the oracle's
and the unpaired path's bit for bit, for every mix of arithmetic classes:
tiles with only small deltas (shared cross term), tiles with 15 < |D| <= 127
(a q phase: both directions computed separately), images with |D| > 127
(exact int64 path), padding, and out-of-range true indices."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_u32, host_u32, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context
    c = Context(0)
    yield c
    c.close()


def _set(seed: int, n: int, big: float = 0.0, huge: int = 0) -> np.ndarray:
    """n images: perturbed copies of a smaller base (so that ranks are
    neither all 0 nor all large), a share `big` with steps up to 60 and
    `huge` images with a step above 127."""
    rng = np.random.default_rng(seed)
    base = synth.step_images(rng, max(1, n // 3), density=0.1, delta_scale=2)
    imgs = synth.perturb(rng, base[rng.integers(0, len(base), n)], frac=0.03, amount=2)
    if big > 0:
        sel = rng.random(n) < big
        imgs[sel] = synth.step_images(rng, int(sel.sum()), density=0.05, max_delta=60)
    for k in rng.choice(n, min(huge, n), replace=False):
        imgs[k, rng.integers(0, 64), rng.integers(1, 64):] += 200
    return imgs


def _truth(seed: int, n: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    return rng.permutation(n).astype(np.uint32)


def _same(got, want, what):
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (f"{what}: {bad.size} of {got.size} differ; first "
                           + ", ".join(f"[{i}] gpu {got[i]} oracle {want[i]}" for i in bad[:6]))


def _rank(ctx, imgs, t, pairs: int):
    ctx.set_tuning("search_pairs", pairs)
    d = dev_u32(imgs)
    rk, ds = ctx.distance_rank(d, d, dev_u32(t))
    ctx.sync()
    return host_u32(rk), ds.cpu().numpy()


@pytest.mark.parametrize("n,big,huge", [(1, 0, 0), (5, 0, 0), (255, 0, 0), (256, 0, 0), (257, 0, 0), (700, 0, 0),
                                        (1500, 0.0, 3), (1500, 0.05, 0), (2600, 0.07, 4), (3000, 0.5, 2)])
def test_paired_ranks_equal_oracle_and_unpaired(ctx, n, big, huge):
    imgs = _set(n * 31 + int(big * 100) + huge, n, big, huge)
    t = _truth(n, n)
    say(f"  paired set of {n} images, {big:.0%} with |D| up to 60, {huge} above 127")
    p_rk, p_ds = _rank(ctx, imgs, t, 1)
    u_rk, u_ds = _rank(ctx, imgs, t, 0)
    o_rk, o_ds = oracle.rank(imgs, imgs, t)
    ctx.set_tuning("search_pairs", 1)
    _same(p_ds, o_ds, "paired true distances")
    _same(p_rk, o_rk, "paired ranks")
    _same(u_ds, o_ds, "unpaired true distances")
    _same(u_rk, o_rk, "unpaired ranks")
    if n > 100:
        assert int(o_rk.max()) > 0 and int(np.median(o_rk)) < n - 1   # ranks are not trivial


def test_paired_cross_terms_beyond_int16(ctx):
    """Dense images whose steps all have |D| = 15 (rows alternating 0 and 15,
    or 15 and 0) share tiles with sparse ones: the kept cross term
    -2 <D_a, D_b> reaches 2 * 63 * 64 * 225 = 1 814 400 for two equal dense
    images, past the int16 form, so those waves keep it as int32 while the
    sparse waves use int16.  Ranks and distances must equal the oracle's."""
    rng = np.random.default_rng(77)
    n = 900
    imgs = synth.step_images(rng, n, density=0.1, delta_scale=2)
    dense = rng.random(n) < 0.4
    cols = np.arange(64)
    for k in np.flatnonzero(dense):
        phase = rng.integers(0, 2, size=64)                       # per row: which columns hold 15
        imgs[k] = np.where(((cols[None, :] + phase[:, None]) % 2) == 1, 15, 0).astype(np.uint32)
        imgs[k, rng.integers(0, 64, 3)] = 0                         # a few flat rows: not all equal
    assert int(np.abs(np.diff(imgs.astype(np.int64), axis=2)).max()) == 15
    t = _truth(91, n)
    p_rk, p_ds = _rank(ctx, imgs, t, 1)
    o_rk, o_ds = oracle.rank(imgs, imgs, t)
    _same(p_ds, o_ds, "paired true distances")
    _same(p_rk, o_rk, "paired ranks")


def test_paired_true_distances_with_deltas_beyond_2_30(ctx):
    """The pass that finds each image's statistics and true-match distance
    works in 32 bits while every delta of both images stays below 2^30 and
    takes the exact int64 sum otherwise.  Images with one step of about 2^30
    up, or down, in the same pixel: the true match of W0 is W1, so the
    difference of their deltas there is about 2^31 (past int32); W2's true
    match is an ordinary image, and an ordinary image's true match is W3.
    Every sum stays below 2^63.  Ranks and distances must equal the oracle's
    (these images have |D| > 127, so their ranks come from the exact path)."""
    n = 700
    imgs = _set(2024, n)
    t = _truth(2024, n)
    w = [17, 300, 511, 650]
    big = [(1 << 30) + 12345, (1 << 30) + 777, (1 << 30) + 5, (1 << 30) + 99]
    r0, c0 = 9, 40
    imgs[w[0], r0, c0:] += np.uint32(big[0])          # one delta of +big[0] at (r0, c0)
    imgs[w[1], r0, :c0] += np.uint32(big[1])          # one delta of about -big[1] at the same pixel
    imgs[w[2], 33, 5:] += np.uint32(big[2])
    imgs[w[3], 50, 63:] += np.uint32(big[3])
    t[w[0]] = w[1]
    t[w[2]] = 3
    t[123] = w[3]
    d0 = np.diff(imgs[w[0]].astype(np.int64), axis=1)[r0, c0 - 1]
    d1 = np.diff(imgs[w[1]].astype(np.int64), axis=1)[r0, c0 - 1]
    assert d0 >= 1 << 30 and d1 <= -(1 << 30) and d0 - d1 > (1 << 31)
    p_rk, p_ds = _rank(ctx, imgs, t, 1)
    o_rk, o_ds = oracle.rank(imgs, imgs, t)
    assert int(o_ds[w[0]]) > 1 << 62 and int(o_ds.max()) < 1 << 63
    _same(p_ds, o_ds, "paired true distances")
    _same(p_rk, o_rk, "paired ranks")


def test_paired_identity_truth_and_duplicates(ctx):
    """t(i) = i gives rank 0 for every image; exact duplicates tie at the
    true distance 0 and keep the best rank."""
    rng = np.random.default_rng(7)
    imgs = synth.step_images(rng, 600, density=0.1, delta_scale=2)
    imgs[300:400] = imgs[0:100]                      # duplicates across tiles
    t = np.arange(600, dtype=np.uint32)
    rk, ds = _rank(ctx, imgs, t, 1)
    assert not rk.any() and not ds.any()
    t2 = t.copy()
    t2[:100] += 300                                  # the duplicate is the "true match": distance 0, rank 0
    rk2, ds2 = _rank(ctx, imgs, t2, 1)
    o_rk, o_ds = oracle.rank(imgs, imgs, t2)
    assert np.array_equal(rk2, o_rk) and np.array_equal(ds2, o_ds)
    assert not rk2[:100].any()


def test_paired_out_of_range_true_index(ctx):
    imgs = _set(11, 900)
    t = _truth(11, 900)
    bad = np.array([0, 255, 256, 899])
    t[bad] = 900 + np.arange(4, dtype=np.uint32)
    rk, ds = _rank(ctx, imgs, t, 1)
    assert np.array_equal(rk[bad], np.full(4, 900, np.uint32))
    good = np.setdiff1d(np.arange(900), bad)
    o_rk, o_ds = oracle.rank(imgs[good], imgs, t[good])
    assert np.array_equal(rk[good], o_rk) and np.array_equal(ds[good], o_ds)


def test_paired_repeated_calls_are_identical(ctx):
    """The persistent kernel's item order and the per-workgroup cross-term
    slots change from call to call; the ranks must not."""
    imgs = _set(5, 4000, big=0.02)
    t = _truth(5, 4000)
    first = _rank(ctx, imgs, t, 1)
    for _ in range(3):
        again = _rank(ctx, imgs, t, 1)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1])


def test_batched_plan_paired_equals_unpaired(ctx):
    """The batched plan ranks every mesh against itself through tile pairs;
    with pairs switched off it must give the same ranks and distances."""
    import torch
    from paper_2007_02306_amd import Context
    rng = np.random.default_rng(21)
    meshes = []
    for k in range(6):
        t = int(round(np.exp(rng.uniform(np.log(300), np.log(9000)))))
        m, _ = synth.configs.random_object(rng, t)
        pos = m.positions.astype(np.float32)
        nrm = synth.vertex_normals(pos, m.triangles)
        meshes.append((pos, m.triangles, nrm, rng.permutation(pos.shape[0]).astype(np.uint32)))
    from gpu_util import dev_f32
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(tr), op_positions=dev_f32(p), op_normals=dev_f32(nr),
                 true_index=dev_u32(ti)) for p, tr, nr, ti in meshes]
    say(f"  batch of {len(jobs)} meshes, vertices {[len(m[0]) for m in meshes]}")
    results = []
    for pairs in (1, 0):
        c = Context(0)
        c.set_tuning("search_pairs", pairs)
        b = c.batch(jobs, 0.3)
        b.run()
        c.sync()
        results.append([(host_u32(b.rank[k]), b.true_distance[k].cpu().numpy(), host_u32(b.images[k]))
                        for k in range(len(jobs))])
        b.close()
        c.close()
    for (pr, pd, pi), (ur, ud, ui) in zip(*results):
        assert np.array_equal(pi, ui)
        assert np.array_equal(pr, ur) and np.array_equal(pd, ud)
    # one mesh against the oracle on the GPU's own images
    img = results[0][2][2]
    o_rk, o_ds = oracle.rank(img, img, meshes[2][3])
    assert np.array_equal(results[0][2][0], o_rk) and np.array_equal(results[0][2][1], o_ds)
    torch.cuda.synchronize()


def test_paired_benchmark_sized_set_sampled(ctx):
    """A set of 23 352 images ranked against itself (92 tiles: 11 full bands
    of 8 tile rows and a partial one; 4 278 tile pairs), with 6 % of the
    images stepping beyond 15 and a few beyond 127, so that shared pairs,
    pairs with a q phase and the exact path all occur.  A sample of 64
    needles is ranked by the oracle over the whole set."""
    n = 23_352
    imgs = _set(99, n, big=0.06, huge=5)
    t = _truth(99, n)
    rk, ds = _rank(ctx, imgs, t, 1)
    rng = np.random.default_rng(100)
    sel = np.unique(np.concatenate([[0, 255, 256, n - 1], rng.choice(n, 60, replace=False)]))
    o_rk, o_ds = oracle.rank(imgs[sel], imgs, t[sel])
    _same(ds[sel], o_ds, "paired true distances (sample)")
    _same(rk[sel], o_rk, "paired ranks (sample)")
    assert int(o_rk.max()) > 0
