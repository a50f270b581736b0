"""GPU parity of the batched describe-and-rank plan (rici_batch_*): a batch of
meshes of uneven size, replayed as a graph, must give exactly the plain
per-mesh results (which the other GPU tests tie to the oracle), and sampled
images must equal the oracle's outside flagged pixels."""

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


def _meshes(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        t = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        m, _ = synth.configs.random_object(rng, t)
        pos = m.positions.astype(np.float32)
        nrm = synth.vertex_normals(pos, m.triangles)
        ti = rng.permutation(pos.shape[0]).astype(np.uint32)
        out.append((pos, m.triangles, nrm, ti))
    return out


def test_batch_matches_plain_path_and_oracle(ctx):
    import torch
    meshes = _meshes(4, 12, 60, 6000)
    jobs = []
    for k, (pos, tri, nrm, ti) in enumerate(meshes):
        j = dict(positions=dev_f32(pos), triangles=dev_u32(tri), op_positions=dev_f32(pos), op_normals=dev_f32(nrm))
        if k != 3:                      # one describe-only job
            j["true_index"] = dev_u32(ti)
        jobs.append(j)
    say(f"  batch of {len(jobs)} meshes, triangles {[len(m[1]) for m in meshes]}")
    b = ctx.batch(jobs, 0.3)
    # plain path, mesh by mesh
    plain = []
    for k, (pos, tri, nrm, ti) in enumerate(meshes):
        img = ctx.generate(jobs[k]["positions"], jobs[k]["triangles"], jobs[k]["op_positions"],
                           jobs[k]["op_normals"], 0.3)
        rk = ds = None
        if k != 3:
            rk, ds = ctx.distance_rank(img, img, jobs[k]["true_index"])
        ctx.sync()
        plain.append((host_u32(img), None if rk is None else host_u32(rk), None if ds is None else ds.cpu().numpy()))
    for rep in range(3):
        b.run()
        ctx.sync()
        # eager work between replays
        scratch = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for k in range(len(meshes)):
            assert np.array_equal(host_u32(b.images[k]), plain[k][0]), f"replay {rep} mesh {k} images"
            if k != 3:
                assert np.array_equal(host_u32(b.rank[k]), plain[k][1]), f"replay {rep} mesh {k} ranks"
                assert np.array_equal(b.true_distance[k].cpu().numpy(), plain[k][2])
            else:
                assert b.rank[k] is None
        del scratch
    # oracle on a sample of images of three meshes
    for k in (0, 5, 11):
        pos, tri, nrm, ti = meshes[k]
        sel = np.unique(np.linspace(0, len(pos) - 1, 12).astype(int))
        o, fl, _ = oracle.rici_rowrange(pos, tri, pos[sel], nrm[sel], 0.3)
        g = host_u32(b.images[k])[sel]
        assert not ((g != o) & ~fl).any(), f"mesh {k} differs from the oracle"
    assert max(int(host_u32(r).max()) for r in b.rank if r is not None) > 0
    b.close()


def test_batch_small_search_tile(ctx):
    """A plan recorded under the 128-needle search tile and 4-image generation
    workgroups gives the plain path's exact results."""
    from paper_2007_02306_amd import Context
    meshes = _meshes(8, 4, 100, 3000)
    c128 = Context(0)
    c128.set_tuning("search_tile_m", 128)
    c128.set_tuning("gen_images_per_group", 4)
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(t), op_positions=dev_f32(p), op_normals=dev_f32(n),
                 true_index=dev_u32(ti)) for p, t, n, ti in meshes]
    b = c128.batch(jobs, 0.3)
    b.run()
    c128.sync()
    for k, j in enumerate(jobs):
        img = ctx.generate(j["positions"], j["triangles"], j["op_positions"], j["op_normals"], 0.3)
        rk, ds = ctx.distance_rank(img, img, j["true_index"])
        ctx.sync()
        assert np.array_equal(host_u32(b.images[k]), host_u32(img))
        assert np.array_equal(host_u32(b.rank[k]), host_u32(rk))
        assert np.array_equal(b.true_distance[k].cpu().numpy(), ds.cpu().numpy())
    b.close()
    c128.close()


def test_batch_sorted_triangles(ctx):
    """A plan whose meshes store their triangles in Morton order gives the
    plain path's images (mesh order) bit for bit, ragged sort blocks included."""
    from paper_2007_02306_amd import Context
    meshes = _meshes(10, 5, 3000, 12000)
    cs = Context(0)
    cs.set_tuning("gen_sort_triangles", 1)
    c0 = Context(0)
    c0.set_tuning("gen_sort_triangles", 0)
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(t), op_positions=dev_f32(p), op_normals=dev_f32(n),
                 true_index=dev_u32(ti)) for p, t, n, ti in meshes]
    b = cs.batch(jobs, 0.3)
    b.run()
    cs.sync()
    for k, j in enumerate(jobs):
        img = c0.generate(j["positions"], j["triangles"], j["op_positions"], j["op_normals"], 0.3)
        rk, ds = c0.distance_rank(img, img, j["true_index"])
        c0.sync()
        assert np.array_equal(host_u32(b.images[k]), host_u32(img)), f"mesh {k}"
        assert np.array_equal(host_u32(b.rank[k]), host_u32(rk))
    b.close()
    cs.close()
    c0.close()


def test_batch_with_early_exit(ctx):
    """A plan recorded with the search's early exit gives the plain path's
    exact ranks (shuffled true matches: non-trivial thresholds)."""
    from paper_2007_02306_amd import Context
    meshes = _meshes(9, 5, 200, 4000)
    ce = Context(0)
    ce.set_tuning("search_early_exit", 1)
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(t), op_positions=dev_f32(p), op_normals=dev_f32(n),
                 true_index=dev_u32(ti)) for p, t, n, ti in meshes]
    b = ce.batch(jobs, 0.3)
    for _ in range(2):
        b.run()
        ce.sync()
        for k, j in enumerate(jobs):
            img = ctx.generate(j["positions"], j["triangles"], j["op_positions"], j["op_normals"], 0.3)
            rk, ds = ctx.distance_rank(img, img, j["true_index"])
            ctx.sync()
            assert np.array_equal(host_u32(b.rank[k]), host_u32(rk)), f"mesh {k}"
            assert np.array_equal(b.true_distance[k].cpu().numpy(), ds.cpu().numpy())
    b.close()
    ce.close()


def _stacked_mesh(seed, copies):
    """A small object with one of its triangles repeated `copies` times: the
    images near that triangle step by more than 127 between neighbouring
    radii, so their pairs take the exact int64 fallback."""
    rng = np.random.default_rng(seed)
    m, _ = synth.configs.random_object(rng, 200)
    pos = m.positions.astype(np.float32)
    tri = np.concatenate([m.triangles, np.repeat(m.triangles[:1], copies, axis=0)])
    nrm = synth.vertex_normals(pos, tri)
    ti = rng.permutation(pos.shape[0]).astype(np.uint32)
    return pos, tri, nrm, ti


def test_batch_out_of_range_deltas(ctx):
    """Meshes whose images have |D| > 127: the batched plan's exact fallback
    (its per-job lists of out-of-range images) gives the plain path's ranks
    and distances, and the plain path's ranks equal the oracle's."""
    meshes = [_stacked_mesh(21, 160), _meshes(22, 1, 300, 2000)[0], _stacked_mesh(23, 140)]
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(t), op_positions=dev_f32(p), op_normals=dev_f32(n),
                 true_index=dev_u32(ti)) for p, t, n, ti in meshes]
    b = ctx.batch(jobs, 0.3)
    slow_seen = 0
    for rep in range(2):
        b.run()
        ctx.sync()
        for k, (j, (pos, tri, nrm, ti)) in enumerate(zip(jobs, meshes)):
            img = ctx.generate(j["positions"], j["triangles"], j["op_positions"], j["op_normals"], 0.3)
            rk, ds = ctx.distance_rank(img, img, j["true_index"])
            ctx.sync()
            h = host_u32(img)
            assert np.array_equal(host_u32(b.images[k]), h), f"mesh {k} images"
            assert np.array_equal(host_u32(b.rank[k]), host_u32(rk)), f"replay {rep} mesh {k} ranks"
            assert np.array_equal(b.true_distance[k].cpu().numpy(), ds.cpu().numpy())
            if rep == 0:
                d = np.diff(h.astype(np.int64), axis=2)
                slow_seen += int((np.abs(d).max(axis=(1, 2)) > 127).sum())
                ork, ods = oracle.rank(h, h, ti)
                assert np.array_equal(host_u32(rk), ork) and np.array_equal(ds.cpu().numpy(), ods), f"mesh {k}"
    say(f"  images with |D| > 127: {slow_seen}")
    assert slow_seen > 0
    b.close()


def test_batch_empty_and_bad_jobs(ctx):
    import torch
    from paper_2007_02306_amd import RiciError
    b = ctx.batch([], 0.3)
    b.run()
    ctx.sync()
    b.close()
    z = torch.zeros((0, 3), device="cuda")
    b = ctx.batch([dict(positions=z, triangles=torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
                        op_positions=z, op_normals=z)], 0.3)
    b.run()
    ctx.sync()
    b.close()
    with pytest.raises(RiciError):
        ctx.batch([], -1.0)


def test_batch_kernel_times_from_graph_events(ctx):
    """The event records inside the plan's graph bracket the two persistent
    kernels: both durations are positive and together below the replay's wall
    time."""
    import time
    import torch
    meshes = _meshes(9, 6, 2000, 20000)
    jobs = [dict(positions=dev_f32(p), triangles=dev_u32(t), op_positions=dev_f32(p), op_normals=dev_f32(n),
                 true_index=dev_u32(ti)) for p, t, n, ti in meshes]
    b = ctx.batch(jobs, 0.3)
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run()
    g = b.kernel_ms("gen")
    s = b.kernel_ms("search")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    say(f"  gen {g:.3f} ms, search {s:.3f} ms, replay {wall:.3f} ms")
    assert g > 0 and s > 0 and g + s < wall
    b.close()
