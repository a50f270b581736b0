"""GPU tests of the device-resident database, incremental queries and the
continuous-batching server (rici_db_*, rici_query_*, rici_db_scan, serve.py).

The database holds oracle images (so no expected value comes from the GPU);
requests describe canonical objects on the GPU and are ranked against it.
Ranks must equal the oracle's, and be the same for a request served alone and
in a mix with other requests in flight."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_u32, host_u32, say

from paper_2007_02306_amd import NOALLOC_WORKSPACE_BYTES  # noqa: E402

pytestmark = pytest.mark.gpu

R = 0.3


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.serve import DescriptorDB
    rng = np.random.default_rng(55)
    db_imgs, objects, base = [], [], 0
    for _ in range(2):
        mesh, canon, offsets, _ = synth.configs.clutter_scene(rng, 3, 400, 1500)
        pos = mesh.positions.astype(np.float32)
        nrm = synth.vertex_normals(pos, mesh.triangles)
        im, _, _ = oracle.rici_rowrange(pos, mesh.triangles, pos, nrm, R)
        db_imgs.append(im)
        for o, m in enumerate(canon):
            objects.append((m, base + offsets[o]))
        base += pos.shape[0]
    db_host = np.concatenate(db_imgs)
    say(f"  database of {len(db_host)} oracle images, {len(objects)} objects")
    ctx = Context(0)
    db = DescriptorDB(ctx, dev_u32(db_host))
    yield ctx, db, db_host, objects
    db.close()
    ctx.close()


def _request(rid, objects, rng, q=160):
    from paper_2007_02306_amd.serve import Request
    m, off = objects[rid % len(objects)]
    pos = m.positions.astype(np.float32)
    nrm = synth.vertex_normals(pos, m.triangles)
    ids = np.sort(rng.choice(pos.shape[0], min(q, pos.shape[0]), replace=False))
    return Request(rid, pos, m.triangles, nrm, ids, (off + ids).astype(np.uint32), support_radius=R)


def _oracle_ranks(req, db_host):
    im, fl, _ = oracle.rici_rowrange(req.positions, req.triangles, req.positions[req.needle_ids],
                                     req.normals[req.needle_ids], R)
    rk, ds = oracle.rank(im, db_host, req.true_index)
    return im, fl, rk, ds


def test_query_scan_in_slices_matches_oracle(setup):
    import torch
    ctx, db, db_host, objects = setup
    rng = np.random.default_rng(1)
    req = _request(0, objects, rng)
    im_o, fl, rk_o, ds_o = _oracle_ranks(req, db_host)
    assert not fl.any()
    needles = dev_u32(im_o)
    ti = dev_u32(req.true_index)
    rank = torch.empty(len(im_o), dtype=torch.int32, device="cuda")
    dist = torch.empty(len(im_o), dtype=torch.int64, device="cuda")
    import ctypes
    from paper_2007_02306_amd import _ptr, check
    h = ctypes.c_void_p()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(ctx._lib.rici_query_create(ctx._h, db._h, _ptr(needles), len(im_o), _ptr(ti), _ptr(rank), _ptr(dist),
                                     None, 0, s, ctypes.byref(h)))
    # scan the tiles in three uneven slices, starting in the middle (wrap-around)
    T = db.tiles
    cuts = [T // 2, T // 2 + max(1, T // 5), T // 2 + T]
    arr = (ctypes.c_void_p * 1)(h.value)
    check(ctx._lib.rici_db_scan(ctx._h, db._h, arr, 1, cuts[0] % T, cuts[1] - cuts[0], s))
    check(ctx._lib.rici_db_scan(ctx._h, db._h, arr, 1, cuts[1] % T, cuts[2] - cuts[1], s))
    ctx.sync()
    assert np.array_equal(dist.cpu().numpy(), ds_o)
    assert np.array_equal(host_u32(rank), rk_o)
    assert rk_o.max() > 0
    ctx._lib.rici_query_destroy(h)


def test_server_alone_and_in_mix(setup):
    from paper_2007_02306_amd.serve import Server
    ctx, db, db_host, objects = setup
    alone = {}
    for rid in range(4):
        srv = Server(db, max_active=1, slices=5, keep_images=True)
        srv.submit(_request(rid, objects, np.random.default_rng(100 + rid)))
        srv.drain()
        (req,) = srv.done
        alone[rid] = req
        im_o, fl, rk_o, ds_o = _oracle_ranks(req, db_host)
        assert not ((req.images != im_o) & ~fl).any(), f"request {rid} images"
        if not fl.any():
            assert np.array_equal(req.rank, rk_o), f"request {rid} ranks"
            assert np.array_equal(req.true_distance, ds_o)
        srv.close()
    srv = Server(db, max_active=3, slices=5)
    for rid in range(4):
        srv.submit(_request(rid, objects, np.random.default_rng(100 + rid)))
    srv.drain()
    assert len(srv.done) == 4 and srv.used == NOALLOC_WORKSPACE_BYTES   # only the describe workspace left
    for req in srv.done:
        assert np.array_equal(req.rank, alone[req.rid].rank), f"request {req.rid} differs in the mix"
        assert np.array_equal(req.true_distance, alone[req.rid].true_distance)
    assert srv.steps < 4 * 5      # requests shared scan steps
    srv.close()


def test_server_admission_by_footprint(setup):
    from paper_2007_02306_amd.serve import Server
    ctx, db, db_host, objects = setup
    reqs = [_request(rid, objects, np.random.default_rng(7 + rid)) for rid in range(3)]
    probe = Server(db, slices=3)
    need = max(probe.footprint(r) for r in reqs)
    probe.close()
    # room for the describe workspace and one request at a time
    srv = Server(db, budget_bytes=NOALLOC_WORKSPACE_BYTES + need + need // 2, max_active=8, slices=3)
    for r in reqs:
        srv.submit(r)
    peak = 0
    while srv.poll():
        peak = max(peak, len(srv.describing) + len(srv.scanning) + len(srv.finishing))
        assert srv.used <= srv.budget
    assert peak == 1 and len(srv.done) == 3
    with pytest.raises(ValueError):
        Server(db, budget_bytes=1024)               # not even the describe workspace fits
    small = Server(db, budget_bytes=NOALLOC_WORKSPACE_BYTES + 1024)
    with pytest.raises(ValueError):
        small.submit(reqs[0])
    small.close()
    srv.close()


def test_scan_with_small_tile_and_mixed_tiles_rejected(setup):
    """A query created under the 128-needle search tile scans to the oracle's
    ranks; queries of different tile shapes are not scanned together."""
    import ctypes
    import torch
    from paper_2007_02306_amd import Context, RiciError, _ptr, check
    ctx, db, db_host, objects = setup
    rng = np.random.default_rng(2)
    req = _request(1, objects, rng, q=150)
    im_o, fl, rk_o, ds_o = _oracle_ranks(req, db_host)
    c128 = Context(0)
    c128.set_tuning("search_tile_m", 128)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    needles, ti = dev_u32(im_o), dev_u32(req.true_index)
    outs, hs = [], []
    for c in (c128, ctx):
        rank = torch.empty(len(im_o), dtype=torch.int32, device="cuda")
        dist = torch.empty(len(im_o), dtype=torch.int64, device="cuda")
        h = ctypes.c_void_p()
        check(c._lib.rici_query_create(c._h, db._h, _ptr(needles), len(im_o), _ptr(ti), _ptr(rank), _ptr(dist),
                                       None, 0, s, ctypes.byref(h)))
        outs.append((rank, dist))
        hs.append(h)
    both = (ctypes.c_void_p * 2)(hs[0].value, hs[1].value)
    with pytest.raises(RiciError):
        check(ctx._lib.rici_db_scan(ctx._h, db._h, both, 2, 0, db.tiles, s))
    one = (ctypes.c_void_p * 1)(hs[0].value)
    check(ctx._lib.rici_db_scan(ctx._h, db._h, one, 1, 0, db.tiles, s))
    ctx.sync()
    rank, dist = outs[0]
    assert np.array_equal(dist.cpu().numpy(), ds_o)
    assert np.array_equal(host_u32(rank), rk_o)
    for h in hs:
        ctx._lib.rici_query_destroy(h)
    c128.close()


def test_scan_with_early_exit_matches_oracle(setup):
    """A query made under the early-exit knob scans (in two slices) to the
    oracle's ranks."""
    import ctypes
    import torch
    from paper_2007_02306_amd import Context, _ptr, check
    ctx, db, db_host, objects = setup
    rng = np.random.default_rng(3)
    req = _request(2, objects, rng, q=200)
    im_o, fl, rk_o, ds_o = _oracle_ranks(req, db_host)
    c = Context(0)
    c.set_tuning("search_early_exit", 1)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    needles, ti = dev_u32(im_o), dev_u32(req.true_index)
    rank = torch.empty(len(im_o), dtype=torch.int32, device="cuda")
    dist = torch.empty(len(im_o), dtype=torch.int64, device="cuda")
    h = ctypes.c_void_p()
    check(c._lib.rici_query_create(c._h, db._h, _ptr(needles), len(im_o), _ptr(ti), _ptr(rank), _ptr(dist),
                                   None, 0, s, ctypes.byref(h)))
    one = (ctypes.c_void_p * 1)(h.value)
    half = db.tiles // 2
    check(c._lib.rici_db_scan(c._h, db._h, one, 1, 0, half, s))
    check(c._lib.rici_db_scan(c._h, db._h, one, 1, half, db.tiles - half, s))
    c.sync()
    assert np.array_equal(dist.cpu().numpy(), ds_o)
    assert np.array_equal(host_u32(rank), rk_o)
    c._lib.rici_query_destroy(h)
    c.close()
