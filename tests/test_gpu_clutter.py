"""GPU parity of the Eq. 8 clutter areas (rici_clutter_areas) against the
FP64 oracle (reading C1: the support cylinder alpha <= R, |beta| <= R/2).

Both sides integrate each triangle's area in the volume exactly in FP64, in
different orders and forms, so they agree to FP64 rounding: the bound is
1e-10 (R^2 + A) per oriented point, far below any area that matters and far
above FP64 rounding of sums of a few thousand terms."""

import numpy as np
import pytest

import oracle
import synth
from gpu_util import dev_f32, dev_u32, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context
    c = Context(0)
    yield c
    c.close()


def _check(ctx, pos, tri, first, count, opp, opn, R, what):
    a, o = ctx.clutter_areas(dev_f32(pos), dev_u32(tri), first, count, dev_f32(opp), dev_f32(opn), R)
    ctx.sync()
    ga, go = a.cpu().numpy(), o.cpu().numpy()
    oa, oo = oracle.clutter_areas(pos, tri, first, count, opp, opn, R)
    tol_a = 1e-10 * (R * R + np.abs(oa))
    tol_o = 1e-10 * (R * R + np.abs(oo))
    assert (np.abs(ga - oa) <= tol_a).all(), (what, np.abs(ga - oa).max())
    assert (np.abs(go - oo) <= tol_o).all(), (what, np.abs(go - oo).max())
    say(f"  {what}: {len(opp)} points, max |dA| {np.abs(ga - oa).max():.2e}, mean A_all {oa.mean():.4f}")
    return ga, go


def test_closed_form_patches(ctx):
    R = 0.3
    sq = lambda z, h: (np.array([[-h, -h, z], [h, -h, z], [h, h, z], [-h, h, z]], np.float32),
                       np.array([[0, 1, 2], [0, 2, 3]], np.uint32))
    v0, t0 = sq(0.0, 0.05)
    v1, t1 = sq(0.05, 0.1)
    v2, t2 = sq(0.0, 1.0)          # a large plane: holds the disc pi R^2
    pos = np.concatenate([v0, v1, v2])
    tri = np.concatenate([t0, t1 + 4, t2 + 8])
    ga, go = _check(ctx, pos, tri, 0, 2, np.zeros((1, 3)), np.array([[0.0, 0, 1]]), R, "patches")
    assert ga[0] == pytest.approx(0.01 + 0.04 + np.pi * R * R, rel=1e-6)
    assert go[0] == pytest.approx(0.01, rel=1e-6)


def test_clutter_scene_reference_vertices(ctx):
    rng = np.random.default_rng(21)
    mesh, canon, offsets, _ = synth.configs.clutter_scene(rng, 4, 2000, 6000)
    pos = mesh.positions.astype(np.float32)
    tri = mesh.triangles.astype(np.uint32)
    nrm = synth.vertex_normals(pos, tri)
    v0 = canon[0].num_vertices
    t0 = canon[0].triangles.shape[0]
    sel = np.unique(np.linspace(0, v0 - 1, 300).astype(int))
    ga, go = _check(ctx, pos, tri, 0, t0, pos[sel], nrm[sel], 0.3, "clutter scene")
    clutter = (ga - go) / ga
    assert (ga > 0).all() and (clutter >= -1e-12).all() and (clutter <= 1).all()


@pytest.mark.parametrize("R", [0.05, 1.0, 3.0])
def test_radii_and_odd_sizes(ctx, R):
    s = synth.config1_icosphere()
    idx = np.arange(0, s.num_haystack, 7)
    _check(ctx, s.positions, s.triangles, 10, 50, s.op_positions[idx], s.op_normals[idx], R, f"icosphere R={R}")


def test_empty_scene_and_bad_index(ctx):
    import torch
    from paper_2007_02306_amd import RiciError
    opp = np.zeros((3, 3), np.float32)
    opn = np.array([[0, 0, 1.0]] * 3, np.float32)
    a, o = ctx.clutter_areas(torch.zeros((0, 3), dtype=torch.float32, device="cuda"),
                             torch.zeros((0, 3), dtype=torch.int32, device="cuda"), 0, 0, dev_f32(opp), dev_f32(opn), 0.3)
    ctx.sync()
    assert float(a.abs().sum()) == 0.0 and float(o.abs().sum()) == 0.0
    pos = np.zeros((3, 3), np.float32)
    tri = np.array([[0, 1, 5]], np.uint32)
    ctx.clutter_areas(dev_f32(pos), dev_u32(tri), 0, 1, dev_f32(opp), dev_f32(opn), 0.3)
    with pytest.raises(RiciError):
        ctx.sync()
