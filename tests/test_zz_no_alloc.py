"""rici_generate_noalloc (generation with the library's static workspace)
against rici_generate, both called through the C ABI: identical images on
consecutive calls whose meshes shrink, so that a call reads only the records it
wrote itself, plus the size limit refused before anything is enqueued."""

import ctypes

import numpy as np
import pytest

import synth
from gpu_util import dev_f32, dev_u32, host_u32, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_2007_02306_amd import Context, _lib
    c = Context(0)
    yield c, _lib.load()
    c.close()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(lib, fn_name, ctx, pos, tri, opp, opn, R, out):
    import torch
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn = getattr(lib, fn_name)
    rc = fn(ctx._h, _p(pos), pos.shape[0], _p(tri), tri.shape[0], _p(opp), _p(opn), opp.shape[0],
            ctypes.c_float(R), _p(out), stream)
    assert rc == 0, (fn_name, rc, lib.rici_last_error())


def _scene(kind: str, rng):
    """(positions, triangles, op_positions, op_normals, R) on the device."""
    if kind == "large":
        # one superquadric above the Morton-sorting size (145 200 triangles)
        m = synth.meshes.superquadric(110, 0.7, 1.9, scales=(1.0, 0.8, 0.6))
        pos, tri = m.positions, m.triangles
        nrm = synth.meshes.vertex_normals(pos, tri)
        sel = np.sort(rng.choice(len(pos), 1536, replace=False))
        return pos, tri, pos[sel], nrm[sel], 0.3
    if kind == "union12":
        s = synth.config2_union12()
        sel = np.sort(rng.choice(s.num_haystack, 777, replace=False))
        return s.positions, s.triangles, s.op_positions[sel], s.op_normals[sel], s.support_radius
    s = synth.config1_icosphere()
    return s.positions, s.triangles, s.op_positions[:61], s.op_normals[:61], s.support_radius


def test_noalloc_equals_generate_on_shrinking_calls(env):
    import torch
    ctx, lib = env
    rng = np.random.default_rng(77)
    for kind in ["large", "union12", "icosphere"]:
        pos, tri, opp, opn, R = _scene(kind, rng)
        say(f"  noalloc vs generate: {kind} T={len(tri)} N={len(opp)}")
        args = [dev_f32(pos), dev_u32(tri), dev_f32(opp), dev_f32(opn)]
        ref = torch.full((len(opp), 64, 64), -1, dtype=torch.int32, device="cuda")
        got = torch.full((len(opp), 64, 64), -1, dtype=torch.int32, device="cuda")
        _call(lib, "rici_generate", ctx, *args, R, ref)
        _call(lib, "rici_generate_noalloc", ctx, *args, R, got)
        ctx.sync()
        a, b = host_u32(ref), host_u32(got)
        assert a.max() > 0 and a.max() != 0xFFFFFFFF
        assert np.array_equal(a, b), f"{kind}: {int((a != b).sum())} pixels differ"


def test_noalloc_refuses_meshes_beyond_its_workspace(env):
    from paper_2007_02306_amd import _lib
    ctx, lib = env
    limit = 1 << 20
    s = synth.config1_icosphere()
    pos, tri = dev_f32(s.positions), dev_u32(s.triangles)
    opp, opn = dev_f32(s.op_positions[:4]), dev_f32(s.op_normals[:4])
    import torch
    out = torch.zeros((4, 64, 64), dtype=torch.int32, device="cuda")
    # the count is checked before any pointer is used, so nothing is read past the small buffers
    rc = lib.rici_generate_noalloc(ctx._h, _p(pos), pos.shape[0], _p(tri), limit + 1, _p(opp), _p(opn), 4,
                                   ctypes.c_float(0.5), _p(out), None)
    assert rc == -5
    assert b"static workspace" in lib.rici_last_error()
    assert _lib.STATUS[rc] == "RICI_ERR_UNSUPPORTED"
    ctx.sync()
    assert int(out.abs().sum()) == 0
