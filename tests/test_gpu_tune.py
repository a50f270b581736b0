"""The autotuner on the GPU: tuned calls give exactly the untuned results, the
choices are valid knob values, and they are cached per shape class."""

import json

import numpy as np
import pytest

import synth
from gpu_util import dev_f32, dev_u32, host_u32, say

pytestmark = pytest.mark.gpu


def test_tuned_calls_match_default_calls(tmp_path):
    import torch
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.tune import GEN_CHOICES, SEARCH_CHOICES, SORT_CHOICES, Tuner
    ctx, ref = Context(0), Context(0)
    s = synth.config1_icosphere()
    pos, tri = dev_f32(s.positions), dev_u32(s.triangles)
    opp, opn = dev_f32(s.op_positions), dev_f32(s.op_normals)
    path = tmp_path / "tune.json"
    t = Tuner(ctx, str(path), reps=2)
    say("  tuning generation and search on the icosphere")
    img = t.generate(pos, tri, opp, opn, s.support_radius)
    img_ref = ref.generate(pos, tri, opp, opn, s.support_radius)
    ti = dev_u32(np.random.default_rng(3).permutation(s.num_haystack).astype(np.uint32))
    rk, ds = t.distance_rank(img, img, ti)
    rk_ref, ds_ref = ref.distance_rank(img_ref, img_ref, ti)
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(img), host_u32(img_ref))
    assert np.array_equal(host_u32(rk), host_u32(rk_ref)) and torch.equal(ds, ds_ref)
    data = json.loads(path.read_text())[t.arch]
    gen_keys = [k for k in data if k.startswith("gen|")]
    search_keys = [k for k in data if k.startswith("search|")]
    assert len(gen_keys) == 1
    g, o = data[gen_keys[0]]
    assert g in GEN_CHOICES and o in SORT_CHOICES
    assert len(search_keys) == 1 and data[search_keys[0]] in SEARCH_CHOICES
    n_meas = len(t.measurements)
    t.generate(pos, tri, opp, opn, s.support_radius)       # cached: no new measurement
    assert len(t.measurements) == n_meas
    ctx.close()
    ref.close()
