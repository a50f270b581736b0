"""The synthetic clutterbox driver (Sec. 4.1 steps) on the GPU: its images
match the oracle outside flagged pixels and its ranks equal the oracle's ranks
of the same images; clutter only makes the correct match harder to find."""

import numpy as np
import pytest

import oracle
from gpu_util import assert_images_match, say

pytestmark = pytest.mark.gpu


def test_clutterbox_trial_against_oracle():
    from paper_2007_02306_amd import Context
    from paper_2007_02306_amd.clutterbox import run_trial, summarise
    ctx = Context(0)
    rng = np.random.default_rng(11)
    say("  clutterbox trial: 3 objects of 300-900 triangles, levels 1 and 3")
    res = run_trial(ctx, rng, levels=(1, 3), tri_lo=300, tri_hi=900, keep=True)
    ref_pos, ref_tri, ref_nrm = res[0]["reference"]
    o_rd, fl_rd, _ = oracle.rici_rowrange(ref_pos, ref_tri, ref_pos, ref_nrm, 0.3)
    for k in (1, 3):
        r = res[k]
        assert_images_match(r["rd"], o_rd, fl_rd, "reference set")
        pos, tri, nrm = r["scene"]
        sel = np.unique(np.linspace(0, len(pos) - 1, 40).astype(int))
        o_cd, fl_cd, _ = oracle.rici_rowrange(pos, tri, pos[sel], nrm[sel], 0.3)
        assert_images_match(r["cd"][sel], o_cd, fl_cd, f"cluttered set, level {k}")
        t = np.arange(r["reference_vertices"], dtype=np.uint32)
        ork, _ = oracle.rank(r["rd"], r["cd"], t)
        assert np.array_equal(r["ranks"], ork), f"ranks, level {k}"
    s = summarise([res])
    assert s[1]["rank0_fraction"] >= s[3]["rank0_fraction"] - 1e-9
    assert s[1]["rank0_fraction"] > 0.3
    ctx.close()
