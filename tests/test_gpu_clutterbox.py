"""The synthetic clutterbox driver (Sec. 4.1 steps) on the GPU: its images
match the oracle outside flagged pixels, its ranks equal the ranks the oracle
computes from its own images, its Eq. 8 clutter values equal the oracle's, and
clutter only makes the correct match harder to find."""

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
        o_cd, fl_cd, _ = oracle.rici_rowrange(pos, tri, pos, nrm, 0.3)
        assert_images_match(r["cd"], o_cd, fl_cd, f"cluttered set, level {k}")
        # ranks from the oracle's own images; a needle whose image differs
        # from the oracle's (only possible at flagged pixels) is skipped, and
        # each differing haystack image may move a rank by one
        v0 = r["reference_vertices"]
        t = np.arange(v0, dtype=np.uint32)
        ork, _ = oracle.rank(o_rd, o_cd, t)
        n_same = ~(r["rd"] != o_rd).any(axis=(1, 2))
        h_diff = int((r["cd"] != o_cd).any(axis=(1, 2)).sum())
        gap = np.abs(r["ranks"].astype(np.int64) - ork.astype(np.int64))[n_same]
        assert (gap <= h_diff).all(), f"ranks, level {k}"
        if h_diff == 0:
            assert np.array_equal(r["ranks"][n_same], ork[n_same])
        say(f"  level {k}: {int(n_same.sum())}/{v0} needles compared, {h_diff} haystack images differ at flags")
        # Eq. 8 around each reference vertex, from the oracle's areas
        oa, oo = oracle.clutter_areas(pos, tri, 0, ref_tri.shape[0], pos[:v0], nrm[:v0], 0.3)
        assert np.allclose(r["area_all"], oa, rtol=1e-10, atol=1e-12)
        assert np.allclose(r["area_object"], oo, rtol=1e-10, atol=1e-12)
        oc = np.where(oa > 0, (oa - oo) / np.where(oa > 0, oa, 1.0), 0.0)
        assert np.allclose(r["clutter"], oc, rtol=0, atol=1e-9)
        if k == 1:
            assert np.abs(r["clutter"]).max() < 1e-9      # the reference alone: no clutter
    s = summarise([res])
    assert s[1]["rank0_fraction"] >= s[3]["rank0_fraction"] - 1e-9
    assert s[1]["rank0_fraction"] > 0.3
    assert s[3]["clutter_mean"] >= s[1]["clutter_mean"]
    assert sum(n for _, n, _ in s[3]["rank0_fraction_by_clutter"]) == s[3]["searches"]
    ctx.close()
