"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small C harness (`oracle_asan_harness.c`) is compiled together with the
oracle's source with both sanitizers and run on degenerate and boundary
scenes: every flag rule fires, output buffers are allocated at exactly their
size, and several images share one run, so a flag or count written outside
its own image, or past the caller's buffer, aborts the run.  The harness's
outputs must also equal those of the ordinary build.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import closed_forms
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NB = 64


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    out = tmp_path_factory.mktemp("asan") / "oracle_asan"
    cmd = ["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
           "-O1", "-ffp-contract=off", "-std=c11", "-D_GNU_SOURCE",
           os.path.join(HERE, "oracle_asan_harness.c"), os.path.join(ROOT, "oracle", "rici_oracle.c"),
           "-lm", "-pthread", "-o", str(out)]
    subprocess.run(cmd, check=True)
    return str(out)


def _run(harness, tmp_path, pos, tri, op, nrm, R):
    pos = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, np.uint32).reshape(-1, 3)
    op = np.ascontiguousarray(op, np.float32).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, np.float32).reshape(-1, 3)
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as f:
        np.array([pos.shape[0], tri.shape[0], op.shape[0]], np.int64).tofile(f)
        np.array([R], np.float64).tofile(f)
        for a in (pos, tri, op, nrm):
            a.tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([harness, str(src), str(dst)], capture_output=True, text=True, env=env, timeout=600)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stderr[-4000:]
    n = op.shape[0]
    px = n * NB * NB
    raw = np.fromfile(dst, np.uint8)
    o = 0
    img = raw[o:o + 4 * px].view(np.uint32).reshape(n, NB, NB); o += 4 * px
    fl = raw[o:o + px].reshape(n, NB, NB).astype(bool); o += px
    brute = raw[o:o + 4 * px].view(np.uint32).reshape(n, NB, NB); o += 4 * px
    rank = raw[o:o + 4 * n].view(np.uint32); o += 4 * n
    mat = raw[o:o + 8 * n * n].view(np.int64).reshape(n, n)
    return img, fl, brute, rank, mat


def _check_against_plain_build(pos, tri, op, nrm, R, img, fl, brute, rank, mat):
    im2, fl2, _ = oracle.rici_rowrange(pos, tri, op, nrm, R)
    ib2, _ = oracle.rici_brute(pos, tri, op, nrm, R)
    assert np.array_equal(img, im2) and np.array_equal(fl, fl2) and np.array_equal(brute, ib2)
    n = op.shape[0]
    rk, _ = oracle.rank(img, img, (np.arange(n) * 7 + 3) % n)
    assert np.array_equal(rank, rk)
    assert np.array_equal(mat, oracle.distance_matrix(img, img))


def test_degenerate_scene_is_clean_under_sanitizers(harness, tmp_path):
    """The degenerate triangles (a triangle in row plane 40, an edge in row
    plane 20, a vertex on row plane 30, an edge on the axis, ...) seen from
    several oriented points, the last of which is the canonical one: rule
    (iii)/(iv) flags at rows 20 and 40 of the last image must stay inside it."""
    v, t = closed_forms.degenerate_triangles()
    op = np.array([[0.01, 0.02, 0.0], [0, 0, 0.25], [0, 0, 0]], np.float32)
    nrm = np.array([[0.1, 0.2, 1.0], [0, 0, 1], [0, 0, 1]], np.float32)
    out = _run(harness, tmp_path, v, t, op, nrm, 1.0)
    img, fl = out[0], out[1]
    assert fl[2, 40].any() and fl[2, 20].any()
    _check_against_plain_build(v, t, op, nrm, 1.0, *out)


def test_boundary_scenes_are_clean_under_sanitizers(harness, tmp_path):
    v1, t1, _ = closed_forms.bin_radius_boundaries()
    v2, t2, _ = closed_forms.row_plane_boundaries()
    v = np.concatenate([v1, v2])
    t = np.concatenate([t1, t2 + len(v1)]).astype(np.uint32)
    op = np.array([[0, 0, 0], [0.05, -0.02, 0.01]], np.float32)
    nrm = np.array([[0, 0, 1], [0.3, 0.1, 0.9]], np.float32)
    out = _run(harness, tmp_path, v, t, op, nrm, 1.0)
    _check_against_plain_build(v, t, op, nrm, 1.0, *out)


def test_snapped_random_scene_is_clean_under_sanitizers(harness, tmp_path):
    """Random triangles whose vertices sit exactly on row planes and bin radii
    of the canonical oriented point (every flag rule fires somewhere), a zero
    normal, and a degenerate point triangle."""
    rng = np.random.default_rng(7)
    b = 1.0 / NB
    nt = 40
    rows = rng.integers(0, NB, size=(nt, 3))
    cols = rng.integers(0, NB, size=(nt, 3))
    ang = rng.uniform(0, 2 * np.pi, size=(nt, 3))
    z = -0.5 + (rows + 0.5) * b
    z[::3, 1] = z[::3, 0]                                   # edges in row planes
    z[::5, :] = z[::5, :1]                                  # triangles in row planes
    r = (cols + 0.5) * b
    pos = np.stack([r * np.cos(ang), r * np.sin(ang), z], axis=-1).reshape(-1, 3).astype(np.float32)
    tri = np.arange(3 * nt, dtype=np.uint32).reshape(nt, 3)
    tri[0] = [0, 0, 0]
    op = np.array([[0, 0, 0], [0, 0, 0], [0.01, 0.0, -0.02], [0, 0, 0]], np.float32)
    nrm = np.array([[0, 0, 1], [0, 0, 0], [0.2, -0.1, 1.0], [0, 0, 1]], np.float32)
    out = _run(harness, tmp_path, pos, tri, op, nrm, 1.0)
    img, fl = out[0], out[1]
    assert fl[1].all() and fl[0].any() and fl[3].any()
    _check_against_plain_build(pos, tri, op, nrm, 1.0, *out)
