"""Host-side contract of bench.py (no GPU): the one-GPU refusal, the profile
records it reports only while the kernel sources still match them, and the
value-distribution classes."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus_requested"] == 2


def test_stale_profile_records_are_not_reported(tmp_path, monkeypatch):
    """bench.py reports a kernel's HBM traffic only while the kernel sources
    hash to the digest recorded with it."""
    rec = {"source_sha256": "0" * 64, "hbm_bytes_per_dispatch": 123.0, "busy": {"valu_busy": 0.5}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k_gen_union12_hbm_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda k: "0" * 64)
    assert bench.measured_traffic("k_gen") == 123.0
    monkeypatch.setattr(bench, "source_digest", lambda k: "1" * 64)
    assert bench.measured_traffic("k_gen") is None


def test_value_distributions_classes():
    import torch
    im = torch.zeros((3, 64, 64), dtype=torch.int32)
    im[1, 5, 10:] = 15          # one delta of 15: two-phase class
    im[2, 7, 20:] = 16          # one delta of 16: three-phase class
    d = bench.value_distributions(im)
    assert d["max_abs_delta_share"] == {"le_15": 2 / 3, "16_to_127": 1 / 3, "gt_127": 0.0}
    assert d["max_count"] == 16
