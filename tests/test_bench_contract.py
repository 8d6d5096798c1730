"""The benchmark's host-side contract (CPU only): one GPU only, the traffic
record is tied to the MTTKRP source it was measured on, and the CPU baseline
is the oracle timed on a bounded sample."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2003_03572_amd import gen  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_record_follows_the_kernel_source(tmp_path, monkeypatch):
    assert bench.measured_traffic("no-such-workload") is None
    # a record whose source hash does not match the current kernel is ignored
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_2003_03572_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2003_03572_amd" / "csrc" / "mttkrp.hip").write_text("// kernel A\n")
    import hashlib
    sha_a = hashlib.sha256(b"// kernel A\n").hexdigest()
    rec = {"hbm_bytes_per_launch": 123.0, "mttkrp_hip_sha256": sha_a}
    (prof / "k_mttkrp_w_counters.md").write_text("# x\n\n```json\n" + json.dumps(rec) + "\n```\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("w") == 123.0
    (tmp_path / "paper_2003_03572_amd" / "csrc" / "mttkrp.hip").write_text("// kernel B\n")
    assert bench.measured_traffic("w") is None


def test_cpu_baseline_is_the_oracle_on_a_bounded_sample(oracle_mod):
    w = gen.SMALL_UNIFORM
    dims, idx, vals = gen.make(w)
    out = bench.cpu_baseline(w, dims, idx, vals, budget_s=0.01)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "nnz*R/s"
    assert out["value"] > 0 and "iteration" in out["sample"]
