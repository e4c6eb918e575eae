"""Host logic of bench.py, on the CPU: the refusal of more than one GPU, and
the HBM traffic figures that the bench line takes from committed counter
summaries only while the kernel source they were measured on is unchanged."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_committed_traffic_summaries_match_their_sources():
    assert bench.measured_traffic("k_interp_tile") > 0
    assert bench.measured_traffic("k_sg_mid", "film_c5_surrogate_hbm_traffic.json",
                                  "surrogate.hip") > 0
    assert bench.measured_traffic("no_such_kernel") is None


def test_traffic_is_dropped_once_the_source_changes(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2409_13958_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = csrc / "k.hip"
    src.write_bytes(b"__global__ void k() {}\n")
    rec = {"k_hip_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "bytes_per_launch": {"k<4>": 1234.0}}
    (tmp_path / "profiles" / "t.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k", "t.json", "k.hip") == 1234.0
    src.write_bytes(b"__global__ void k() { }\n")
    assert bench.measured_traffic("k", "t.json", "k.hip") is None
    shutil.rmtree(csrc)
    assert bench.measured_traffic("k", "t.json", "k.hip") is None
