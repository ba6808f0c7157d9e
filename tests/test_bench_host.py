"""Host logic of bench.py that needs no GPU: the one-GPU guard, and the rule that the
measured HBM traffic of a kernel is taken from the committed counter summary only while the
kernel sources hash to the ones the counters were taken on."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


def _tree(tmp_path, src_text, recorded_sha):
    csrc = tmp_path / "paper_1807_02752_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "ld.hip").write_text(src_text)
    (csrc / "ld_device.h").write_text("// device helpers\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"source_sha256": recorded_sha, "bytes_per_launch": {"k_vdisp_hist": 2125967047}}
    (prof / "lane_path_1242x375_hbm_bytes.md").write_text("# summary\n\ntraffic_json: " + json.dumps(rec) + "\n")


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    src = "// kernels\n"
    h = hashlib.sha256()
    h.update(src.encode())
    h.update(b"// device helpers\n")
    _tree(tmp_path, src, h.hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_vdisp_hist") == 2125967047
    assert bench.measured_traffic("k_energy") is None
    (tmp_path / "paper_1807_02752_amd" / "csrc" / "ld.hip").write_text(src + "// changed\n")
    assert bench.measured_traffic("k_vdisp_hist") is None


def test_no_summary_no_traffic(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_vdisp_hist") is None
