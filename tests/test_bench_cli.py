"""bench.py's contract on the host: more than one GPU is refused with a
message (this build runs on one GPU), and the recorded PMC traffic is only
reported while the kernel sources it was taken with are unchanged."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"] and out["n_gpus"] == 2


def test_traffic_record_needs_unchanged_sources(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    rec = {"workload": "CX", "precision": "c64", "kernel_id": 7, "step": 3, "bytes_per_launch": 123,
           "sources": {"bench.py": "0" * 64}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "x.md").write_text("text\n<!-- traffic " + json.dumps(rec) + " -->\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "bench.py").write_text("changed")
    assert bench.pmc_traffic("CX", "c64", 7, 3) is None
    import hashlib
    rec["sources"] = {"bench.py": hashlib.sha256(b"changed").hexdigest()}
    (prof / "x.md").write_text("<!-- traffic " + json.dumps(rec) + " -->\n")
    assert bench.pmc_traffic("CX", "c64", 7, 3) == 123.0
    assert bench.pmc_traffic("CX", "c64", 8, 3) is None
    assert bench.pmc_traffic("CX", "c64", 7, 4) is None


def test_shipped_tuning_file_is_valid():
    # the tile configurations bench.py loads by default: one entry per step
    # class, each an index into the configuration table of its kernel
    import json
    import re
    from paper_2212_04749_amd import binding as B
    tuned = json.load(open(os.path.join(ROOT, "paper_2212_04749_amd", "tuning_mi355x.json")))
    assert tuned
    for key, cfg in tuned.items():
        m = re.fullmatch(r"(c64|chalf)/(f|h)/(fan/)?(\d+),(\d+),(\d+)/(\d+)", key)
        assert m, key
        bound = B.matnc_mfma_config_count() if m.group(2) == "f" else 9
        assert 0 <= cfg < bound, key
