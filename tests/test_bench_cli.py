"""Host-side behaviour of bench.py: the one-GPU guard and the rule that HBM
traffic is reported only while the counted kernel's source is unchanged."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def _summary(tmp_path, sha):
    p = tmp_path / "counters.md"
    p.write_text("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled read B | "
                 "scaled write B | scaled total B |\n|---|---|---|---|---|---|---|\n"
                 "| mrf::k_example | 1 | 1 | 1 | 2.0e+03 | 1.0e+03 | 3.0e+03 |\n\n"
                 f"- csrc/match.hip: {sha}\n")
    return str(p)


def test_traffic_only_for_the_counted_source(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_1506_05393_amd", "csrc", "match.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    monkeypatch.setattr(bench, "COUNTERS", _summary(tmp_path, sha))
    assert bench.counted_traffic("mrf::k_example", "match.hip") == 3.0e3
    assert bench.counted_traffic("mrf::k_other", "match.hip") is None
    monkeypatch.setattr(bench, "COUNTERS", _summary(tmp_path, "0" * 64))
    assert bench.counted_traffic("mrf::k_example", "match.hip") is None
    monkeypatch.setattr(bench, "COUNTERS", str(tmp_path / "missing.md"))
    assert bench.counted_traffic("mrf::k_example", "match.hip") is None
