"""Host checks of bench.py's contract: more than one GPU is refused with a message, and a stored
counter record is reported only for the kernel sources, workload, configuration and work
decomposition it was taken on."""

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
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_record_lookup(tmp_path):
    rec = tmp_path / "rec.json"
    entry = {"config": "cfgA", "work_items": 100, "hbm_bytes_per_launch": 12345}
    rec.write_text(json.dumps({"workload": "wl", "source_sha256": bench.kernel_source_digest(), "entries": [entry]}))
    assert bench.measured_traffic("wl", "cfgA", 100, str(rec)) == 12345
    assert bench.measured_traffic("wl", "cfgA", 101, str(rec)) is None    # another work decomposition
    assert bench.measured_traffic("wl", "cfgB", 100, str(rec)) is None    # another configuration
    assert bench.measured_traffic("other", "cfgA", 100, str(rec)) is None  # another workload
    rec.write_text(json.dumps({"workload": "wl", "source_sha256": "0" * 64, "entries": [entry]}))
    assert bench.measured_traffic("wl", "cfgA", 100, str(rec)) is None    # other kernel sources
    assert bench.measured_traffic("wl", "cfgA", 100, str(tmp_path / "missing.json")) is None
