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


def test_source_digest_follows_the_code_not_its_comments():
    csrc = os.path.join(ROOT, "paper_2201_01257_amd", "csrc")
    texts = {n: open(os.path.join(csrc, n), encoding="utf-8").read()
             for n in ("kernels.hip", "device_util.h", "internal.h", "plan.cpp")}
    base = bench.kernel_source_digest(texts)
    assert base == bench.kernel_source_digest()
    commented = dict(texts, **{"kernels.hip": "// a new comment\n/* and a block\n   comment */\n" + texts["kernels.hip"]})
    assert bench.kernel_source_digest(commented) == base
    changed = dict(texts, **{"kernels.hip": texts["kernels.hip"].replace("constexpr int NS = KT / 4;", "constexpr int NS = KT / 8;", 1)})
    assert changed["kernels.hip"] != texts["kernels.hip"]
    assert bench.kernel_source_digest(changed) != base
    # string literals are code: "//" inside one does not start a comment
    assert bench._code_only('f("a // b");  // c') == 'f("a // b");'
    assert bench._code_only('x = 1; /* y */ z = "/* w */";') == 'x = 1; z = "/* w */";'
