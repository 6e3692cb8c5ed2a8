"""Host logic of bench.py that needs no GPU: the HBM-traffic lookup and its source guard,
the roofline arithmetic per launch, and the one-GPU limit."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def write_traffic(root, workload, src, bytes_per_launch):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "traffic_%s.json" % workload), "w") as f:
        json.dump({"source_sha256": {os.path.basename(src): bench.file_sha(src)},
                   "bytes_per_launch": bytes_per_launch}, f)


def test_traffic_is_read_only_for_the_profiled_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "kernel.hip"
    src.write_text("first version\n")
    write_traffic(str(tmp_path), "w", str(src), {"k_a<1>": 123.0})
    assert bench.measured_traffic("w", "k_a<1>", str(src)) == 123.0
    assert bench.measured_traffic("w", "k_b<1>", str(src)) is None      # kernel not profiled
    assert bench.measured_traffic("other", "k_a<1>", str(src)) is None  # no counters taken
    src.write_text("second version\n")                                   # source changed since
    assert bench.measured_traffic("w", "k_a<1>", str(src)) is None


def test_committed_traffic_files_name_their_sources():
    for w in ("dna_long", "text", "protein"):
        with open(os.path.join(ROOT, "profiles", "traffic_%s.json" % w)) as f:
            t = json.load(f)
        assert {"partition.hip", "verify_lg.hip"} <= set(t["source_sha256"])
        assert all(v > 0 for v in t["bytes_per_launch"].values())


def test_anchor_roofline_counts_one_launch_per_repetition():
    reps, steps = 4, 3
    stats = [{"positions": 1e8 * reps} for _ in range(steps)]
    kms = {"anchors": 2.0 * steps}            # 2 ms of anchor launches per step
    kln = {"anchors": reps * steps}
    r = bench.roofline("anchors", stats, kms, kln, bits=6, q=6, workload="none")  # text
    assert r["kernel"] == "k_anchor_tiles<uint64_t>" and r["ops_per_position"] == 42
    assert r["avg_launch_ms"] == pytest.approx(0.5)
    assert r["achieved"] == pytest.approx(1e8 * reps * steps * 42 / 6e-3 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.INT_PEAK_TOPS)
    assert r["traffic"] is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU only" in p.stderr
