"""bench.py's host logic (no GPU): the committed profile summaries parse, and
the contract for more than one GPU fails with a message."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_profile_summaries_parse():
    """Keys may contain a colon ("sha256[:16]"); every number the bench reads
    from a committed summary parses, and the hash field is a 16-digit hex."""
    for name, keys in (("trace_seq64_traffic.txt", ["hbm bytes per launch",
                                                     "algorithmic bytes per launch (8 x distinct passed voxels)"]),
                       ("atomics_seq64.txt", ["line requests per traversal phase"]),
                       ("trace_seq64_instructions.txt", ["k_trace<false> SQ_INSTS_VALU"]),
                       ("calibration_mi355x.txt", ["copy GB/s", "peak atomic line requests per s"])):
        s = bench.read_summary(name)
        assert s is not None, name
        for k in keys:
            assert float(s[k]) > 0, (name, k)
        if name != "calibration_mi355x.txt":
            h = s["kernel sources sha256[:16]"]
            assert len(h) == 16 and int(h, 16) >= 0


def test_line_requests_below_updates():
    """A line request carries at least one update: the recorded traversal
    line requests cannot exceed its run-merged updates."""
    s = bench.read_summary("atomics_seq64.txt")
    lr = float(s["line requests per traversal phase"])
    upd = float(s["pass updates per launch (outside the sensor box, one per non-zero voxel counter a wave item flushes)"])
    assert 0 < lr <= upd


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "single GPU" in (r.stdout + r.stderr)


def test_oracle_baseline_processes():
    """The CPU baseline's worker processes (started before any GPU use) time
    the oracle on their stretches of a saved sequence and report the host."""
    from synth import scenegen
    w = scenegen.single_scan_16beam(seed=1)
    seq = dict(params=w["params"], scans=w["scans"] * 8, poses=w["poses"] * 8)
    b = bench.OracleBaseline(1, 2, 2, 8)
    try:
        r = b.run(seq)
    finally:
        b.close()
    assert r["kind"] == "oracle" and r["cores"] == 2 and r["value"] > 0
    assert r["single_core"]["cores"] == 1 and r["single_core"]["value"] > 0
    assert r["host"]["nproc"] >= 1
