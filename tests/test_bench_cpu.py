"""bench.py contract checks that need no GPU: it measures one GPU only and
says so when asked for more."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_profiled_source_and_tile():
    """The roofline block's `traffic` comes from the committed counter summary
    and only applies to the step sources and the tile it was taken on."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    for workload in ("3d-256-o8", "3d-512-o16", "batch2d-o8"):
        rec = json.load(open(os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")))
        tile = rec["tile"]
        if rec["kernel_source_sha256_16"] == bench.step_kernel_sha():
            assert bench.measured_traffic(workload, tile) == rec["hbm_bytes_per_launch"]
        else:
            assert bench.measured_traffic(workload, tile) is None
        assert bench.measured_traffic(workload, tile + 1) is None
    assert bench.measured_traffic("no-such-workload", 0) is None
