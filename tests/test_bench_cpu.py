"""Host-side checks of bench.py that need no GPU."""
import os
import subprocess
import sys

import bench

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_reported_only_for_the_profiled_kernel_sources():
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    lines = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert lines, "profiles/traffic.txt lists no measurement"
    wl, kernel, sha, rd, wr = lines[-1]
    got = bench.measured_traffic(wl, kernel)
    if sha == bench.kernel_source_hash():
        assert got == {"bytes_per_launch": float(rd) + float(wr), "read": float(rd), "written": float(wr)}
    else:
        assert got is None  # the kernels changed since the counters were taken
    assert bench.measured_traffic("no-such-workload", kernel) is None
