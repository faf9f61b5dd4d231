"""Command-line contract of bench.py that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    # The solver runs on one GPU: asking for more must end with exit code 2
    # and one JSON line that names the error, before any GPU work starts.
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    msg = json.loads(lines[0])
    assert "error" in msg and "one GPU" in msg["error"]


def test_rho_last_skips_unchecked_cycles():
    # cycles without a check carry NaN in the history; the rate is taken
    # per cycle between the last two checked entries
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    nan = float("nan")
    h = np.array([1.0, 0.5, 0.25, nan, nan, 0.25 * 0.125, nan, 0.25 * 0.125 * 0.25])
    assert abs(bench.rho_last(h) - 0.5) < 1e-15
    assert abs(bench.rho_last(np.array([1.0, 0.5, 0.2])) - 0.4) < 1e-15
    assert bench.rho_last(np.array([1.0, 0.5])) is None


def test_workloads_that_take_N_have_a_default():
    # every workload that reads --N has its own default (a missing one once
    # made --workload neumann divide by zero), and --N overrides it
    import argparse
    sys.path.insert(0, ROOT)
    import bench
    for w, n in (("flower513", 512), ("flower257", 256), ("probe513", 512), ("cycle_options", 256),
                 ("neumann", 256)):
        assert bench.intervals(argparse.Namespace(N=0, workload=w)) == n
        assert bench.intervals(argparse.Namespace(N=64, workload=w)) == 64
