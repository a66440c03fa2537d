"""bench.py command line on the host: the single-GPU guard and the argument
set (no device work)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "single GPU" in msg["error"]


def test_workload_choices():
    r = _run("--help")
    assert r.returncode == 0
    for name in ("prism_f4_np_1024", "prism_f8_np_2048", "prism_f2_sc_256"):
        assert name in r.stdout
    r = _run("--workload", "no_such_workload")
    assert r.returncode != 0


def test_subset_index_and_detector_errors():
    """The benchmark's accuracy report: the probe subset it reads out of the
    timed scan is the scan's every n-th position, and its element-wise gate
    catches one wrong dark-field bin that the norm-wise errors miss."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    w = W.WORKLOADS["prism_f4_np_1024"]
    full = W.scan_positions(w.cell, *w.scan)
    idx = bench.subset_index(w.scan, 8)
    assert np.array_equal(full[idx], W.scan_positions(w.cell, *w.scan, sub=8))
    rng = np.random.default_rng(3)
    ref = np.concatenate([rng.uniform(0.01, 0.05, (20, 20)), rng.uniform(1e-6, 1e-5, (20, 45))], axis=1)
    ok = bench.detector_errors(ref * (1 + 1e-6), ref)
    assert ok["within_1e-4"] and ok["rel_all"] < 2e-6
    bad = ref.copy()
    bad[3, 50] *= 2.0                       # one dark-field bin 100% off
    e = bench.detector_errors(bad, ref)
    assert e["rel_all"] < 1e-4 and not e["within_1e-4"] and e["worst_bin"] == 50
