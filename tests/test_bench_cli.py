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
