"""The benchmark's command-line contract that needs no GPU: more than one GPU is refused
with a JSON message and a non-zero status before anything touches a device."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_help_lists_the_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for sw in ("--steps", "--warmup", "--gpus", "--semi-implicit", "--no-cpu-baseline"):
        assert sw in r.stdout


def test_unknown_forms_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--forms-only", "--forms", "batched_paths,nope"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "unknown forms ['nope']" in r.stderr and "batched_paths" in r.stderr
