"""Host-side contract of bench.py that needs no GPU: more than one GPU is
refused with one JSON line and exit status 2, the options that pick and size
the sections exist (the profiling commands in profiles/ use them), and an
unknown section is rejected."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_is_refused_with_a_json_line():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, cwd=ROOT, timeout=120)
    assert res.returncode == 2
    line = res.stdout.strip().splitlines()[-1]
    assert "one GPU" in json.loads(line)["error"]


def test_side_workload_switches_exist():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                         cwd=ROOT, timeout=120)
    assert res.returncode == 0
    for opt in ("--steps", "--warmup", "--only", "--fp64-steps", "--batch", "--large", "--large-reps",
                "--tune-large", "--roofline-kernel", "--skip-continuation", "--tune-batch", "--batch-precisions", "--batch-reps", "--cpu-sizes", "--accel-steps", "--ras-steps",
                "--mic-steps", "--robust-iters", "--no-cpu-baseline", "--tuning-db", "--reuse-tuning",
                "--adjoint-precisions", "--adjoint-reps", "--fd-cells", "--large-fp64-reps"):
        assert opt in res.stdout, opt


def test_unknown_section_is_rejected():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--only", "headline,nosuch"],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert res.returncode == 2
    assert "nosuch" in res.stderr
