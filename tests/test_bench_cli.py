"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message, and the oracle-only timing prints one JSON line per size."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args, timeout=300):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_cpu_only_oracle_timing_prints_one_line_per_size():
    r = _run("--cpu-only", "8,16", "--cpu-seconds", "0")
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [json.loads(x) for x in r.stdout.splitlines() if x.startswith("{")]
    assert [x["n"] for x in lines] == [8, 16]
    for x in lines:
        cb = x["cpu_baseline"]
        assert cb["kind"] == "oracle" and cb["unit"] == "cells/s" and cb["value"] > 0 and cb["cores"] >= 1
