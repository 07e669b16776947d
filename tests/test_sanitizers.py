"""Address and undefined-behaviour sanitizers on the CPU-side code.

  * the oracle (oracle/amber_oracle.c) built by gcc with
    -fsanitize=address,undefined runs every oracle pin of the CPU tier in a
    child Python process (the sanitizer runtime preloaded, the build chosen by
    AMBER_ORACLE_LIB);
  * the library's host logic (csrc/amber_api.cpp: the history fit, the
    inversion and growth tables, the workspace layout of every grid size, the
    host argument checks) built by hipcc with host-side sanitizers into a
    CPU-only harness (tests/sanitize/), leak detection on.
Neither touches a GPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _libasan() -> str:
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-o", lib,
                           os.path.join(ROOT, "oracle", "amber_oracle.c"), "-lm"])
    env = dict(os.environ, AMBER_ORACLE_LIB=lib, LD_PRELOAD=_libasan(), ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    probe = ("import oracle; oracle.lib(); "
             "assert any(l.rstrip().endswith('liboracle_san.so') for l in open('/proc/self/maps')), 'not loaded'")
    subprocess.check_call([sys.executable, "-c", probe], cwd=ROOT, env=env)
    tests = sorted(f for f in os.listdir(os.path.join(ROOT, "tests")) if f.startswith("test_oracle_"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join("tests", f) for f in tests]], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    print(r.stdout[-600:])
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_logic_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_harness")
    csrc = os.path.join(ROOT, "paper_2109_10375_amd", "csrc")
    subprocess.check_call([HIPCC, "-x", "hip", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                           "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
                           "-o", exe, os.path.join(ROOT, "tests", "sanitize", "host_harness.cpp"),
                           os.path.join(ROOT, "tests", "sanitize", "host_stubs.cpp"),
                           os.path.join(csrc, "amber_api.cpp")], stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"), capture_output=True, text=True,
                       timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "fits:" in r.stdout and "argument checks done" in r.stdout
