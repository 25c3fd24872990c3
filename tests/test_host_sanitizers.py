"""The library's host code (partitioner, workspace layout, argument checks) built with
AddressSanitizer and UBSan and driven by a small C++ program that starts no device work.
The device objects come from the regular build; only ibmi.cpp and batch.cpp are rebuilt
with the sanitizers (host pass only)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_06377_amd", "csrc")
OBJ = os.path.join(ROOT, "_build")
OUT = os.path.join(OBJ, "host_sanitized")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DEVICE_OBJS = ["kernels", "gemm_f64_a", "gemm_f64_b", "gemm_f32", "gemm_grouped", "gemm_split"]
# Sanitizers on the host pass only (each flag behind -Xarch_host): device code is never
# instrumented.
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, " ".join(cmd[-4:]) + "\n" + r.stdout + r.stderr


def test_host_code_under_address_and_ub_sanitizers():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    objs = [os.path.join(OBJ, n + ".o") for n in DEVICE_OBJS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built (run python paper_2502_06377_amd/build.py)")
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host_objs = []
    for name in ("ibmi", "batch"):
        o = os.path.join(OUT, name + ".o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + SAN + inc +
             ["-c", os.path.join(CSRC, name + ".cpp"), "-o", o])
        host_objs.append(o)
    drv_o = os.path.join(OUT, "abi_host_checks.o")
    _run([HIPCC, "-x", "c++", "-O1", "-g", "-std=c++17"] + SAN + inc +
         ["-c", os.path.join(ROOT, "tests", "host", "abi_host_checks.cpp"), "-o", drv_o])
    drv = os.path.join(OUT, "abi_host_checks")
    _run([HIPCC, "--offload-arch=gfx950"] + SAN + [drv_o] + host_objs + objs + ["-o", drv])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([drv], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
