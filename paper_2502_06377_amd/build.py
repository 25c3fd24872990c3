"""Build libibmi.so (HIP for gfx950) in-tree with hipcc.

    python paper_2502_06377_amd/build.py        # or build() from __graft_entry__

Always recompiles: every translation unit to an object under _build/ (in parallel), then one
shared library next to this file so that it travels with the tree.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libibmi.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["kernels.hip", "gemm_f64_a.hip", "gemm_f64_b.hip", "gemm_f32.hip", "gemm_grouped.hip",
           "gemm_split.hip", "ibmi.cpp", "batch.cpp"]
# Packed FP32 instructions are disabled on purpose for every device pass.  Matrix-core
# instructions take their accumulators in ordinary vector registers: with the default
# (accumulation registers) the compiler copies every accumulator out and back once per K
# stage of the GEMM loops.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-mllvm", "-amdgpu-mfma-vgpr-form=1",
            "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd[-3:])}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    incs = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
    cmds, objs = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        cmds.append([hipcc] + HIPFLAGS + incs + ["-c", os.path.join(HERE, "csrc", s), "-o", obj])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
