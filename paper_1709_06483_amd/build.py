"""Build libmagnus.so in-tree for gfx950.

    python -m paper_1709_06483_amd.build

Compiles the host planner with g++, the HIP sources with hipcc
(--offload-arch=gfx950, packed-FP32 instructions disabled), and links one
shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmagnus.so")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    return cmd, p.returncode, p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = [
        ["g++", "-O2", "-fPIC", "-std=c++17", "-Wall", "-c", os.path.join(CSRC, "planner.cpp"),
         "-o", os.path.join(OBJ, "planner.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(OBJ, "kernels.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_multi.hip"), "-o", os.path.join(OBJ, "kernels_multi.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_mfma.hip"), "-o", os.path.join(OBJ, "kernels_mfma.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_persist.hip"), "-o", os.path.join(OBJ, "kernels_persist.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_gemm.hip"), "-o", os.path.join(OBJ, "kernels_gemm.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_comm.hip"), "-o", os.path.join(OBJ, "kernels_comm.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels_stream.hip"), "-o", os.path.join(OBJ, "kernels_stream.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "abi.hip"), "-o", os.path.join(OBJ, "abi.o")],
    ]
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        results = list(ex.map(_run, jobs))
    for cmd, rc, out in results:
        if verbose or rc != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + out)
        if rc != 0:
            raise RuntimeError("compilation failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC",
           os.path.join(OBJ, "planner.o"), os.path.join(OBJ, "kernels.o"), os.path.join(OBJ, "kernels_multi.o"),
           os.path.join(OBJ, "kernels_mfma.o"), os.path.join(OBJ, "kernels_persist.o"),
           os.path.join(OBJ, "kernels_gemm.o"), os.path.join(OBJ, "kernels_comm.o"),
           os.path.join(OBJ, "kernels_stream.o"), os.path.join(OBJ, "abi.o"),
           "-o", tmp]
    _, rc, out = _run(cmd)
    if verbose or rc != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + out)
    if rc != 0:
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
