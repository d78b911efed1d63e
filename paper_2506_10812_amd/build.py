"""Build the HIP library libsg.so for gfx950 (in-tree) with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsg.so")
SOURCES = ["sg_api.hip", "sg_table.hip", "sg_direct.hip", "sg_fftpath.hip", "sg_adjoint.hip",
           "sg_semispec.hip"]
ARCH = os.environ.get("SG_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


GEN = os.path.join(OBJ, "include")  # generated headers


def _generate() -> None:
    """Host step: build and run gen_cheb64.cpp, which writes sg_cheb64.h (the
    Chebyshev coefficients of the double mid-range F(x) branch)."""
    os.makedirs(GEN, exist_ok=True)
    exe = os.path.join(OBJ, "gen_cheb64")
    subprocess.check_call(["g++", "-O2", "-std=c++17", os.path.join(CSRC, "gen_cheb64.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("gen_cheb64 failed")
    with open(os.path.join(GEN, "sg_cheb64.h"), "w") as fh:
        fh.write(r.stdout)


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, "-I", GEN, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    _generate()
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
