"""Builds the HIP library libpolfed.so for gfx950 in-tree.

    python -m paper_2605_10191_amd.build          (from the repository root)

Every source under csrc/ is compiled by hipcc into _build/ and linked into
paper_2605_10191_amd/libpolfed.so.  It always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpolfed.so")
BUILD = os.path.join(ROOT, "_build")

ARCH = os.environ.get("POLFED_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
# Packed FP32 instructions are disabled: the compiler must not form
# v_pk_* FP32 arithmetic on its own.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Wno-unknown-pragmas", f"-I{os.path.join(ROOT, 'include')}"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


# plain host C++ (no HIP headers), built by the system compiler with OpenMP
HOST_ONLY = {"eig.cpp"}
HOST_CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-fopenmp"]


def compile_one(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if os.path.basename(src) in HOST_ONLY:
        cmd = [shutil.which("g++") or "g++", *HOST_CXXFLAGS, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj
    cmd = [hipcc(), f"--offload-arch={ARCH}", *NO_PACKED_FP32, *CXXFLAGS,
           "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # hipcc's host pass warns about the device-only feature flag; drop that
    lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln
             and "not a recognized feature" not in ln]
    if any("warning" in ln for ln in lines):
        sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = OUT + ".tmp"
    # the host eigensolvers use GNU OpenMP (the runtime PyTorch loads too)
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}", "-lgomp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
