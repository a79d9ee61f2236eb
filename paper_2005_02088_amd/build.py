"""Builds libcamelot.so (HIP kernels for gfx950 + the host runtime) in-tree.

    python -m paper_2005_02088_amd.build        # or build() from Python

Every source is compiled with hipcc for gfx950 only. Packed FP32 instructions
are disabled for device code (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcamelot.so")
ROOFLINE_EXE = os.path.join(HERE, "camelot_mlp_roofline")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["stages.hip", "handoff.hip", "predictor.hip", "noalloc.hip", "stream.hip", "runtime.cpp", "learned.cpp", "server.cpp", "alloc.cpp",
           "dtree.cpp"]
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", "runtime.cpp", "learned.cpp")) else []
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    # the standalone roofline driver of the MLP stage (links the library in place)
    inc = os.path.join(os.path.dirname(HERE), "include")
    cmd = [HIPCC, "-O2", "-std=c++17", f"--offload-arch={ARCH}", f"-I{inc}", os.path.join(CSRC, "mlp_roofline.cpp"),
           "-o", ROOFLINE_EXE + ".tmp", f"-L{HERE}", "-lcamelot", "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"roofline driver build failed:\n{r.stderr}")
    os.replace(ROOFLINE_EXE + ".tmp", ROOFLINE_EXE)
    if verbose:
        print(f"built {LIB} and {ROOFLINE_EXE}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
