"""Build libcdcc.so (the C-ABI ladder library) for gfx950 with hipcc, in tree.

Usage: python -m paper_2512_21909_amd.build [-v]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcdcc.so")
BUILD = os.path.join(PKG, "_build")

HIP_SOURCES = ["kernels_f64.hip", "kernels_mixed.hip", "kernels_split128.hip", "kernels_density.hip",
               "kernels_partial.hip", "kernels_cd.hip", "noalloc.hip"]
CXX_SOURCES = ["layout.cpp", "cdcc.cpp"]

ARCH = "gfx950"
# Packed-FP32 instructions are switched off for all device code.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-ffp-contract=fast",
                # keep MFMA accumulators in VGPRs: avoids an AGPR<->VGPR copy of
                # every accumulator on each K step of the main loops (the AGPRs
                # then hold MFMA operands and values that are seldom touched)
                "-mllvm", "-amdgpu-mfma-vgpr-form"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    jobs = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([hipcc, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + DEVICE_FLAGS + inc)
    for src in CXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        # host-only translation units (HIP runtime API, no device code)
        jobs.append([hipcc, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(CSRC, src), "-o", obj]
                    + HOST_FLAGS + inc + ["-I/opt/rocm/include"])
    with ThreadPoolExecutor(max_workers=min(4, len(jobs))) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
         + ["-L/opt/rocm/lib", "-lamdhip64", "-ldl", "-Wl,-rpath,/opt/rocm/lib"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
