"""Compiles libwct.so (HIP for gfx950) in-tree from paper_2104_08265_amd/csrc.

Usage: python -m paper_2104_08265_amd.build  (or build() from Python).  hipcc
cross-compiles for gfx950 without a GPU present.
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
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libwct.so")
DIGEST = os.path.join(PKG, "libwct.sha256")  # digest of the sources libwct.so was built from

ARCH = "gfx950"
COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware float/double atomic adds on coarse-grained device memory
    "-munsafe-fp-atomics",
]
# Sources and per-file extra flags.  The raster carries the deterministic fluctuation
# chain, the drift its FP64 arithmetic in the order written and the ADC one rounding per
# operation: none of them may contract a*b+c into fused multiply-adds.
SOURCES = {
    "api.cpp": ["-x", "hip"],
    "raster.hip": ["-ffp-contract=off"],
    "conv.hip": [],
    "conv_ct.hip": [],
    "wiredirect.hip": [],
    "plan.hip": [],
    "grad.hip": [],
    "probe.cpp": ["-x", "hip"],
    "adc.hip": ["-ffp-contract=off"],
    "drift.hip": ["-ffp-contract=off"],
}


def sources_digest() -> str:
    """SHA-256 over the kernel and ABI sources (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".hpp", ".cpp", ".h")):
                with open(os.path.join(d, name), "rb") as f:
                    h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


ROCM_LIB = "/opt/rocm/lib"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain (ROCm) is required to build libwct.so")


def _compile(src: str, flags: list[str], verbose: bool) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link libwct.so; returns the library path."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    digest = sources_digest()
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    # roctx (named ranges around the ABI calls) from the ROCm install, found at run time there
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, f"-L{ROCM_LIB}",
           "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libwct.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    with open(DIGEST, "w") as f:
        f.write(digest + "\n")
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
