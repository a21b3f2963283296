"""Builds the HIP library ``lib/libispl.so`` for gfx950 with hipcc.

Usage: ``python -m paper_2311_18737_amd.build`` (or ``build()`` from Python).
Every call compiles from source.
"""

from __future__ import annotations

import os
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_DIR = os.path.join(PKG_DIR, "lib")
LIB_PATH = os.path.join(LIB_DIR, "libispl.so")
SOURCES = ["ispl_kernels.hip", "ispl_zoom.hip", "ispl_cnn.hip", "ispl_lzoom.hip", "ispl_noalloc.hip",
           "ispl_api.cpp", "ispl_stream.cpp"]
ARCH = "gfx950"


def hipcc_command(out_path: str = LIB_PATH, extra=()) -> list:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    return [
        hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are disabled for the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-command-line-argument",
        "-I", INCLUDE, "-I", CSRC,
        *extra,
        "-o", out_path,
        *[os.path.join(CSRC, s) for s in SOURCES],
    ]


def build(verbose: bool = True) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    if verbose and res.stderr.strip():
        # hipcc's host pass does not know the packed-fp32 feature; keep other warnings
        lines = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l]
        if any(l.strip() for l in lines):
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build()
