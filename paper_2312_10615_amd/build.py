"""Build the gfx950 shared libraries in-tree with hipcc: the MG-SQMR solver
(libstokes_mgsqmr.so) and the warm-start network kernels (libstokes_unet.so).

Usage: python -m paper_2312_10615_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libstokes_mgsqmr.so")
SOURCES = [os.path.join(PKG, "csrc", "stokes_mgsqmr.hip"), os.path.join(PKG, "csrc", "batched.hip")]
UNET_LIB = os.path.join(PKG, "libstokes_unet.so")
UNET_SOURCES = [os.path.join(PKG, "csrc", "unet.hip")]
TARGETS = ((LIB, SOURCES), (UNET_LIB, UNET_SOURCES))

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _build_one(lib: str, sources, verbose: bool) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), *sources, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build " + lib)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False):
    """Compile every library (always, even when one is already there); returns their paths."""
    return [_build_one(lib, src, verbose) for lib, src in TARGETS]


if __name__ == "__main__":
    print(build(verbose=True))
