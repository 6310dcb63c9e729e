"""Builds libsfqed.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SOURCES = ["csrc/tables.hip", "csrc/step.hip", "csrc/grid.hip", "csrc/mlp.hip", "csrc/api.cpp", "csrc/mlp_api.cpp",
           "csrc/noalloc.hip", "csrc/validate.hip"]
LIB = PKG / "libsfqed.so"


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def flags() -> list[str]:
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-x", "hip",
            # packed FP32 instructions stay off (device feature; the host pass ignores it)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", str(ROOT / "include"), "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> Path:
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), *flags(), *[str(PKG / s) for s in SOURCES], "-o", str(tmp)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
