"""Compile the HIP library (gfx950) in-tree: paper_2606_09275_amd/libmpmgimp.so."""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libmpmgimp.so"
SOURCES = ["mesh_gpu.hip", "assemble.hip", "solve.hip", "ghost.hip", "ghost_faces.hip", "split.hip", "prim.hip", "tree.hip", "pattern.hip"]
ARCH = os.environ.get("MPM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware FP atomics on coarse-grained device memory (hipMalloc / torch allocations)
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def build(verbose: bool = False, extra=None) -> Path:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [str(CSRC / s) for s in SOURCES]
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc] + FLAGS + list(extra or []) + ["-x", "hip"] + srcs + ["-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("HIP build failed:\n" + r.stderr[-8000:])
    if verbose and r.stderr.strip():
        print(r.stderr[-4000:], file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
