"""Compiles the HIP sources into libsrgrav.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB_PATH = os.path.join(PKG, "libsrgrav.so")
SOURCES = ["api.hip", "build.hip", "walk.hip", "pm.hip", "sph.hip"]

# -ffp-contract=off: the FP64 decisions and moment folds are reproduced bit for
# bit, so nothing may be fused behind the source's back (FP32 code asks for FMA
# explicitly).  Packed FP32 instructions are disabled on purpose.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-munsafe-fp-atomics", "-mllvm", "-amdgpu-atomic-optimizer-strategy=None", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = ["hipcc", "-c", *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    # hipFFT provides the PM mesh's 3D FFTs
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
                    "-L/opt/rocm/lib", "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    os.replace(tmp, LIB_PATH)
    for o in objs:
        os.remove(o)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
