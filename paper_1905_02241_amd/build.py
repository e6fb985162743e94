"""Build libmech.so (HIP, gfx950) in-tree.

    python -m paper_1905_02241_amd.build          # compile
    python -m paper_1905_02241_amd.build --asm [DIR]   # also write the gfx950 assembly
                                                       # to DIR (default _build/asm)

Flags: -O3, FP64 hardware atomics (-munsafe-fp-atomics), packed FP32
instructions disabled (-target-feature -packed-fp32-ops), C++17; linked
against the roctx library for the entry points' trace ranges.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmech.so")
SOURCES = [os.path.join(CSRC, f) for f in ("mech_kernels.hip", "mech_runtime.hip")]
HEADERS = [os.path.join(CSRC, "mech_internal.h"), os.path.join(CSRC, "mech_math.h"), os.path.join(ROOT, "include", "mech.h")]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wl,-rpath,/opt/rocm/lib", "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
]


def build(asm: str = "", verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if asm:
        out = asm
        os.makedirs(out, exist_ok=True)
        subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-munsafe-fp-atomics",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
                               SOURCES[0], "-o", os.path.join(out, "mech_kernels.s")])
    return LIB


if __name__ == "__main__":
    asm_dir = ""
    if "--asm" in sys.argv:
        i = sys.argv.index("--asm")
        asm_dir = sys.argv[i + 1] if i + 1 < len(sys.argv) else os.path.join(ROOT, "_build", "asm")
    build(asm=asm_dir, verbose=True)
