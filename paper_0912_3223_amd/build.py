"""Build liblpm.so (HIP, gfx950) in-tree with hipcc.

    python paper_0912_3223_amd/build.py

(Run it as a script: importing the package loads the library being built.)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = [os.path.join(PKG, "csrc", "lpm.hip"), os.path.join(PKG, "csrc", "lpm_receptor.hip")]
DEPS = SRC + [os.path.join(PKG, "csrc", "lpm_device.h"), os.path.join(PKG, "csrc", "lpm_host.h"),
              os.path.join(ROOT, "include", "lpm.h")]
LIB = os.path.join(PKG, "liblpm.so")
ARCH = os.environ.get("LPM_OFFLOAD_ARCH", "gfx950")

# Packed FP32 VALU ops are disabled: hand-written or compiler-formed
# v_pk_*_f32 have given silent wrong results on these parts.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), *SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
