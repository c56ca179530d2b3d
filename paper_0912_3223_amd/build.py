"""Build liblpm.so (HIP, gfx950) in-tree with hipcc.

    python paper_0912_3223_amd/build.py

(Run it as a script: importing the package loads the library being built.)
The translation units -- host code and gridding, the receptor adjoint, one
slice of the plain step-kernel variants per (wind components, time
interpolation), one block size of the ensemble step kernels per unit -- are
compiled to objects in parallel and linked into one shared library.
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
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liblpm.so")
ARCH = os.environ.get("LPM_OFFLOAD_ARCH", "gfx950")

# (object name, source, defines)
UNITS = [
    ("lpm", "lpm.hip", []),
    ("lpm_receptor", "lpm_receptor.hip", []),
    ("lpm_ensemble", "lpm_ensemble.hip", []),
] + [
    (f"step_plain_{nc}{'stp'[t]}", "lpm_step_plain.hip",
     [f"-DLPM_SLICE_NCOMP={nc}", f"-DLPM_SLICE_TIME={t}"])
    for nc in (2, 3) for t in (0, 1, 2)
] + [
    (f"step_ensemble_{b}", "lpm_step_ensemble.hip", [f"-DLPM_SLICE_BLOCK={b}"])
    for b in (128, 256, 512)
]
DEPS = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))] + \
    [os.path.join(ROOT, "include", "lpm.h")]

# Packed FP32 VALU ops are disabled: hand-written or compiler-formed
# v_pk_*_f32 have given silent wrong results on these parts.
HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(unit, verbose):
    name, src, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [hipcc(), *HIPCC_FLAGS, *defs, "-I", os.path.join(ROOT, "include"), "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    return obj, r.returncode, out


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    failed = [(o, out) for o, rc, out in results if rc != 0]
    for o, rc, out in results:
        if out.strip() and (verbose or rc != 0):
            print(out, flush=True)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(os.path.basename(o) for o, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC",
           *[o for o, _, _ in results], "-o", tmp]
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
    print(build(verbose="-v" in sys.argv))
    sys.exit(0)
