"""Build libmcx.so (HIP for gfx950) in-tree with hipcc.

Each source is compiled on its own; the FP64 kernels are compiled without
multiply-add contraction, the mixed-precision kernels with it and with
reciprocal-based FP32 division.  Packed FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmcx.so")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", os.path.join(ROOT, "include"),
          "-I", CSRC, "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function"]

UNITS = [
    # FP64 path: IEEE division and square root, no multiply-add fusion
    ("kernels_fp64.hip", ["-ffp-contract=off"]),
    # mixed path: FP32 physics may use reciprocal-based division (v_rcp, 1 ulp)
    # and the hardware square root, and flushes FP32 denormals; infinities and
    # NaNs keep their IEEE meaning
    ("kernels_mixed.hip", ["-freciprocal-math", "-fno-signed-zeros", "-fno-trapping-math", "-fno-math-errno",
                           "-fgpu-flush-denormals-to-zero", "-fno-hip-fp32-correctly-rounded-divide-sqrt"]),
    ("runtime.hip", []),
    ("influence.hip", []),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {os.path.basename(cmd[-1])}")
    return r


def build(verbose: bool = False, defines=(), lib: str = LIB, out: str = OUT) -> str:
    """Compile and link; `defines` are extra -D flags for the device code."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    os.makedirs(out, exist_ok=True)
    cmds, objs = [], []
    for src, extra in UNITS:
        obj = os.path.join(out, src + ".o")
        cmds.append([hipcc] + COMMON + [f"-D{d}" for d in defines] + extra + ["-c", "-o", obj, os.path.join(CSRC, src)])
        objs.append(obj)
    tobj = os.path.join(out, "tables.o")
    cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"),
                 "-I", CSRC, "-c", "-o", tobj, os.path.join(CSRC, "tables.cpp")])
    objs.append(tobj)
    # the units are independent: compile them side by side
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd))
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    failed = None
    for cmd, pr in procs:
        so, se = pr.communicate()
        if pr.returncode != 0 and failed is None:
            sys.stderr.write(" ".join(cmd) + "\n" + so + se)
            failed = os.path.basename(cmd[-1])
    if failed:
        raise RuntimeError(f"build step failed: {failed}")
    tmp = lib + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
