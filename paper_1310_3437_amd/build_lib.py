"""Build libkmc.so (gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with -ffp-contract=off (the only
fused multiply-adds are the explicit fma() calls of the step's definition)
and with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkmc.so")
SOURCES = [os.path.join(CSRC, "kmc_api.hip"), os.path.join(CSRC, "kmc_device.hip")]
HEADERS = [os.path.join(CSRC, "kmc_internal.h"), os.path.join(ROOT, "include", "kmc.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(force=True, verbose=False, extra=()):
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(f) for f in SOURCES + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, *extra, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + msgs)
    if verbose and msgs:
        print(msgs, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
