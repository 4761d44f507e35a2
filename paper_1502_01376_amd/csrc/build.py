"""Build libhpic.so (HIP kernels for gfx950 + host runtime) with hipcc, in-tree.

The library lands in paper_1502_01376_amd/_lib/libhpic.so.  Packed FP32
instructions are disabled (-packed-fp32-ops) for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libhpic.so")
SOURCES = ["push.hip", "push3.hip", "pushc.hip", "pushq.hip", "solve.hip", "solveq.hip",
           "antenna.hip", "io.hip", "runtime.cpp"]
ARCH = os.environ.get("HPIC_ARCH", "gfx950")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def build(verbose=False, jobs=None):
    os.makedirs(LIBDIR, exist_ok=True)
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [
        "-std=c++17", "-O3", "-fPIC", "--offload-arch=%s" % ARCH,
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", HERE,
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    ]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [_hipcc()] + common + ["-x", "hip", "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    bad = [p.wait() for p in procs]
    if any(bad):
        raise RuntimeError("hipcc failed")
    link = [_hipcc(), "-shared", "-fPIC", "--offload-arch=%s" % ARCH, "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
