"""Compile the C oracle into oracle/libhpic_oracle.so with gcc.

The oracle is test infrastructure: building it is part of the build check, but
nothing on the product path loads it.  Compiled with floating-point contraction
off so that every FP32/FP64 operation rounds once, in source order, and with
OpenMP: its parallel loops give the same bits for any number of threads
(OMP_NUM_THREADS).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hpic_oracle.c")
LIB = os.path.join(HERE, "libhpic_oracle.so")


def build(verbose=False):
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall", "-Wno-unused-function",
        SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
