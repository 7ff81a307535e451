"""Build the CPU oracle (liboracle_mco.so) with plain gcc.

Test infrastructure: the oracle is the reference for the GPU library.  Flags keep
IEEE semantics: no fused multiply-add contraction, no fast-math, SSE2 floating
point (x86-64 default), so every fp32/fp64 operation rounds exactly once.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mco.c")
LIB = os.path.join(HERE, "liboracle_mco.so")

CFLAGS = ["-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
          "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
          "-Wall", "-Wextra", "-Wno-unused-parameter", "-pthread"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
