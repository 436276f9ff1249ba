"""Compile the FP64 oracle (plain C, OpenMP) into oracle/libbp_oracle.so.

Test infrastructure: the resulting library is loaded only by the test suite,
the smoke check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["bp_oracle.c", "bp_oracle_adjoint.c", "bp_oracle_remap.c", "bp_oracle_features.c"]
LIB = os.path.join(HERE, "libbp_oracle.so")
# Optimised for the AVX2/FMA generation of x86-64 (the library travels to
# other hosts with the tree, so not -march=native); no contraction of
# multiply-adds, so every value is the plain C expression's.
FLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11"] + FLAGS + ["-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
