"""Compile the FP64 oracle into oracle/libccfr_oracle.so (test infrastructure).

gcc, C11, OpenMP over vertices and pairs, no fast-math and no FP contraction, so
that the FP32 box arithmetic of the candidate contract is plain IEEE single and
the FP64 arithmetic follows the source expression by expression.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libccfr_oracle.so")
SOURCES = ["oracle_geometry.c", "oracle_candidates.c", "oracle_regions.c",
           "oracle_projection.c", "oracle_response.c", "oracle_xpbd.c", "oracle_checks.c"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
