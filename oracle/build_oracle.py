"""Builds oracle/liboracle.so with g++ (test infrastructure only).

Round-to-nearest IEEE double, no FMA contraction, no fast-math, so the
reference's rounding is the plain sequence of operations written in oracle.hpp.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", LIB, os.path.join(HERE, "oracle_capi.cpp")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
