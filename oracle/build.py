"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is compiled with plain g++; its flags keep every floating-point
operation under the rounding mode that fesetround() selected: no constant
folding or contraction across mode switches, no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-frounding-math",
         "-fno-fast-math", "-ffp-contract=off", "-fno-builtin", "-Wall", "-Wextra"]


def build(verbose=False):
    cmd = ["g++", *FLAGS, SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
