"""Builds the FP64 oracle library (test infrastructure) with g++.

The oracle is compiled without fast-math so that every operation is IEEE
double precision in program order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lensed_oracle.cpp")
LIB = os.path.join(HERE, "liblensed_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-Wall", "-Wextra",
           "-shared", "-fPIC", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
