"""Compile the FP64 oracle into ``oracle/librbo.so`` with g++ and OpenMP."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.environ.get("RBO_ORACLE_LIB") or os.path.join(HERE, "librbo.so")
SRC = [os.path.join(HERE, "rbo.cpp")]


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-o", LIB + ".tmp"] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
