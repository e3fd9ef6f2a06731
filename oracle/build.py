"""Build the CPU oracle (test infrastructure) into oracle/libffo.so.

Plain g++ -O2, single-threaded code, no vectorisation flags beyond the
default, no fused multiply-add contraction (the three double-precision tables
are generated with exactly the operations written in the source).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ff_oracle.cpp")
LIB = os.path.join(HERE, "libffo.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
