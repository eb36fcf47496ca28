"""Build step for the CPU oracle library (test infrastructure only).

Compiles ``osc_oracle.c`` into ``liboscoracle.so`` next to this file with
plain gcc: FP64, no FMA contraction, OpenMP over events, portable x86-64
code (no ``-march=native``, so the library also runs on another host).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "osc_oracle.c")
LIB = os.path.join(HERE, "liboscoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
