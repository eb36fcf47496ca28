"""Build step for the CPU oracle library (test infrastructure only).

Compiles ``osc_oracle.c`` with plain gcc: FP64, no FMA contraction, OpenMP
over events.  The library the tests load, ``liboscoracle.so``, is portable
x86-64 code at -O2 (it also runs on another host).  For timing the oracle
on the host that runs the benchmark, ``build(native=True)`` compiles the
same source at -O3 -march=native into ``liboscoracle_native.so``; only the
CPU-baseline leg of the benchmark loads that one, after building it on the
host it times.  Both builds keep -ffp-contract=off and no fast-math, so
they compute the same values.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "osc_oracle.c")
LIB = os.path.join(HERE, "liboscoracle.so")
NATIVE_LIB = os.path.join(HERE, "liboscoracle_native.so")


def build(verbose: bool = False, native: bool = False) -> str:
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    out = NATIVE_LIB if native else LIB
    cmd = ["gcc", "-std=gnu11", *opt, "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
