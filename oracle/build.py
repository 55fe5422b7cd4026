"""Compile the FP64 oracle (plain C) into ``oracle/liboracle.so`` and, from the
same source with OpenMP, ``oracle/liboracle_omp.so``.

Test infrastructure: the libraries built here are loaded only by the tests,
the smoke check and the CPU-baseline leg of the benchmark.  The OpenMP build
splits the loops of Algorithm 1 without changing the order of any sum, so both
builds give identical bits (checked by the tests).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ibx_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _cc(out: str, extra, verbose: bool) -> None:
    # -ffp-contract=off: no fused multiply-adds, every operation rounds as written.
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra"] + extra + ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _cc(LIB, ["-Wno-unknown-pragmas"], verbose)
    _cc(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
