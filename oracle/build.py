"""Build the oracle shared library (plain C, gcc) -- test infrastructure only.

The oracle is compiled without floating-point contraction so that every
operation rounds exactly as written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "fmm_oracle.c"), os.path.join(HERE, "mlp_oracle.c")]
PAR_LIB = os.path.join(HERE, "libcpu_parallel.so")  # the paper's OpenMP block solver
PAR_SOURCES = [os.path.join(HERE, "cpu_parallel.c")]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter",
           "-o", LIB + ".tmp"] + [s for s in SOURCES if os.path.exists(s)] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    par = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", "-Wno-unused-function",
           "-o", PAR_LIB + ".tmp"] + PAR_SOURCES + ["-lm"]
    if verbose:
        print(" ".join(par), flush=True)
    subprocess.run(par, check=True)
    os.replace(PAR_LIB + ".tmp", PAR_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
