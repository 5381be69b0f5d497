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


# Sanitizer builds (AddressSanitizer and UndefinedBehaviorSanitizer, host code only):
# liboracle_san.so and libcpu_parallel_san.so, loaded instead of the plain ones when
# FMM_SANITIZE=1 (with libasan preloaded into the interpreter).
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer", "-g"]


def lib_path(name: str, sanitize: bool) -> str:
    return os.path.join(HERE, name.replace(".so", "_san.so") if sanitize else name)


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = lib_path("liboracle.so", sanitize)
    par_lib = lib_path("libcpu_parallel.so", sanitize)
    extra = SAN_FLAGS if sanitize else []
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"] + extra + [
           "-o", lib + ".tmp"] + [s for s in SOURCES if os.path.exists(s)] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    par = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", "-Wno-unused-function"
           ] + extra + ["-o", par_lib + ".tmp"] + PAR_SOURCES + ["-lm"]
    if verbose:
        print(" ".join(par), flush=True)
    subprocess.run(par, check=True)
    os.replace(par_lib + ".tmp", par_lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
