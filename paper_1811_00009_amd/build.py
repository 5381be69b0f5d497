"""Build the HIP library (libfmm_hip.so) in-tree for gfx950 with hipcc.

Flags: -O3; no floating-point contraction, correctly rounded FP32 divide and
square root (the solver's arithmetic rounds exactly as written); packed FP32
instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmm_hip.so")
SOURCES = ["fmm_host.hip", "fmm_mlp.hip"]
ARCH = os.environ.get("FMM_OFFLOAD_ARCH", "gfx950")


# The profiling build: the same sources with the per-segment cycle account compiled in
# (timestamps at each segment boundary of a pop, read back by fmm_cycle_account).
CYCLES_LIB = os.path.join(HERE, "libfmm_hip_cycles.so")
# The sanitizer build: host code (argument checks, source set-up, workspace layout, tune
# cache) under AddressSanitizer and UBSan, device code as usual; loaded instead of the
# plain library when FMM_SANITIZE=1 (CPU tests, with libasan preloaded).
SAN_LIB = os.path.join(HERE, "libfmm_hip_san.so")
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose: bool = False, cycles: bool = False, sanitize: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    lib = CYCLES_LIB if cycles else (SAN_LIB if sanitize else LIB)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
           "-I", os.path.join(os.path.dirname(HERE), "include"),
           "-o", lib + ".tmp"] + (["-DFMM_CYCLES"] if cycles else []) + (
           SAN_HOST_FLAGS if sanitize else []) + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, cycles="--cycles" in sys.argv,
          sanitize="--sanitize" in sys.argv)
