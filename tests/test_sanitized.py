"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the sanitizer variants (paper_1811_00009_amd/build.py --sanitize: the library's
host code -- argument checks, source set-up, workspace layout, tune cache -- with ASan
and UBSan, its device code as usual; oracle/build.py --sanitize: the oracle and the
OpenMP block solver) and runs the CPU tests that exercise them in child processes with
FMM_SANITIZE=1 and the sanitizer runtime preloaded into the interpreter.  The library is
compiled by clang and the oracle by gcc, whose runtimes cannot share a process, so they
run in two passes.  A report from either sanitizer fails the child and this test.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _clang_asan():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _gcc_runtime(name):
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run(preload, tests):
    env = dict(os.environ, FMM_SANITIZE="1", LD_PRELOAD=" ".join(preload),
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"]
    cmd += [os.path.join(ROOT, "tests", t) for t in tests]
    out = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
    text = out.stdout + out.stderr
    assert out.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("hipcc") is None or _clang_asan() is None
                    or _gcc_runtime("libasan.so") is None,
                    reason="needs hipcc, the ROCm clang ASan runtime and gcc's libasan")
def test_host_code_is_clean_under_asan_and_ubsan():
    subprocess.run([sys.executable, os.path.join(ROOT, "paper_1811_00009_amd", "build.py"),
                    "--sanitize"], check=True, capture_output=True)
    subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "build.py"), "--sanitize"],
                   check=True, capture_output=True)
    try:
        # the library's host code (clang runtime; the ASan runtime holds the UBSan handlers)
        _run([_clang_asan()], ["test_abi.py", "test_zz_no_alloc.py"])
        # the oracle and the OpenMP block solver (gcc runtimes)
        _run([_gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")], ["test_oracle_pins.py"])
    finally:
        # the instrumented builds are for this test only
        for lib in glob.glob(os.path.join(ROOT, "oracle", "*_san.so")) + \
                glob.glob(os.path.join(ROOT, "paper_1811_00009_amd", "*_san.so")):
            os.remove(lib)
