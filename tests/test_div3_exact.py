"""The FP32 division by 3 of the upwind solve (div3 in fmm_device.hpp) is the IEEE
quotient for every finite binary32 input.

div3 takes q0 = x * RN(1/3), the exact residual r = fma(-3, q0, x) and returns
fma(r, RN(1/3), q0).  This test runs that sequence over all 2^31 non-negative binary32
values, denormals included, in C on the host (IEEE binary32 arithmetic with true fused
multiply-adds, as on the device with its FP32 denormals on) and compares every result
bit for bit with x / 3.  The rounding is odd-symmetric, so negative inputs follow.
"""
import os
import platform
import shutil
import subprocess

import pytest

SRC = r"""
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float f(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }
static uint32_t b(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
int main(void) {
    const float c = f(0x3eaaaaabu);
    if (b(1.0f / 3.0f) != 0x3eaaaaabu) return 2;
    long long bad = 0;
#pragma omp parallel for reduction(+ : bad) schedule(static, 1 << 20)
    for (long long u = 0; u < 0x7f800000LL; ++u) {
        const float x = f((uint32_t)u);
        const float q0 = x * c;
        const float r = __builtin_fmaf(-3.0f, q0, x);
        const float q1 = __builtin_fmaf(r, c, q0);
        if (b(q1) != b(x / 3.0f)) ++bad;
    }
    printf("%lld\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None or platform.machine() not in ("x86_64", "AMD64"),
                    reason="needs gcc on x86-64 (-mfma)")
def test_div3_is_the_ieee_quotient_for_all_binary32(tmp_path):
    src = tmp_path / "div3.c"
    exe = tmp_path / "div3"
    src.write_text(SRC)
    subprocess.run(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-o", str(exe),
                    str(src)], check=True)
    env = dict(os.environ, OMP_NUM_THREADS=str(min(8, os.cpu_count() or 1)))
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout + out.stderr
