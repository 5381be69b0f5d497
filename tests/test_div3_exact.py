"""The FP32 divisions by k = 1, 2, 3 of the upwind solve (div_k in fmm_device.hpp) are
the IEEE quotient for every finite binary32 input.

div_k takes q0 = x * c_k with c_k = 1, 1/2, RN(1/3), the exact residual
r = fma(-k, q0, x) and returns fma(r, c_k, q0).  For k = 1 and 2 the product is the
correctly rounded quotient already and the correction leaves it unchanged; for k = 3 the
correction makes it so.  This test runs that sequence over all 2^31 non-negative binary32
values, denormals included, for each k, in C on the host (IEEE binary32 arithmetic with
true fused multiply-adds, as on the device with its FP32 denormals on) and compares every
result bit for bit with x / k.  The rounding is odd-symmetric, so negative inputs follow.
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
    if (b(1.0f / 3.0f) != 0x3eaaaaabu) return 2;
    const float cs[3] = {1.0f, 0.5f, f(0x3eaaaaabu)};
    long long bad = 0;
    for (int k = 1; k <= 3; ++k) {
        const float c = cs[k - 1], kf = (float)k;
#pragma omp parallel for reduction(+ : bad) schedule(static, 1 << 20)
        for (long long u = 0; u < 0x7f800000LL; ++u) {
            const float x = f((uint32_t)u);
            const float q0 = x * c;
            const float r = __builtin_fmaf(-kf, q0, x);
            const float q1 = __builtin_fmaf(r, c, q0);
            if (b(q1) != b(x / kf)) ++bad;
        }
    }
    printf("%lld\n", bad);
    return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None or platform.machine() not in ("x86_64", "AMD64"),
                    reason="needs gcc on x86-64 (-mfma)")
def test_div_k_is_the_ieee_quotient_for_all_binary32(tmp_path):
    src = tmp_path / "div3.c"
    exe = tmp_path / "div3"
    src.write_text(SRC)
    subprocess.run(["gcc", "-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-o", str(exe),
                    str(src)], check=True)
    env = dict(os.environ, OMP_NUM_THREADS=str(min(8, os.cpu_count() or 1)))
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert out.returncode == 0 and out.stdout.strip() == "0", out.stdout + out.stderr
