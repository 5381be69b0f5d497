"""The pair tests of the two-point march step (fmm_device.hpp) never take two points closer
than Manhattan distance 4 as a pair.

far_apart<P>(a, b) decides from the index difference of two tile points; the persistent
kernel instead compares that difference with a table of the index offsets of the short
displacements (make_close_offsets<P>, one per lane).  This test takes the functions' own
text from the header, compiles them on the host with g++ and checks them against the
distance from the coordinates for every ordered pair of distinct points of
the padded tiles of 8^3 and 16^3 blocks (P = 10, 18), of P = 8 (the smallest tile the
index form allows) and of 4^3 blocks (P = 6, where the coordinates are used directly):
every close pair must be declined.  It also bounds the
distant pairs that are declined (one-point steps that a pair could have taken).
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1811_00009_amd", "csrc", "fmm_device.hpp")

MAIN = r"""
#include <cstdio>
#include <cstdlib>
template <int P>
static int check(double *declined)
{
    const int T = P * P * P;
    long bad = 0, far = 0, dec = 0;
    for (int a = 0; a < T; ++a)
        for (int b = 0; b < T; ++b) {
            if (a == b) continue;
            const int m = abs(a % P - b % P) + abs((a / P) % P - (b / P) % P) + abs(a / (P * P) - b / (P * P));
            const bool f = far_apart<P>(a, b);
            if (m < 4) bad += f;
            else { ++far; dec += !f; }
        }
    *declined = (double)dec / (double)far;
    return (int)bad;
}
// the table: 62 distinct nonzero offsets (then zeros), and every close pair's difference
// among them
template <int P>
static int check_table(double *declined)
{
    constexpr CloseOffsets c = make_close_offsets<P>();
    int bad = 0;
    for (int l = 0; l < 64; ++l) {
        if ((l < 62) != (c.off[l] != 0)) ++bad;
        for (int k = 0; k < l; ++k) bad += l < 62 && c.off[k] == c.off[l];
    }
    const int T = P * P * P;
    long far = 0, dec = 0;
    for (int a = 0; a < T; ++a)
        for (int b = 0; b < T; ++b) {
            if (a == b) continue;
            const int m = abs(a % P - b % P) + abs((a / P) % P - (b / P) % P) + abs(a / (P * P) - b / (P * P));
            bool hit = false;
            for (int l = 0; l < 64; ++l) hit |= c.off[l] == b - a;
            if (m < 4) bad += !hit;
            else { ++far; dec += hit; }
        }
    *declined = (double)dec / (double)far;
    return bad;
}
int main()
{
    double d6, d8, d10, d18, t6, t10, t18;
    const int bad = check<6>(&d6) + check<8>(&d8) + check<10>(&d10) + check<18>(&d18);
    const int tbad = check_table<6>(&t6) + check_table<10>(&t10) + check_table<18>(&t18);
    printf("%d %.6f %.6f %.6f %.6f %d %.6f %.6f %.6f\n", bad, d6, d8, d10, d18, tbad, t6, t10, t18);
    return 0;
}
"""


def _function_text():
    src = open(HDR).read()
    m = re.search(r"template <int P>\n__device__ __forceinline__ bool far_apart\(int a, int b\)\n\{.*?\n\}\n",
                  src, re.S)
    assert m, "far_apart not found in fmm_device.hpp"
    t = m.group(0).replace("__device__ __forceinline__", "static inline")
    m2 = re.search(r"struct CloseOffsets \{.*?\n\};\ntemplate <int P>\nconstexpr CloseOffsets make_close_offsets\(\)\n\{.*?\n\}\n",
                   src, re.S)
    assert m2, "make_close_offsets not found in fmm_device.hpp"
    return "#include <cstdint>\n" + t + m2.group(0)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pair_tests_decline_every_close_pair(tmp_path):
    src = tmp_path / "far.cpp"
    exe = tmp_path / "far"
    src.write_text(_function_text() + MAIN)
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    bad, d6, d8, d10, d18, tbad, t6, t10, t18 = out.stdout.split()
    assert int(bad) == 0 and int(tbad) == 0
    # the coordinates themselves at P = 6; few distant pairs declined at the larger tiles
    assert float(d6) == 0.0
    assert float(d8) < 0.03 and float(d10) < 0.012 and float(d18) < 0.0015
    assert float(t10) < 0.012 and float(t18) < 0.0015
