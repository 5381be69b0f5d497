"""The band load of a march (load_band_lds in fmm_device.hpp) leaves the LDS band holding the
first m entries of the block's band array and tile point 0 in every slot from m on.

The two-point step scans whole groups of slots with no bounds test, relying on the slots
at n and beyond holding tile point 0 (psi +inf); the march restores that on every
Remove_Min, and this load sets it up.  The test takes the function's own text from the
header, compiles it on the host with the ROCm clang (the 16-byte vector type is a clang
extension), runs it for every thread of a one-wave and a two-wave work-group, for every m
from 0 to the slot count, with a source array that holds garbage beyond m, and checks
every slot.
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1811_00009_amd", "csrc", "fmm_device.hpp")
CLANG = "/opt/rocm/llvm/bin/clang++"

MAIN = r"""
#include <cstdio>
#include <cstring>
template <int NT, int SLOTS>
static int check()
{
    int bad = 0;
    for (int m = 0; m <= SLOTS; ++m) {
        uint16_t src[SLOTS + 64], dst[SLOTS];
        for (int k = 0; k < SLOTS + 64; ++k) src[k] = (uint16_t)(k < m ? 1 + (k * 7919) % 65000 : 0xbeef);
        for (int k = 0; k < SLOTS; ++k) dst[k] = 0x5a5a;
        for (int tid = 0; tid < NT; ++tid)
            load_band_lds<NT, SLOTS>(reinterpret_cast<v4u *>(dst), reinterpret_cast<const v4u *>(src), m, tid);
        for (int k = 0; k < SLOTS; ++k) bad += dst[k] != (k < m ? src[k] : 0);
    }
    return bad;
}
int main()
{
    printf("%d\n", check<64, 512>() + check<64, 1024>() + check<128, 1024>());
    return 0;
}
"""


def _function_text():
    src = open(HDR).read()
    m = re.search(r"template <int NT, int SLOTS>\n__device__ __forceinline__ void load_band_lds\(.*?\n\}\n", src, re.S)
    assert m, "load_band_lds not found in fmm_device.hpp"
    body = m.group(0).replace("__device__ __forceinline__", "static inline").replace("FMM_LDS ", "")
    return ("#include <cstdint>\n"
            "typedef unsigned int v4u __attribute__((ext_vector_type(4)));\n" + body)


@pytest.mark.skipif(not os.path.exists(CLANG) and shutil.which("clang++") is None, reason="needs clang++")
def test_band_load_fills_the_tail_with_tile_point_zero(tmp_path):
    cc = CLANG if os.path.exists(CLANG) else shutil.which("clang++")
    src = tmp_path / "tail.cpp"
    exe = tmp_path / "tail"
    src.write_text(_function_text() + MAIN)
    subprocess.run([cc, "-O1", "-std=c++17", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "0"
