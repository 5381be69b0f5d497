"""The two-point step's pick of the band's two smallest (psi, key) entries (fmm_device.hpp).

- lane_top2_f32, the per-lane top-2 network on 64-bit keys (value bits above the key),
  compiled on the host from the header's own text, returns the two smallest (value, key)
  pairs of 1, 2, 4 and 8 slots, compared with a sort, on random values with many ties
  and +inf.
- The cross-lane merge schedule of wave_top2_u32 (quad swaps, half-row and row mirrors,
  then the 16- and 32-lane swaps) combines disjoint sets of lanes at every stage, which a
  top-2 merge needs (merging a lane's pair with a copy of itself would count its first
  value twice): a model of the schedule over 64 lanes, with the merge rule written as in
  top2_merge_u32, leaves the two smallest values of all lanes' pairs in every lane.  The
  model states the lane mapping of each stage; the GPU parity tests check the hardware.
"""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HDR = os.path.join(os.path.dirname(HERE), "paper_1811_00009_amd", "csrc", "fmm_device.hpp")

MAIN = r"""
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <algorithm>
#include <utility>
#include <vector>
template <int S>
static int check(unsigned seed)
{
    srand(seed);
    int bad = 0;
    for (int t = 0; t < 20000; ++t) {
        float vs[S];
        uint32_t ks[S];
        std::vector<std::pair<uint32_t, uint32_t>> all;
        for (int j = 0; j < S; ++j) {
            const int r = rand() % 10;
            vs[j] = r == 0 ? INFINITY : (float)(rand() % 4) * 0.25f;  // ties and +inf
            ks[j] = ((uint32_t)(rand() % 5832) << 16) | (uint32_t)(8 * (rand() % 64) + j);
            all.push_back({__float_as_uint(vs[j]), ks[j]});
        }
        std::sort(all.begin(), all.end());
        uint64_t x1, x2;
        lane_top2_f32<S>(vs, ks, x1, x2);
        const uint64_t e1 = ((uint64_t)all[0].first << 32) | all[0].second;
        const uint64_t e2 = S > 1 ? (((uint64_t)all[1].first << 32) | all[1].second) : ~0ull;
        bad += x1 != e1 || x2 != e2;
    }
    return bad;
}
int main()
{
    printf("%d\n", check<1>(1) + check<2>(2) + check<4>(3) + check<8>(4));
    return 0;
}
"""


def _function_text():
    src = open(HDR).read()
    parts = []
    for pat in (r"__device__ __forceinline__ void sort2_u64\(.*?\n\}\n",
                r"__device__ __forceinline__ void merge_top2_u64\(.*?\n\}\n",
                r"template <int S>\n__device__ __forceinline__ void lane_top2_f32\(.*?\n\}\n"):
        m = re.search(pat, src, re.S)
        assert m, pat
        parts.append(m.group(0).replace("__device__ __forceinline__", "static inline"))
    return ("#include <cstdint>\n#include <cstring>\n"
            "static inline uint32_t __float_as_uint(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }\n"
            + "".join(parts))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_lane_top2_network_matches_a_sort(tmp_path):
    src = tmp_path / "top2.cpp"
    exe = tmp_path / "top2"
    src.write_text(_function_text() + MAIN)
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "0"


def _merge(a1, a2, b1, b2):
    # top2_merge_u32: first = min(a1, b1), second = min(max(a1, b1), min(a2, b2))
    return np.minimum(a1, b1), np.minimum(np.maximum(a1, b1), np.minimum(a2, b2))


def _stages():
    lane = np.arange(64)
    q = lane & 3
    base = lane & ~3
    yield base + np.array([1, 0, 3, 2])[q]               # quad_perm [1,0,3,2]
    yield base + np.array([2, 3, 0, 1])[q]               # quad_perm [2,3,0,1]
    yield (lane & ~7) + (7 - (lane & 7))                 # row_half_mirror
    yield (lane & ~15) + (15 - (lane & 15))              # row_mirror
    yield lane ^ 16                                      # permlane16_swap: rows 0<->1, 2<->3
    yield lane ^ 32                                      # permlane32_swap: halves


def test_cross_lane_top2_schedule_merges_disjoint_lanes():
    rng = np.random.default_rng(7)
    for _ in range(2000):
        v = rng.integers(0, 40, size=(64, 2)).astype(np.int64)
        v.sort(axis=1)  # each lane's (first, second)
        a1, a2 = v[:, 0].copy(), v[:, 1].copy()
        sets = [{i} for i in range(64)]  # which lanes' pairs each lane has merged
        for partner in _stages():
            assert all(sets[i].isdisjoint(sets[partner[i]]) for i in range(64))
            sets = [sets[i] | sets[partner[i]] for i in range(64)]
            a1, a2 = _merge(a1, a2, a1[partner], a2[partner])
        assert all(len(s) == 64 for s in sets)
        allv = np.sort(v.ravel())
        assert (a1 == allv[0]).all() and (a2 == allv[1]).all()
