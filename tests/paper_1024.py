"""The paper's four test cases of Sec. 3.1 at its finest grid (cell-centred 1024^3, centre
source, FP64) on the GPU solver: for each case the device time of one solve (after one
warm-up solve of the same problem) at 16^3 blocks and stride 2h, at 8^3 blocks and 2h,
and at 8^3 blocks and 1.5h, with the restart counts, and the largest difference between
the 16^3 and the 8^3 solves at 2h (parity against the references at this size is the
business of the full-size and paper-scale tests; every solve is bitwise the block
reference for its own block size and stride, which the parity tests check).

    python tests/paper_1024.py [--n 1024]

Prints one line per solve and a markdown table: "s, Mpts/s (restarts)" per setting.
"""
import argparse
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

SETTINGS = ((16, 2.0), (8, 2.0), (8, 1.5))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    args = ap.parse_args()
    import torch
    from paper_1811_00009_amd import fmm, inputs
    fmm.load()
    npts = args.n ** 3
    rows = {}
    for case in (1, 2, 3, 4):
        print(f"[paper1024] case {case}: building F", flush=True)
        prob = inputs.paper_case(case, args.n)
        h, sources = prob.h, prob.sources
        F = torch.from_numpy(np.asarray(prob.F, dtype=np.float64)).cuda()
        del prob  # the host copy of F (8 GB at 1024^3)
        outs = {}
        for b, sh in SETTINGS:
            fmm.solve(F, h, sources, block=b, stride=sh * h)  # warm-up
            psi, st = fmm.solve(F, h, sources, block=b, stride=sh * h, with_stats=True)
            torch.cuda.synchronize()
            ms = st["elapsed_ms"]
            rows[(case, b, sh)] = (ms, npts / (ms / 1e3) / 1e6, st["restarts"])
            print(f"[paper1024] case {case}, block {b}, {sh}h: {ms:.0f} ms, "
                  f"{rows[(case, b, sh)][1]:.0f} Mpts/s, {st['restarts']} restarts", flush=True)
            if sh == 2.0:
                outs[b] = psi
            else:
                del psi
        fin = torch.isfinite(outs[16])
        d = float((outs[16][fin] - outs[8][fin]).abs().max())
        same_inf = bool(torch.equal(torch.isinf(outs[16]), torch.isinf(outs[8])))
        rows[(case, "diff")] = (d, same_inf)
        print(f"[paper1024] case {case}: max |psi(16^3) - psi(8^3)| at 2h = {d:.3e}, "
              f"unreached points the same: {same_inf}", flush=True)
        del outs, F, fin
        torch.cuda.empty_cache()
    lines = ["| case | B=16, 2h | B=8, 2h | B=8, 1.5h | max abs diff 16³ vs 8³ |", "|---|---|---|---|---|"]
    for case in (1, 2, 3, 4):
        cells = [f"{rows[(case, b, sh)][0] / 1e3:.2f} s, {rows[(case, b, sh)][1]:.0f} ({rows[(case, b, sh)][2]})"
                 for b, sh in SETTINGS]
        lines.append(f"| {case} | " + " | ".join(cells) + f" | {rows[(case, 'diff')][0]:.1e} |")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
