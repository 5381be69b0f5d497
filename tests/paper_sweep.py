"""The stride sweep of the paper's Sec. 3.4-3.6 on the GPU solver: for each of the four
point-source problems of Sec. 3.1 at one grid size, every block size and restart stride,
the restart count and the device time of one solve (FP64, after one warm-up solve of the
same problem), and psi against the solve with the smallest stride (they must agree to
the FP64 bar, 1e-12 max psi; every solve is bitwise the block reference for its own
block size and stride, which the parity tests check).

    python tests/paper_sweep.py [--n 256] [--blocks 8 16 32]

Prints a markdown table per block size: one row per case, "restarts / ms" per stride.
"""
import argparse
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

STRIDES_H = (0.5, 1.5, 2.0, 2.5, 3.5, math.inf)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--blocks", type=int, nargs="+", default=[8, 16, 32])
    args = ap.parse_args()
    import torch
    from paper_1811_00009_amd import fmm, inputs
    fmm.load()
    cells = {}
    for case in (1, 2, 3, 4):
        p = inputs.paper_case(case, args.n)
        F = torch.from_numpy(np.array(p.F)).cuda()
        for b in args.blocks:
            ref = None
            fmm.solve(F, p.h, p.sources, block=b, stride=2 * p.h)  # warm-up
            for sh in STRIDES_H:
                psi, st = fmm.solve(F, p.h, p.sources, block=b, stride=sh * p.h, with_stats=True)
                torch.cuda.synchronize()
                if ref is None:
                    ref = psi.clone()
                fin = torch.isfinite(ref)
                d = float((psi[fin] - ref[fin]).abs().max())
                assert d <= 1e-12 * float(ref[fin].max()), (case, b, sh, d)
                assert torch.equal(torch.isinf(psi), torch.isinf(ref)), (case, b, sh)
                cells[(case, b, sh)] = (st["restarts"], st["elapsed_ms"])
                del psi
            print(f"[sweep] case {case}, block {b}: "
                  + ", ".join(f"{sh}h {cells[(case, b, sh)][0]} / {cells[(case, b, sh)][1]:.0f} ms"
                              for sh in STRIDES_H), flush=True)
            del ref
        del F
    heads = ["∞" if math.isinf(sh) else f"{sh:g}h" for sh in STRIDES_H]
    lines = [f"| case | B | " + " | ".join(heads) + " |", "|---|---|" + "---|" * len(heads)]
    for case in (1, 2, 3, 4):
        for b in args.blocks:
            row = [f"{cells[(case, b, sh)][0]} / {cells[(case, b, sh)][1]:.0f}" for sh in STRIDES_H]
            lines.append(f"| {case} | {b} | " + " | ".join(row) + " |")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
