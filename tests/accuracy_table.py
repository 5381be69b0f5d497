"""The accuracy study of the paper's Sec. 3.2 on the GPU solver: for each of the four
point-source problems of Sec. 3.1 and each grid, the largest relative difference
psi^rd = max |psi^B - psi^M| / psi^B between the single-heap baseline solution psi^B
(the oracle, FP64) and every multi-block solution psi^M of the HIP path (FP64, block
sizes 8 and 16, strides 0.5, 1.5, 2, 2.5, 3.5 and infinitely many h), over the points
where psi^B is finite and positive.

    python tests/accuracy_table.py [--grids 128 256 512] [--blocks 8 16]

Prints a markdown table (one row per case, one column per grid) and the time the
baseline took.  The baseline solves run in worker processes started before the GPU
is touched, while the GPU solves run in the main process and stay in device memory
(48 FP64 solutions of 512^3 take 48 GB) until their baseline arrives.
"""
import argparse
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

STRIDES_H = (0.5, 1.5, 2.0, 2.5, 3.5, math.inf)


def _baseline(args):
    case, n = args
    import oracle
    from paper_1811_00009_amd import inputs
    p = inputs.paper_case(case, n)
    t0 = time.perf_counter()
    psi = oracle.fmm(p.F, p.h, p.sources)
    return case, n, psi, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--grids", type=int, nargs="+", default=[128, 256, 512])
    ap.add_argument("--blocks", type=int, nargs="+", default=[8, 16])
    ap.add_argument("--workers", type=int, default=4)
    args = ap.parse_args()
    jobs = [(c, n) for n in args.grids for c in (1, 2, 3, 4)]
    ctx = mp.get_context("spawn")
    pool = ctx.Pool(args.workers)
    pending = pool.imap_unordered(_baseline, sorted(jobs, key=lambda j: -j[1]))

    import torch
    from paper_1811_00009_amd import fmm, inputs
    fmm.load()
    gpu = {}
    for n in args.grids:
        for case in (1, 2, 3, 4):
            p = inputs.paper_case(case, n)
            F = torch.from_numpy(np.array(p.F)).cuda()
            sols = []
            for b in args.blocks:
                for sh in STRIDES_H:
                    psi, st = fmm.solve(F, p.h, p.sources, block=b, stride=sh * p.h,
                                        with_stats=True)
                    sols.append(((b, sh), psi, st["restarts"]))
            gpu[(case, n)] = sols
            print(f"[accuracy] GPU case {case} {n}^3: {len(sols)} multi-block solves", flush=True)
            del F
    rd = {}
    for case, n, base, dt in pending:
        b = torch.from_numpy(base).cuda()
        fin = torch.isfinite(b) & (b > 0)
        bf = b[fin]
        worst, at = 0.0, None
        for cfg, psi, nr in gpu[(case, n)]:
            assert torch.equal(torch.isinf(psi), torch.isinf(b)), (case, n, cfg)
            r = float(((psi[fin] - bf).abs() / bf).max())
            if r > worst:
                worst, at = r, cfg
        rd[(case, n)] = (worst, at)
        del gpu[(case, n)], b, fin, bf
        print(f"[accuracy] case {case} {n}^3: baseline {dt:.1f} s, psi^rd = {worst:.3e} "
              f"(largest at block {at[0] if at else '-'}, stride {at[1] if at else '-'}h)",
              flush=True)
    pool.close()
    pool.join()
    lines = ["| case | " + " | ".join(f"{n}^3" for n in args.grids) + " |",
             "|---|" + "---|" * len(args.grids)]
    for case in (1, 2, 3, 4):
        cells = []
        for n in args.grids:
            w, at = rd[(case, n)]
            cells.append(f"{w:.2e}")
        lines.append(f"| {case} | " + " | ".join(cells) + " |")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
