"""Per-segment cycle account of one pop of the march, on the profiling build.

    python paper_1811_00009_amd/build.py --cycles      # on the build machine
    python -m paper_1811_00009_amd.cycle_account [--block 16] [--n 1024]

Runs the coarse-cell workload (n^3, 64^3 cells, seed 3, FP32, stride 2h) once on
libfmm_hip_cycles.so and prints, per pop, the shader cycles of each segment of the
march (Alg. 4 with Alg. 2-3) as a markdown table.  Each timestamp first waits for the
LDS operations in flight (the h^2/F^2 mark and the per-march marks also for device
memory), so the segments serialise what the normal build overlaps; the table gives
both the instrumented total and the cycles per pop of the run itself.
"""
import argparse
import ctypes as C
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

SEGMENTS = [
    (0, "band read (16-byte LDS read of the lane's band slots)"),
    (1, "psi gather of the slots and per-lane minimum"),
    (2, "cross-lane minimum and key (DPP, permlane swaps, ballot, readlane)"),
    (3, "bound test, neighbour tag/psi reads, Remove_Min, retag of p"),
    (4, "the six neighbour solves (Alg. 2-3), quads 0-5"),
    (5, "insert (ballot, append) and loop back"),
]
LANE0 = [
    (8, "stencil reads (tags and psi of q's six neighbours)"),
    (9, "wait for h^2/F^2 of q (device memory)"),
    (10, "quadratic root (Alg. 3) and psi/tag write"),
]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--block", type=int, default=16)
    ap.add_argument("--stride-h", type=float, default=2.0)
    args = ap.parse_args()

    import torch
    from paper_1811_00009_amd import build, fmm, inputs
    if not os.path.exists(build.CYCLES_LIB):
        raise SystemExit(f"{build.CYCLES_LIB} is missing: run build.py --cycles first")
    fmm.LIB_PATH = build.CYCLES_LIB
    lib = fmm.load()
    lib.fmm_cycle_account.argtypes = [C.POINTER(C.c_ulonglong), C.c_int]
    lib.fmm_cycle_account.restype = C.c_int
    acc = (C.c_ulonglong * 19)()

    p = inputs.coarse_cells(args.n, 64, seed=(3,), materialize=False)
    F = inputs.expand_cells_device(p.meta["V"], args.n, torch)
    print(f"[cycles] {args.n}^3 coarse cells, FP32, block {args.block}, stride {args.stride_h}h",
          file=sys.stderr, flush=True)
    assert lib.fmm_cycle_account(acc, 1) == 0
    psi, st = fmm.solve(F, p.h, p.sources, block=args.block, stride=args.stride_h * p.h,
                        with_stats=True)
    torch.cuda.synchronize()
    assert lib.fmm_cycle_account(acc, 0) == 0
    a = list(acc)
    hz = a[18]
    pops, marches, solves0 = a[12], a[13], a[11]
    print(f"[cycles] loop {st['loop_ms']:.1f} ms, {st['pops']} pops, {st['restarts']} restarts; "
          f"account: {pops} pops, {marches} marches, clock {hz / 1e9:.3f} GHz",
          file=sys.stderr, flush=True)
    per_pop = [a[k] / max(pops, 1) for k in range(16)]
    total = sum(per_pop[k] for k, _ in SEGMENTS)
    lines = ["| segment | cycles per pop | share |", "|---|---|---|"]
    for k, name in SEGMENTS:
        lines.append(f"| {k}: {name} | {per_pop[k]:.0f} | {per_pop[k] / total * 100:.1f} % |")
    lines.append(f"| **sum over a pop (instrumented)** | **{total:.0f}** | 100 % |")
    lines.append("")
    lines.append(f"Lane 0's own solves ({solves0} of {pops} pops, {solves0 / max(pops, 1):.2f} per pop):")
    lines.append("")
    lines.append("| sub-segment | cycles per lane-0 solve |")
    lines.append("|---|---|")
    for k, name in LANE0:
        lines.append(f"| {k}: {name} | {a[k] / max(solves0, 1):.0f} |")
    lines.append("")
    lines.append("Per march (tile in and out):")
    lines.append("")
    lines.append("| segment | cycles per march | cycles per pop |")
    lines.append("|---|---|---|")
    for k, name in ((6, "tile, tags and band load to LDS (+ h^2/F^2 touch)"),
                    (7, "last Locate_Min, face test, tile store, flags")):
        lines.append(f"| {k}: {name} | {a[k] / max(marches, 1):.0f} | {per_pop[k]:.0f} |")
    small, mid = a[14], a[15] - a[14]
    lines.append("")
    lines.append(f"Band size at the pick: {small / max(pops, 1) * 100:.1f} % of pops at most 64 slots, "
                 f"{mid / max(pops, 1) * 100:.1f} % 65-256, "
                 f"{(pops - a[15]) / max(pops, 1) * 100:.1f} % more than 256.")
    lines.append(f"Steps of the two-point march (band in LDS): {a[16]:,}, of which {a[17]:,} accepted two "
                 f"points; {pops:,} pops in {pops - a[17]:,} steps "
                 f"({(pops - a[17]) / max(pops, 1) * 100:.1f} % of the pops).")
    inst_pop_s = (sum(a[k] for k in range(8))) / hz / max(pops, 1)
    lines.append("")
    lines.append(f"Run: {st['pops']} pops, {marches} marches, {st['restarts']} restarts, loop "
                 f"{st['loop_ms']:.1f} ms with the marks in place; shader clock {hz / 1e9:.3f} GHz "
                 f"(s_memtime against the 100 MHz constant clock); instrumented march time per pop "
                 f"{inst_pop_s * 1e6:.3f} us.")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
