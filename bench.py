#!/usr/bin/env python3
"""Benchmark: accepted grid points per second (Mpts/s) of the block-based restarted
narrow-band FMM on one MI355X.

Default workload: 1024^3 grid, h = 1/1023, speed piecewise constant on 64^3 coarse
cells with i.i.d. U[0.5, 2.0] values (seed 3), one random interior source, FP32
psi and F, 16^3 blocks, fixed stride 2h.  One step = one full solve (layout,
initialisation, every restart of the persistent kernel, copy back) with F
already resident in HBM.

Other workloads (--workload): smooth_sine_256_f32/_f64, smooth_point_64, and
batched_512 (512 solves of uneven sizes with Fourier speeds, one persistent
launch with the autotuned block size and waves per block, against 512
sequential solves).

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      HBM roofline of the dominant kernel (the persistent restart loop)
  cpu_baseline  the CPU oracle (single-heap FMM, one thread) timed on a bounded
                sample of the same workload on this host
  extra         restarts, pops, pops/s, device times, launch shape; for the
                default workload also the other configurations, each timed once
                after a warm-up: the learned stride and 8^3 blocks on the same
                field, the paper's case 1 at 1024^3 in FP64, the 64^3 and 256^3
                workloads, the 512-solve batch against 512 sequential solves, and a
                held-out 512^3 field with the learned stride against fixed ones
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "accepted grid points/sec (Mpts/s) at 256^3/1024^3; learned vs fixed stride"
HBM_PEAK_GBS = 8000.0
ALGO_BYTES_PER_POINT = {"f32": 8, "f64": 16}  # read F once, write psi once


def source_code_text(text):
    """C++ source text without its comments and with its blank space collapsed: what a
    change to the compiled kernels has to change."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(csrc=None):
    """Hash of the kernel sources (comments and blank space left out, so that editing a
    comment keeps the profiles measured on the same code valid)."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_1811_00009_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), encoding="utf-8") as f:
                h.update(name.encode())
                h.update(source_code_text(f.read()).encode())
    return h.hexdigest()[:16]


PROFILED = {"block": 16, "waves_per_block": 1, "stride_h": 2.0}  # the configuration profiled


def measured_traffic(workload, config=None):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None when
    the summary is missing, was taken on different kernel sources, or the run's launch
    configuration is not the profiled one."""
    if config is not None and any(config.get(k) != v for k, v in PROFILED.items()):
        return None
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    return float(t["hbm_bytes_per_launch"])


def build_workload(name, torch):
    import numpy as np
    from paper_1811_00009_amd import inputs
    if name == "coarse_cells_1024":
        p = inputs.coarse_cells(1024, 64, seed=(3,), materialize=False)
        return p, inputs.expand_cells_device(p.meta["V"], 1024, torch), "f32"
    if name == "smooth_sine_256_f32":
        p = inputs.smooth_sine(256, dtype=np.float32)
        return p, torch.from_numpy(p.F).cuda(), "f32"
    if name == "smooth_sine_256_f64":
        p = inputs.smooth_sine(256, dtype=np.float64)
        return p, torch.from_numpy(p.F).cuda(), "f64"
    if name == "smooth_point_64":
        p = inputs.smooth_point(64)
        return p, torch.from_numpy(p.F).cuda(), "f64"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(p, workload, seconds_target=15.0):
    """Oracle (single-heap FMM, one thread) on a box around the source cut from the same
    speed field; Mpts/s = box points / time."""
    import numpy as np
    import oracle
    from paper_1811_00009_amd import inputs
    n = p.F.shape[0] if p.F is not None else p.meta["n"]
    side = min(n, 320)  # ~15 s of one host core
    src = p.sources[0]
    lo = [min(max(int(src[a]) - side // 2, 0), n - side) for a in range(3)]
    if workload == "coarse_cells_1024":
        V = p.meta["V"]
        r = n // V.shape[0]
        ks = np.arange(lo[2], lo[2] + side) // r
        js = np.arange(lo[1], lo[1] + side) // r
        is_ = np.arange(lo[0], lo[0] + side) // r
        F = np.ascontiguousarray(V[ks][:, js][:, :, is_], dtype=np.float64)
    else:
        F = np.ascontiguousarray(p.F[lo[2]:lo[2] + side, lo[1]:lo[1] + side,
                                     lo[0]:lo[0] + side], dtype=np.float64)
    s = [(int(src[0]) - lo[0], int(src[1]) - lo[1], int(src[2]) - lo[2], 0.0)]
    t0 = time.perf_counter()
    oracle.fmm(F, p.h, s)
    dt = time.perf_counter() - t0
    pts = F.size
    base = {"value": round(pts / dt / 1e6, 4), "unit": "Mpts/s", "cores": 1, "kind": "oracle",
            "sample": f"single-heap FMM in FP64 on the {side}^3 box around the source cut from "
                      f"the same speed field ({pts} points, {dt:.1f} s, one thread)"}
    # the paper's parallel CPU solver (block method, OpenMP over the blocks) on the same box
    t0 = time.perf_counter()
    _, st = oracle.block_fmm_parallel(F, p.h, s, block=16, stride=2 * p.h, stats=True)
    dtp = time.perf_counter() - t0
    par = {"value": round(pts / dtp / 1e6, 4), "unit": "Mpts/s", "threads": st["threads"],
           "kind": "block method, OpenMP over the blocks of each step, FP64, 16^3 blocks, 2h",
           "sample": f"the same {side}^3 box ({dtp:.1f} s, {st['restarts']} restarts)"}
    return base, par


WEIGHTS = os.path.join(ROOT, "paper_1811_00009_amd", "weights", "stride_mlp_b16.f32")


def load_weights(torch):
    """Trained stride-network blob (parameters, feature mean and std) on the device, or None."""
    import numpy as np
    if not os.path.exists(WEIGHTS):
        return None
    blob = np.fromfile(WEIGHTS, dtype="<f4")
    return torch.from_numpy(blob).cuda()


def timed(fn, steps, warmup, label):
    import torch
    for w in range(warmup):
        st = fn()
        print(f"[bench] {label} warmup {w}: {st['elapsed_ms']:.1f} ms device", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        stats.append(fn())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for k, st in enumerate(stats):
        print(f"[bench] {label} step {k}: {st['elapsed_ms']:.1f} ms device, loop "
              f"{st['loop_ms']:.1f} ms, {st['restarts']} restarts, {st['pops']} pops",
              file=sys.stderr, flush=True)
    return stats, wall


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="coarse_cells_1024")
    ap.add_argument("--block", type=int, default=16)
    ap.add_argument("--waves", type=int, default=1)
    ap.add_argument("--stride-h", type=float, default=2.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned-stride and 8^3-block solves of the default workload")
    ap.add_argument("--per-problem-restarts", action="store_true",
                    help="batched_512: time the launch in which every solve restarts on its own")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 1 GiB device copy (counter calibration)")
    return ap.parse_args()


def roofline(dtype, npts, loop_ms, workload, config):
    algo_bytes = ALGO_BYTES_PER_POINT[dtype] * npts
    achieved = algo_bytes / (loop_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
            "traffic": measured_traffic(workload, config),
            "kernel": "k_persistent (restart loop)",
            "algorithmic_bytes_per_launch": algo_bytes,
            "kernel_ms": round(loop_ms, 3)}


def contract(args, value, ms_per_step, dtype, config):
    return {"metric": METRIC, "value": round(value, 3), "unit": "Mpts/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def run_single(args, torch, fmm):
    p, F, dtype = build_workload(args.workload, torch)
    nz, ny, nx = F.shape
    npts = nx * ny * nz
    stride = args.stride_h * p.h
    psi = torch.empty_like(F)
    print(f"[bench] workload {args.workload}: {nx}x{ny}x{nz} {dtype}, block {args.block}, "
          f"waves {args.waves}, stride {args.stride_h}h, source {p.sources[0][:3]}",
          file=sys.stderr, flush=True)

    def step():
        return fmm.solve(F, p.h, p.sources, block=args.block, stride=stride, out=psi,
                         with_stats=True, waves_per_block=args.waves)[1]

    stats, wall = timed(step, args.steps, args.warmup, "fixed")
    if args.copy_calibration:
        # known traffic for counter calibration: fill 1 GiB, then copy 1 GiB into a second
        # buffer (the copy reads 2^30 bytes and writes 2^30 bytes)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # sanity of the output: every point reached, zero at the source
    s0 = p.sources[0]
    assert bool(torch.isfinite(psi).all()), "unreached points in a fully connected field"
    assert float(psi[s0[2], s0[1], s0[0]]) == 0.0

    ms_per_step = wall / args.steps * 1e3
    value = npts / (ms_per_step / 1e3) / 1e6
    loop_ms = sum(s["loop_ms"] for s in stats) / len(stats)
    dev_ms = sum(s["elapsed_ms"] for s in stats) / len(stats)
    st = stats[-1]
    out = contract(args, value, ms_per_step, dtype,
                   {"workload": args.workload, "grid": [nx, ny, nz], "h": p.h,
                    "block": args.block, "waves_per_block": args.waves,
                    "stride_h": args.stride_h, "sources": [list(s[:3]) for s in p.sources],
                    "stride_mode": "fixed"})
    out["roofline"] = roofline(dtype, npts, loop_ms, args.workload, out["config"])
    out["extra"] = {"restarts": st["restarts"], "pops": st["pops"],
                    "pops_per_s": round(st["pops"] / (st["loop_ms"] / 1e3), 1),
                    "march_calls": st["march_calls"], "tile_loads": st["tile_loads"],
                    "exchange_calls": st["exchange_calls"], "device_ms": round(dev_ms, 3),
                    "loop_ms": round(loop_ms, 3), "grid": st["grid"],
                    "device_Mpts_per_s": round(npts / (dev_ms / 1e3) / 1e6, 3),
                    "kernel_hash": kernel_source_hash()}

    if args.workload == "coarse_cells_1024" and not args.no_extras:
        fixed = psi.clone()
        tol = 1e-5 * float(fixed.max())
        blob = load_weights(torch)
        if blob is not None:
            out2 = torch.empty_like(F)
            ls, lwall = timed(lambda: fmm.solve(F, p.h, p.sources, block=args.block,
                                                stride=stride, out=out2, with_stats=True,
                                                stride_mode="learned", mlp_weights=blob)[1],
                              1, 1, "learned")
            diff = float((out2 - fixed).abs().max())
            out["extra"]["learned_stride"] = {
                "Mpts_per_s": round(npts / lwall / 1e6, 3),
                "vs_fixed_2h": round((npts / lwall / 1e6) / value, 4),
                "restarts": ls[-1]["restarts"], "pops": ls[-1]["pops"],
                "final_bound": ls[-1]["final_bound"],
                "max_abs_diff_vs_fixed": diff, "within_fp32_bar": diff <= tol,
                "weights": os.path.relpath(WEIGHTS, ROOT)}
            del out2
        out8 = torch.empty_like(F)
        bs, bwall = timed(lambda: fmm.solve(F, p.h, p.sources, block=8, stride=stride, out=out8,
                                            with_stats=True)[1], 1, 1, "block8")
        diff = float((out8 - fixed).abs().max())
        out["extra"]["block8"] = {"Mpts_per_s": round(npts / bwall / 1e6, 3),
                                  "pops": bs[-1]["pops"], "grid": bs[-1]["grid"],
                                  "max_abs_diff_vs_block16": diff, "within_fp32_bar": diff <= tol}
        del out8, fixed, psi, F
        torch.cuda.empty_cache()
        out["extra"]["fp64_1024_paper_case1"] = leg_fp64_1024(torch, fmm)
        out["extra"]["small_workloads"] = leg_small(torch, fmm)
        out["extra"]["batched_512"] = leg_batched(torch, fmm)
        out["extra"]["heldout_512_learned_stride"] = leg_heldout(torch, fmm)
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["extra"]["cpu_parallel_block_solver"] = cpu_baseline(p, args.workload)
    return out


def _once(fn, label):
    """One warm-up, then one timed call on a drained device: (stats, seconds)."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] {label}: {dt * 1e3:.1f} ms, {st.get('restarts')} restarts, "
          f"{st.get('pops')} pops", file=sys.stderr, flush=True)
    return st, dt


def leg_fp64_1024(torch, fmm):
    """The paper's case 1 (F = 1, source at the centre of the cell-centred unit cube) at
    its finest grid, 1024^3, in FP64, with 16^3 and 8^3 blocks, stride 2h."""
    n = 1024
    h = 1.0 / n
    F = torch.ones((n, n, n), dtype=torch.float64, device="cuda")
    src = [(n // 2, n // 2, n // 2, 0.0)]
    res = {"grid": [n, n, n], "stride_h": 2.0, "dtype": "f64"}
    outs = {}
    for b in (16, 8):
        psi = torch.empty_like(F)
        st, dt = _once(lambda: fmm.solve(F, h, src, block=b, stride=2 * h, out=psi,
                                         with_stats=True)[1], f"fp64 1024^3 case 1 block {b}")
        res[f"block{b}"] = {"Mpts_per_s": round(n ** 3 / dt / 1e6, 3), "restarts": st["restarts"],
                            "pops": st["pops"], "loop_ms": round(st["loop_ms"], 3)}
        outs[b] = psi
    # multi-block solutions agree to rounding (Sec. 3.2): block 8 against block 16
    res["max_abs_diff_block8_vs_block16"] = float((outs[8] - outs[16]).abs().max())
    res["source_value"] = float(outs[16][n // 2, n // 2, n // 2])
    del outs, F
    torch.cuda.empty_cache()
    return res


def leg_small(torch, fmm):
    """The 64^3 point-source workload (FP64, 8^3 blocks) and the 256^3 sine workload (FP32
    and FP64, 16^3 blocks), each the mean of 5 timed solves after 2 warm-ups."""
    import numpy as np
    from paper_1811_00009_amd import inputs
    res = {}
    cases = (("point_64_f64_b8", inputs.smooth_point(64), np.float64, 8),
             ("sine_256_f32_b16", inputs.smooth_sine(256, dtype=np.float32), np.float32, 16),
             ("sine_256_f64_b16", inputs.smooth_sine(256, dtype=np.float64), np.float64, 16))
    for name, p, dt_, b in cases:
        F = torch.from_numpy(np.ascontiguousarray(p.F, dtype=dt_)).cuda()
        psi = torch.empty_like(F)
        for _ in range(2):
            fmm.solve(F, p.h, p.sources, block=b, stride=2 * p.h, out=psi)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            st = fmm.solve(F, p.h, p.sources, block=b, stride=2 * p.h, out=psi, with_stats=True)[1]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        res[name] = {"Mpts_per_s": round(F.numel() / dt / 1e6, 3), "ms": round(dt * 1e3, 3),
                     "restarts": st["restarts"], "pops": st["pops"]}
        print(f"[bench] {name}: {dt * 1e3:.2f} ms", file=sys.stderr, flush=True)
    return res


def leg_batched(torch, fmm, nsolve=512):
    """512 solves of uneven sizes in one persistent launch (block and waves from the
    autotuner) against the same solves as 512 plain launches; psi identical, and two of
    the solves against the single-heap oracle."""
    import numpy as np
    import oracle
    from paper_1811_00009_amd import inputs
    t0 = time.perf_counter()
    probs = [inputs.batched_problem_device(s, torch) for s in range(nsolve)]
    torch.cuda.synchronize()
    npts = sum(int(p.F.numel()) for p in probs)
    tune = fmm.autotune([(p.F, p.h, p.sources) for p in probs[::16]])
    B, W = tune["block"], tune["waves_per_block"]
    print(f"[bench] batched_512: {npts} points, built and tuned in {time.perf_counter() - t0:.1f} s"
          f" (block {B}, waves {W})", file=sys.stderr, flush=True)
    batch = [(p.F, p.h, p.sources) for p in probs]
    outs = [torch.empty_like(p.F) for p in probs]
    st, dt = _once(lambda: fmm.solve_batched(batch, block=B, waves_per_block=W, outs=outs,
                                             with_stats=True)[1][0], "batched_512 one launch")
    seq_out = [torch.empty_like(p.F) for p in probs]
    for p, o in zip(probs[:4], seq_out):
        fmm.solve(p.F, p.h, p.sources, block=B, waves_per_block=W, out=o)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p, o in zip(probs, seq_out):
        fmm.solve(p.F, p.h, p.sources, block=B, waves_per_block=W, out=o)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    same = all(torch.equal(a, b) for a, b in zip(outs, seq_out))
    other = _batched_other_mode(torch, fmm, batch, B, W, True, seq_out, npts)
    # two of the batch's solves against the single-heap oracle on the same speed values
    sides = [int(p.F.shape[0]) for p in probs]
    pick = sorted(range(nsolve), key=lambda s: sides[s])[:2]
    checks = []
    for s in pick:
        Fh = probs[s].F.cpu().numpy()
        ref32 = oracle.fmm(Fh, probs[s].h, probs[s].sources, dtype=np.float32)
        ref64 = oracle.fmm(Fh.astype(np.float64), probs[s].h, probs[s].sources)
        got = outs[s].cpu().numpy()
        checks.append({"solve": s, "side": sides[s],
                       "max_abs_diff_vs_fp32_oracle": float(np.max(np.abs(got - ref32))),
                       "max_abs_diff_vs_fp64_oracle": float(np.max(np.abs(got - ref64))),
                       "bar_1e-5_max_psi": float(1e-5 * ref32.max())})
    res = {"solves": nsolve, "points": npts, "block": B, "waves_per_block": W,
           "Mpts_per_s": round(npts / dt / 1e6, 3), "ms": round(dt * 1e3, 3),
           "sequential_Mpts_per_s": round(npts / seq / 1e6, 3),
           "batched_over_sequential": round(seq / dt, 3), "identical_to_sequential": same,
           "per_problem_restarts": other, "oracle_checks": checks}
    del probs, outs, seq_out, batch
    torch.cuda.empty_cache()
    return res


def leg_heldout(torch, fmm):
    """A held-out 512^3 coarse-cell field (the stride network never saw it): the learned
    stride against the fixed strides 1h, 2h and 4h (multipliers 1/2, 1, 2 of 2h)."""
    from paper_1811_00009_amd import inputs
    blob = load_weights(torch)
    if blob is None:
        return None
    n = 512
    p = inputs.stride_field((50, 0), n, materialize=False)
    F = inputs.expand_cells_device(p.meta["V"], n, torch)
    psi = torch.empty_like(F)
    res = {"field": "SeedSequence([50, 0]), 512^3, 64^3 coarse cells", "block": 16}
    fixed = {}
    for m in (0.5, 1.0, 2.0):
        st, dt = _once(lambda: fmm.solve(F, p.h, p.sources, block=16, stride=m * 2 * p.h,
                                         out=psi, with_stats=True)[1], f"heldout fixed {m}x2h")
        fixed[m] = dt
        res[f"fixed_{m}x2h_Mpts_per_s"] = round(n ** 3 / dt / 1e6, 3)
    ref = psi.clone()
    st, dt = _once(lambda: fmm.solve(F, p.h, p.sources, block=16, stride=2 * p.h, out=psi,
                                     with_stats=True, stride_mode="learned",
                                     mlp_weights=blob)[1], "heldout learned")
    best = min(fixed.values())
    res.update({"learned_Mpts_per_s": round(n ** 3 / dt / 1e6, 3),
                "learned_restarts": st["restarts"],
                "learned_over_best_fixed": round(best / dt, 4),
                "learned_over_fixed_2h": round(fixed[1.0] / dt, 4),
                "max_abs_diff_learned_vs_fixed_4h": float((psi - ref).abs().max())})
    del F, psi, ref
    torch.cuda.empty_cache()
    return res


def run_batched(args, torch, fmm):
    """512 solves of uneven sizes: one persistent launch (autotuned) vs 512 plain launches."""
    from paper_1811_00009_amd import inputs
    nsolve = 512
    t0 = time.perf_counter()
    probs = [inputs.batched_problem_device(s, torch) for s in range(nsolve)]
    torch.cuda.synchronize()
    npts = sum(int(p.F.numel()) for p in probs)
    print(f"[bench] batched_512: {nsolve} fields, {npts} points, built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    # every 16th field: a sample with enough work per restart to stand for the batch (on
    # 8 fields the grid barrier dominates and favours fewer, larger work-groups)
    tune = fmm.autotune([(p.F, p.h, p.sources) for p in probs[::16]])
    print(f"[bench] autotuned on 32 sample fields: block {tune['block']}, waves "
          f"{tune['waves_per_block']}", file=sys.stderr, flush=True)
    B, W = tune["block"], tune["waves_per_block"]
    batch = [(p.F, p.h, p.sources) for p in probs]
    outs = [torch.empty_like(p.F) for p in probs]

    pp = bool(args.per_problem_restarts)

    def step():
        per = fmm.solve_batched(batch, block=B, waves_per_block=W, outs=outs,
                                with_stats=True, per_problem_restarts=pp)[1]
        st = dict(per[0])  # times and launch shape are the launch's, the same in every row
        st["pops"] = sum(s["pops"] for s in per)
        st["restarts"] = max(s["restarts"] for s in per)
        return st

    stats, wall = timed(step, args.steps, args.warmup, "batched")
    ms_per_step = wall / args.steps * 1e3
    value = npts / (ms_per_step / 1e3) / 1e6
    loop_ms = sum(s["loop_ms"] for s in stats) / len(stats)
    # the same 512 solves as separate plain launches (same block size, default stride)
    seq_out = [torch.empty_like(p.F) for p in probs]
    for p, o in zip(probs[:4], seq_out):
        fmm.solve(p.F, p.h, p.sources, block=B, waves_per_block=W, out=o)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for p, o in zip(probs, seq_out):
        fmm.solve(p.F, p.h, p.sources, block=B, waves_per_block=W, out=o)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t1
    same = all(torch.equal(a, b) for a, b in zip(outs, seq_out))
    print(f"[bench] sequential: {seq * 1e3:.1f} ms for {nsolve} launches; identical: {same}",
          file=sys.stderr, flush=True)
    other = _batched_other_mode(torch, fmm, batch, B, W, not pp, seq_out, npts)
    out = contract(args, value, ms_per_step, "f32",
                   {"workload": "batched_512", "solves": nsolve, "points": npts,
                    "sides": "uniform over {32, 48, ..., 192}", "block": B, "waves_per_block": W,
                    "stride_h": 2.0, "stride_mode": "fixed", "per_problem_restarts": pp,
                    "tuned_on": "fields 0, 16, ..., 496"})
    out["roofline"] = roofline("f32", npts, loop_ms, "batched_512", out["config"])
    out["extra"] = {"pops": stats[-1]["pops"], "max_restarts": stats[-1]["restarts"],
                    "pops_per_s": round(stats[-1]["pops"] / (loop_ms / 1e3), 1),
                    "sequential_Mpts_per_s": round(npts / seq / 1e6, 3),
                    "batched_over_sequential": round(seq / (wall / args.steps), 3),
                    "identical_to_sequential": same, "loop_ms": round(loop_ms, 3),
                    "grid": stats[-1]["grid"], "kernel_hash": kernel_source_hash(),
                    "other_mode": other}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched()
    return out


def _batched_other_mode(torch, fmm, batch, B, W, per_problem, ref_outs, npts):
    """The same batch once more with the other restart discipline (one warm-up, one timed
    launch): all solves behind one grid barrier per step, or each solve restarting on its
    own.  psi must not change."""
    outs = [torch.empty_like(b[0]) for b in batch]
    label = "per-problem restarts" if per_problem else "shared restarts"
    st, dt = _once(lambda: fmm.solve_batched(batch, block=B, waves_per_block=W, outs=outs,
                                             with_stats=True,
                                             per_problem_restarts=per_problem)[1][0],
                   f"batched, {label}")
    same = all(torch.equal(a, b) for a, b in zip(outs, ref_outs))
    del outs
    return {"per_problem_restarts": per_problem, "Mpts_per_s": round(npts / dt / 1e6, 3),
            "ms": round(dt * 1e3, 3), "loop_ms": round(st["loop_ms"], 3),
            "identical_to_sequential": same}


def cpu_baseline_batched(seconds_target=12.0):
    """Oracle (one thread, FP64) on the batched fields in order until ~seconds_target."""
    import numpy as np
    import oracle
    from paper_1811_00009_amd import inputs
    pts, dt, k = 0, 0.0, 0
    while dt < seconds_target and k < 512:
        p = inputs.batched_problem(k, dtype=np.float64)
        t0 = time.perf_counter()
        oracle.fmm(p.F, p.h, p.sources)
        dt += time.perf_counter() - t0
        pts += p.F.size
        k += 1
    return {"value": round(pts / dt / 1e6, 4), "unit": "Mpts/s", "cores": 1, "kind": "oracle",
            "sample": f"single-heap FMM in FP64 on batched fields 0-{k - 1} ({pts} points, "
                      f"{dt:.1f} s, one thread)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus must be 1 "
              "(sharding the block grid over several GPUs is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1811_00009_amd import fmm
    fmm.load()
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(torch.device("cuda:0"))
    if args.workload == "batched_512":
        out = run_batched(args, torch, fmm)
    else:
        out = run_single(args, torch, fmm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
