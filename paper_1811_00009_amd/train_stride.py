"""Train and evaluate the restart-stride network on the GPU.

    python -m paper_1811_00009_amd.train_stride --fields 60 --out paper_1811_00009_amd/weights

1. Labels.  The default rule ("rollout") labels restarts, not fields: for each
   training field (coarse-cell speeds, 64^3 cells, seeds (5, s), n^3 grid) a base
   solve at the fixed stride base_m * 2h is stopped at `decisions` restarts spread
   over the solve; from each stopped state (saved and restored through the
   library's workspace calls) every multiplier m in stride.MULTIPLIERS continues
   with stride m * 2h until the bound has advanced by window_h * h, and the
   restart's label is the m whose rollout made every value below that advance
   final in the least device time (stride.label_rollouts).  The older rules
   label every restart of a field with the multiplier whose whole fixed-stride
   solve was fastest ("field") or per slab of the bound ("slab"); Fourier
   (6, s) and sine (7, s) fields can be mixed into those.
2. Full-batch training with the library's forward / backward / Adam kernels.
3. Held-out evaluation on coarse-cell fields with seeds (50, s) at eval_n^3, and
   on a few unseen fields of the other families at n^3: device time of every
   fixed multiplier and of the learned stride, and psi of the learned solve
   against the fixed 2h solve (FP32 bar).

Collection can be split over several runs: --collect-only with --first-field
writes the samples of a range of fields, and --samples trains on such files.

Writes <out>/stride_mlp_b<B>.f32 (the device blob: 1505 parameters, 12 feature
means, 12 feature standard deviations, little-endian FP32) and
<out>/stride_mlp_b<B>.json (data, training and evaluation record).

    python -m paper_1811_00009_amd.train_stride --eval-only

evaluates the blob already in <out> (step 3 only) and writes
<out>/stride_mlp_b<B>.eval.json.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def log(msg):
    print(f"[train_stride] {msg}", flush=True)


def field(seed_words, n, torch):
    """(problem, device speed) of a stride-network field; the family is seed_words[0]:
    5 / 50 coarse cells, 6 Fourier, 7 sine."""
    from . import inputs
    if seed_words[0] in (5, 50):
        p = inputs.stride_field(seed_words, n, materialize=False)
        return p, inputs.expand_cells_device(p.meta["V"], n, torch)
    if seed_words[0] == 6:
        p = inputs.fourier_field_device(seed_words, n, torch)
    else:
        p = inputs.sine_field_device(seed_words, n, torch)
    return p, p.F


def collect(fmm, stride, torch, plan, n, block, rule, mults):
    """plan: [(family seed word, count)]; mults: the fixed multipliers traced."""
    Xs, ys, best, t0, k = [], [], [], time.perf_counter(), 0
    for fam, count in plan:
        for s in range(count):
            p, F = field([fam, s], n, torch)
            traces = {}
            for m in mults:
                _, st, rows = stride.trace_solve(fmm, F, p.h, p.sources, block=block,
                                                 multiplier=m)
                traces[m] = rows
            X, y = stride.label_traces(traces, rule=rule)
            Xs.append(X)
            ys.append(y)
            secs = {m: round(stride.solve_seconds(traces[m]) * 1e3, 1) for m in traces}
            best.append((fam, s, min(secs, key=secs.get)))
            if k % 5 == 0:
                log(f"field {fam}/{s}: {len(y)} samples, ms per m {secs}, "
                    f"{time.perf_counter() - t0:.0f} s")
            k += 1
            del F
    return np.concatenate(Xs), np.concatenate(ys), best


def rollout_field(fmm, stride, torch, p, F, block, mults, base_m, n_dec, window_h, extra):
    """Rollout labels of one field.  The base solve (fixed stride base_m * 2h) is stopped
    after each of n_dec decision restarts r_d; from that state (saved once, restored for
    each rollout) every multiplier m continues with stride m * 2h until the bound has
    advanced by window_h * h, then with the base stride for `extra` restarts; its cost is
    the device time until the values below bound_{r_d} + window were final.  Returns
    (X, y, C, R, costs): samples, rollout costs and decision restarts from
    stride.label_rollouts, and the costs by decision."""
    s0 = 2 * p.h
    base_stride = base_m * s0
    window = window_h * p.h
    _, st, rows = stride.trace_solve(fmm, F, p.h, p.sources, block=block, multiplier=base_m)
    R = len(rows)
    bounds = [r["bound"] for r in rows]
    decisions = sorted(set(int(round(x)) for x in np.linspace(2, max(R - 3, 2), n_dec)))
    out = torch.empty_like(F)
    cap_rows = R + int(math.ceil(window / (min(mults) * s0))) + extra + 8
    trace = torch.zeros(cap_rows * fmm.TRACE_ROW_BYTES, dtype=torch.uint8, device=F.device)
    state = None
    prev = 0
    costs = {}
    for r_d in decisions:
        if r_d >= R:
            break
        # the base solve, stopped after restart r_d
        if prev == 0:
            _, sb = fmm.solve(F, p.h, p.sources, block=block, stride=base_stride, out=out,
                              with_stats=True, max_restarts=r_d, stop_at_cap=True)
        else:
            fmm.workspace_restore(state)
            _, sb = fmm.solve_resume(F, p.h, p.sources, prev, block=block, stride=base_stride,
                                     out=out, with_stats=True, max_restarts=r_d,
                                     stop_at_cap=True)
        if not sb.get("stopped_at_cap"):
            break  # the solve ended before r_d
        state = fmm.workspace_save(state)
        costs[r_d] = {}
        for m in mults:
            fmm.workspace_restore(state)
            sched = stride.rollout_bounds(bounds, r_d, m, s0, window)
            fmm.solve_resume(F, p.h, p.sources, r_d, block=block, stride=base_stride, out=out,
                             stride_mode="schedule", bounds=sched, trace=trace,
                             max_restarts=len(sched) + extra, stop_at_cap=True)
            torch.cuda.synchronize()
            rws = fmm.trace_rows(trace, min(len(sched) + extra, cap_rows))
            last = max(i for i in range(len(rws)) if rws[i]["t_end"] > 0)
            costs[r_d][m] = stride.window_seconds(rws[:last + 1], r_d, bounds[r_d - 1] + window)
            trace.zero_()
        prev = r_d
    X, y, C, R = stride.label_rollouts(rows, costs, mults)
    return X, y, C, R, costs


def collect_rollouts(fmm, stride, torch, fields, n, block, mults, base_m, n_dec, window_h,
                     extra, first_seed=0):
    """Rollout-labelled samples of coarse-cell training fields (seeds (5, s)): features,
    targets, each sample's rollout costs (seconds, in the order of mults), its decision
    restart and its field seed, and the histogram of the picked multipliers."""
    Xs, ys, Cs, Rs, Ss, picks, t0 = [], [], [], [], [], [], time.perf_counter()
    for k, s in enumerate(range(first_seed, first_seed + fields)):
        p, F = field([5, s], n, torch)
        X, y, C, R, costs = rollout_field(fmm, stride, torch, p, F, block, mults, base_m,
                                          n_dec, window_h, extra)
        Xs.append(X)
        ys.append(y)
        Cs.append(C)
        Rs.append(R)
        Ss.append(np.full(len(y), s, dtype=np.int32))
        picks.extend(round(math.exp(v), 4) for v in y)
        if k % 10 == 0:
            show = {r: min(c, key=c.get) for r, c in costs.items()}
            log(f"field 5/{s}: {len(y)} decisions, picks {show}, "
                f"{time.perf_counter() - t0:.0f} s")
        del F
    hist = {}
    for m in picks:
        hist[m] = hist.get(m, 0) + 1
    return (np.concatenate(Xs), np.concatenate(ys), hist,
            {"C": np.concatenate(Cs), "R": np.concatenate(Rs), "S": np.concatenate(Ss)})


def evaluate(fmm, stride, torch, blob_dev, seeds, n, block, mults=None):
    """Device time of every fixed multiplier (mults, default stride.MULTIPLIERS; 1.0, the
    fixed 2h, among them) and of the learned stride on the held-out fields `seeds` (seed
    words); psi of the learned solve against the fixed 2h solve."""
    mults = tuple(mults or stride.MULTIPLIERS)
    res = []
    for sw in seeds:
        p, F = field(sw, n, torch)
        out = torch.empty_like(F)
        row = {"seed": list(sw), "source": list(p.sources[0][:3]), "fixed_ms": {}}
        fmm.solve(F, p.h, p.sources, block=block, out=out)  # warm-up
        for m in mults:
            _, st = fmm.solve(F, p.h, p.sources, block=block, stride=m * 2 * p.h, out=out,
                              with_stats=True)
            row["fixed_ms"][str(m)] = st["elapsed_ms"]
            if m == 1.0:
                ref = out.clone()
        _, st = fmm.solve(F, p.h, p.sources, block=block, stride=2 * p.h, out=out,
                          with_stats=True, stride_mode="learned", mlp_weights=blob_dev)
        row["learned_ms"] = st["elapsed_ms"]
        row["learned_restarts"] = st["restarts"]
        row["learned_pops"] = st["pops"]
        row["learned_final_bound"] = st["final_bound"]
        d = float((out - ref).abs().max())
        row["max_abs_diff_learned_vs_fixed_2h"] = d
        row["within_fp32_bar_vs_fixed"] = d <= 1e-5 * float(ref.max())
        res.append(row)
        log(f"eval field {sw} at {n}^3: fixed {row['fixed_ms']} learned "
            f"{row['learned_ms']:.1f} ms")
        del F, out, ref
    tot = {m: sum(r["fixed_ms"][str(m)] for r in res) for m in mults}
    best_m = min(tot, key=tot.get)
    learned = sum(r["learned_ms"] for r in res)
    pts = len(res) * n ** 3
    return {"n": n, "fields": res, "total_ms_fixed": {str(m): tot[m] for m in tot},
            "best_fixed_multiplier": best_m, "total_ms_learned": learned,
            "speedup_vs_fixed_2h": tot[1.0] / learned,
            "speedup_vs_best_fixed": tot[best_m] / learned,
            "Mpts_per_s_learned": pts / (learned / 1e3) / 1e6,
            "Mpts_per_s_fixed_2h": pts / (tot[1.0] / 1e3) / 1e6,
            "Mpts_per_s_best_fixed": pts / (tot[best_m] / 1e3) / 1e6}


def run_evals(fmm, stride, torch, blob_dev, args):
    """Step 4: held-out coarse-cell fields at eval_n^3, unseen fields of the other
    families at n^3."""
    evals = {"coarse_cells_held_out": evaluate(
        fmm, stride, torch, blob_dev, [[50, s] for s in range(args.eval_fields)], args.eval_n,
        args.block, args.multipliers)}
    # unseen fields of the other families (seeds beyond the training range)
    for name, fam in (("fourier_unseen", 6), ("sine_unseen", 7)):
        if args.other_eval_fields <= 0:
            continue
        evals[name] = evaluate(fmm, stride, torch, blob_dev,
                               [[fam, 1000 + s] for s in range(args.other_eval_fields)],
                               args.n, args.block, args.multipliers)
    for name, ev in evals.items():
        log(f"{name}: learned {ev['Mpts_per_s_learned']:.1f} Mpts/s, fixed 2h "
            f"{ev['Mpts_per_s_fixed_2h']:.1f}, best fixed (m={ev['best_fixed_multiplier']}) "
            f"{ev['Mpts_per_s_best_fixed']:.1f}")
    return evals


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--fields", type=int, default=60, help="coarse-cell training fields")
    ap.add_argument("--first-field", type=int, default=0,
                    help="rollout rule: seed of the first training field (5, s)")
    ap.add_argument("--collect-only", action="store_true",
                    help="rollout rule: write the samples of fields [first, first + fields) "
                         "to <out>/stride_samples_b<B>_<first>_<last>.npz and stop")
    ap.add_argument("--samples", nargs="+", default=None,
                    help="train on these sample files (from --collect-only) instead of "
                         "collecting")
    ap.add_argument("--label-tol", type=float, default=0.0,
                    help="with --samples: relabel every sample with the largest multiplier "
                         "whose rollout cost is within (1 + tol) of the least "
                         "(stride.pick_multiplier); files without costs are left out")
    ap.add_argument("--fourier-fields", type=int, default=0)
    ap.add_argument("--sine-fields", type=int, default=0)
    ap.add_argument("--rule", default="rollout", choices=("rollout", "field", "slab"))
    ap.add_argument("--base-multiplier", type=float, default=0.5,
                    help="rollout rule: the fixed multiplier of the base solve")
    ap.add_argument("--decisions", type=int, default=8,
                    help="rollout rule: decision restarts per field")
    ap.add_argument("--window-h", type=float, default=16.0,
                    help="rollout rule: bound advance of a rollout, in h")
    ap.add_argument("--extra", type=int, default=16,
                    help="rollout rule: base-stride restarts after the window")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--block", type=int, default=16)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--eval-fields", type=int, default=8)
    ap.add_argument("--eval-n", type=int, default=512)
    ap.add_argument("--other-eval-fields", type=int, default=2)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "weights"))
    ap.add_argument("--eval-only", action="store_true",
                    help="evaluate the blob already in --out instead of training one")
    ap.add_argument("--multipliers", default=None,
                    help="comma-separated fixed multipliers to trace and compare (1.0 among "
                         "them); default: stride.MULTIPLIERS")
    args = ap.parse_args(argv)

    import torch
    from . import fmm, stride
    args.multipliers = (tuple(float(m) for m in args.multipliers.split(","))
                        if args.multipliers else tuple(stride.MULTIPLIERS))
    if 1.0 not in args.multipliers:
        raise SystemExit("--multipliers must include 1.0 (the fixed 2h)")
    fmm.load()
    if not torch.cuda.is_available():
        raise SystemExit("train_stride needs a GPU")
    if args.eval_only:
        path = os.path.join(args.out, f"stride_mlp_b{args.block}.f32")
        blob = np.fromfile(path, dtype="<f4")
        if blob.size != 1505 + 24 or not np.all(np.isfinite(blob)):
            raise SystemExit(f"{path}: not a stride network blob")
        evals = run_evals(fmm, stride, torch, torch.from_numpy(blob).cuda(), args)
        with open(os.path.join(args.out, f"stride_mlp_b{args.block}.eval.json"), "w") as f:
            json.dump({"blob": os.path.basename(path), "eval": evals}, f, indent=1)
        return
    t0 = time.perf_counter()
    os.makedirs(args.out, exist_ok=True)
    if args.samples:
        parts = [np.load(f) for f in args.samples]
        if args.label_tol > 0:
            kept = [q for q in parts if "C" in q.files]
            if len(kept) < len(parts):
                log(f"{len(parts) - len(kept)} sample files without rollout costs left out")
            parts = kept
            for q in parts:
                if list(q["multipliers"]) != list(args.multipliers):
                    raise SystemExit("sample files were collected with other multipliers")
        X = np.concatenate([q["X"] for q in parts])
        if args.label_tol > 0:
            y = np.concatenate([[math.log(stride.pick_multiplier(dict(zip(args.multipliers, c)),
                                                                 args.label_tol))
                                 for c in q["C"]] for q in parts]).astype(np.float32)
        else:
            y = np.concatenate([q["y"] for q in parts])
        args.fields = int(sum(int(q["fields"]) for q in parts))
        picks = {}
        for v in y:
            m = round(math.exp(float(v)), 4)
            picks[m] = picks.get(m, 0) + 1
        hist = {"5": picks}
        log(f"{len(y)} samples of {args.fields} fields from {len(parts)} files; picks {picks}")
    elif args.rule == "rollout":
        X, y, picks, meta = collect_rollouts(fmm, stride, torch, args.fields, args.n,
                                             args.block, args.multipliers,
                                             args.base_multiplier, args.decisions,
                                             args.window_h, args.extra,
                                             first_seed=args.first_field)
        hist = {"5": picks}
        log(f"{len(y)} samples in {time.perf_counter() - t0:.0f} s; rollout picks {picks}")
        if args.collect_only:
            last = args.first_field + args.fields
            path = os.path.join(args.out, f"stride_samples_b{args.block}_{args.first_field}_{last}.npz")
            np.savez(path, X=X, y=y, C=meta["C"], R=meta["R"], S=meta["S"],
                     multipliers=np.array(args.multipliers), fields=args.fields,
                     first=args.first_field, n=args.n, base_multiplier=args.base_multiplier,
                     decisions=args.decisions, window_h=args.window_h, extra=args.extra)
            log(f"wrote {path}")
            return
    else:
        plan = [(5, args.fields), (6, args.fourier_fields), (7, args.sine_fields)]
        X, y, best = collect(fmm, stride, torch, plan, args.n, args.block, args.rule,
                             args.multipliers)
        hist = {}
        for fam, _, m in best:
            hist.setdefault(fam, {}).setdefault(m, 0)
            hist[fam][m] += 1
        log(f"{len(y)} samples in {time.perf_counter() - t0:.0f} s; fastest multiplier per "
            f"family {hist}")
    if not args.samples:
        np.savez(os.path.join(args.out, f"stride_samples_b{args.block}.npz"), X=X, y=y)
    blob, params, lh = stride.train(fmm, X, y, steps=args.steps, lr=args.lr)
    log(f"loss {lh[0]:.4f} -> {lh[-1]:.4f} after {args.steps} steps")
    path = os.path.join(args.out, f"stride_mlp_b{args.block}.f32")
    blob.astype("<f4").tofile(path)
    blob_dev = torch.from_numpy(blob.astype(np.float32)).cuda()
    evals = run_evals(fmm, stride, torch, blob_dev, args)
    rec = {"blob": os.path.basename(path), "layout": "1505 params (W1 32x12, b1, W2 32x32, b2, "
           "W3 1x32, b3), 12 feature means, 12 feature stds; FP32 little-endian",
           "train": {"fields": {"coarse_cells (5, s)": args.fields,
                                "fourier (6, s)": args.fourier_fields,
                                "sine (7, s)": args.sine_fields},
                     "n": args.n, "rule": args.rule, "label_tol": args.label_tol,
                     "sample_files": [os.path.basename(f) for f in (args.samples or [])],
                     "fastest_multiplier_per_family": hist,
                     "rollout": {"base_multiplier": args.base_multiplier,
                                 "decisions_per_field": args.decisions,
                                 "window_h": args.window_h, "extra_restarts": args.extra},
                     "block": args.block, "multipliers": list(args.multipliers),
                     "samples": int(len(y)), "steps": args.steps, "lr": args.lr,
                     "loss_first": float(lh[0]), "loss_last": float(lh[-1])},
           "eval": evals}
    with open(os.path.join(args.out, f"stride_mlp_b{args.block}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    log(f"wrote {path}")


if __name__ == "__main__":
    main()
