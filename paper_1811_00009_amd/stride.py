"""Learned restart stride: traces, labels, training driver and weight blobs.

The paper leaves the stride a free parameter and finds about 2h a good fixed
choice (Sec. 3.5-3.6); smaller strides favour coarse grids with fast-varying
speed, larger ones favour simple fronts.  Here a 12-32-32-1 network evaluated on
the device at the end of every restart picks the next stride as m * stride0,
m in [1/4, 8].  Any bound sequence reaches the same solution (the stride only
schedules the restarts), so the network trades time, never accuracy.

Data flow (all GPU work through the library's C ABI):
  1. trace plain solves with fixed multipliers m in MULTIPLIERS: every restart
     records its raw features, bound and device time;
  2. label: per field, m* = the multiplier whose solve took the least device
     time, the target ln m* of every trace row of that field (a per-slab rule,
     the slab of values made final fastest, is kept for analysis);
  3. standardise the features (training-set mean and std) and fit the network
     with the library's forward / backward / Adam kernels (full batch);
  4. pack the parameters and the standardisation into the device blob that
     fmm_options.mlp_weights points to.
"""
from __future__ import annotations

import math
from typing import List, Sequence

import numpy as np

NFEAT = 12
NPARAMS = 1505
MULTIPLIERS = (0.25, 0.5, 1.0, 2.0, 4.0, 8.0)
LOG_MIN, LOG_MAX = math.log(0.25), math.log(8.0)
TICKS_PER_S = 1.0e8  # device wall clock


def init_params(seed: int = 0) -> np.ndarray:
    """He-initialised parameters, output bias 0 (m = sqrt(1/4 * 8) = 1.41 at start)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2.0 / 12), size=(32, 12))
    W2 = rng.normal(0, math.sqrt(2.0 / 32), size=(32, 32))
    W3 = rng.normal(0, math.sqrt(1.0 / 32), size=(1, 32))
    parts = [W1.ravel(), np.zeros(32), W2.ravel(), np.zeros(32), W3.ravel(), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def pack_blob(params: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    p = np.asarray(params, dtype=np.float32).ravel()
    assert p.size == NPARAMS
    return np.concatenate([p, np.asarray(mean, np.float32), np.asarray(std, np.float32)])


def trace_solve(fmm, F, h, sources, block=16, stride0=None, multiplier=1.0, rows=20000,
                blob=None):
    """One traced solve; returns (psi, stats, trace rows)."""
    import torch
    stride0 = 2.0 * h if stride0 is None else stride0
    trace = torch.zeros(rows * fmm.TRACE_ROW_BYTES, dtype=torch.uint8, device=F.device)
    kw = {}
    if blob is not None:
        kw = dict(stride_mode="learned", mlp_weights=blob)
        stride = stride0
    else:
        stride = multiplier * stride0
    psi, st = fmm.solve(F, h, sources, block=block, stride=stride, with_stats=True, trace=trace,
                        **kw)
    torch.cuda.synchronize()
    n = min(st["restarts"], rows)
    return psi, st, fmm.trace_rows(trace, n)


def finality_times(rows, edges):
    """Device seconds from the start of the solve until no later restart accepts a value at
    or below each edge: the time at which the solution below the edge is final (later
    restarts of the block method can still correct values below the current bound)."""
    t0 = rows[0]["t_start"]
    T = np.zeros(len(edges))
    for r in rows:
        mp = r.get("min_popped", math.inf)
        if math.isfinite(mp):
            T = np.where(edges >= mp, np.maximum(T, (r["t_end"] - t0) / TICKS_PER_S), T)
    return T


def solve_seconds(rows):
    """Device seconds of a traced solve (first restart start to last restart end)."""
    return (rows[-1]["t_end"] - rows[0]["t_start"]) / TICKS_PER_S


def label_traces(traces_by_m: dict, rule: str = "field", nbins: int = 12, window: int = 1):
    """traces_by_m: {m: rows} for one field.  Returns (X, y): the raw features of every
    restart that chose a next stride, and the target ln m*.

    rule "field": m* is the multiplier whose whole solve took the least device time (every
    restart of the field gets it).  rule "slab": the values [0, top] are cut into nbins
    slabs (top = the largest value any restart accepted first); the cost of m on slab k is
    the time its solve took to make slabs k-window .. k+window final (finality_times), and
    the restarts whose bound lies in slab k get the cheapest m."""
    ms = sorted(m for m, rows in traces_by_m.items() if rows)
    if rule == "field":
        best_m = min(ms, key=lambda m: solve_seconds(traces_by_m[m]))
        label = lambda r: best_m  # noqa: E731
    elif rule == "slab":
        tops = [r.get("min_popped", math.inf) for m in ms for r in traces_by_m[m]]
        top = max(v for v in tops if math.isfinite(v))
        edges = np.linspace(0.0, top * (1 + 1e-9), nbins + 1)
        fin = {m: finality_times(traces_by_m[m], edges) for m in ms}
        best = []
        for k in range(nbins):
            lo, hi = max(k - window, 0), min(k + window + 1, nbins)
            best.append(ms[int(np.argmin([fin[m][hi] - fin[m][lo] for m in ms]))])

        def label(r):
            b = int(np.clip(np.searchsorted(edges, r["bound"], side="right") - 1, 0, nbins - 1))
            return best[b]
    else:
        raise ValueError(rule)
    X, y = [], []
    for m in ms:
        for r in traces_by_m[m]:
            if r["next_active"] == 0:
                continue  # the last restart has no next stride to choose
            X.append(r["feat"])
            y.append(math.log(label(r)))
    return np.array(X, dtype=np.float32).reshape(-1, NFEAT), np.array(y, dtype=np.float32)


def rollout_bounds(base_bounds: Sequence[float], r_d: int, m: float, s0: float,
                   window: float) -> List[float]:
    """Bound schedule of a rollout from decision restart r_d: the base solve's bounds of
    restarts 1 .. r_d (the state after restart r_d is then the base solve's, bit for bit),
    then a stride of m * s0 until the bound reaches bound_{r_d} + window."""
    sched = [float(b) for b in base_bounds[:r_d]]
    b0 = sched[-1]
    j = 1
    while True:
        b = b0 + j * m * s0
        sched.append(b)
        if b >= b0 + window:
            break
        j += 1
    return sched


def window_seconds(rows, r_d: int, edge: float) -> float:
    """Device seconds from the start of restart r_d + 1 until the end of the last later
    restart that accepted a value at or below edge: the time the rollout took to make the
    values below edge final."""
    t0 = rows[r_d]["t_start"]
    t_last = t0
    for r in rows[r_d:]:
        if r.get("min_popped", math.inf) <= edge:
            t_last = max(t_last, r["t_end"])
    return (t_last - t0) / TICKS_PER_S


def pick_multiplier(costs: dict, tol: float = 0.0) -> float:
    """The label of one decision: the multiplier of least cost, or with tol > 0 the
    largest multiplier whose cost is within (1 + tol) of the least (fewer restarts among
    rollouts that the timing cannot tell apart)."""
    c_min = min(costs.values())
    return max(m for m, c in costs.items() if c <= (1.0 + tol) * c_min)


def label_rollouts(base_rows, costs_by_decision: dict, mults: Sequence[float] = None,
                   tol: float = 0.0):
    """Samples of the rollout rule.  costs_by_decision: {r_d: {m: seconds}}; the sample of
    decision r_d is the base solve's features at the end of restart r_d, and its target is
    ln of the multiplier whose rollout made the next window of values final fastest
    (pick_multiplier).  Returns (X, y, C, R): C holds each sample's costs in the order of
    mults (default: sorted multipliers of the first decision), R its decision restart."""
    X, y, C, R = [], [], [], []
    for r_d in sorted(costs_by_decision):
        costs = costs_by_decision[r_d]
        if not costs:
            continue
        if mults is None:
            mults = sorted(costs)
        X.append(base_rows[r_d - 1]["feat"])
        y.append(math.log(pick_multiplier(costs, tol)))
        C.append([costs.get(m, math.inf) for m in mults])
        R.append(r_d)
    nm = len(mults) if mults is not None else 0
    return (np.array(X, dtype=np.float32).reshape(-1, NFEAT), np.array(y, dtype=np.float32),
            np.array(C, dtype=np.float64).reshape(-1, nm), np.array(R, dtype=np.int32))


def standardise(X: np.ndarray):
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    return mean.astype(np.float32), std.astype(np.float32)


def train(fmm, X: np.ndarray, y: np.ndarray, steps: int = 2000, lr: float = 3e-3, seed: int = 0):
    """Fit on the GPU with the library's kernels.  Returns (blob, params, loss history)."""
    import torch
    mean, std = standardise(X)
    Xs = ((X - mean) / std).astype(np.float32)
    params = torch.from_numpy(init_params(seed)).cuda()
    xd = torch.from_numpy(np.ascontiguousarray(Xs)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    hist = torch.zeros(steps, dtype=torch.float32, device="cuda")
    fmm.mlp_train(params, xd, yd, steps, lr, hist)
    p = params.cpu().numpy()
    return pack_blob(p, mean, std), p, hist.cpu().numpy()
