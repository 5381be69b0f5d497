"""Learned restart stride and the network's kernels, through the C ABI.

* forward / loss-gradient / Adam kernels (FP32) against the FP64 CPU reference;
* a learned-stride solve is bitwise the Alg. 6 block reference replaying the
  bound sequence the device chose (read back from the trace), and within the
  FP64 tolerance of the single-heap baseline;
* the multiplier the device applied equals the network evaluated on the host
  (FP64 reference) on the features the device recorded;
* fallback to the fixed stride when the weights are absent or not finite.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1811_00009_amd import inputs, stride as stride_mod

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_mlp_forward_matches_cpu_reference(fmm_lib):
    rng = np.random.default_rng(1)
    P = rng.normal(0, 0.3, size=1505).astype(np.float32)
    X = rng.normal(0, 1, size=(1000, 12)).astype(np.float32)
    y = fmm_lib.mlp_forward(_t(P), _t(X)).cpu().numpy()
    ref = oracle.mlp_forward(P.astype(np.float64), X.astype(np.float64))
    assert np.max(np.abs(y - ref)) <= 1e-5


@pytest.mark.parametrize("n", [7, 64, 1000, 20000])
def test_mlp_gradient_matches_cpu_reference(fmm_lib, n):
    rng = np.random.default_rng(n)
    P = rng.normal(0, 0.3, size=1505).astype(np.float32)
    X = rng.normal(0, 1, size=(n, 12)).astype(np.float32)
    T = rng.uniform(math.log(0.25), math.log(8), size=n).astype(np.float32)
    loss, g = fmm_lib.mlp_loss_grad(_t(P), _t(X), _t(T))
    rl, rg = oracle.mlp_loss_grad(P.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert float(loss.cpu()[0]) == pytest.approx(rl, rel=1e-4)
    g = g.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(rg))
    assert np.max(np.abs(g - rg)) <= 1e-4 * scale


def test_adam_matches_cpu_reference(fmm_lib):
    rng = np.random.default_rng(3)
    P = rng.normal(0, 1, size=1505)
    G = rng.normal(0, 1, size=1505)
    m = rng.normal(0, 0.1, size=1505)
    v = rng.uniform(0, 0.1, size=1505)
    Pd, Gd, md, vd = (_t(a.astype(np.float32)) for a in (P, G, m, v))
    fmm_lib.mlp_adam(Pd, Gd, md, vd, 1e-3, 0.9, 0.999, 1e-8, 7)
    Pr, mr, vr = P.copy(), m.copy(), v.copy()
    oracle.adam_step(Pr, G, mr, vr, 1e-3, 0.9, 0.999, 1e-8, 7)
    assert np.max(np.abs(Pd.cpu().numpy() - Pr)) <= 1e-5
    assert np.max(np.abs(md.cpu().numpy() - mr)) <= 1e-6
    assert np.max(np.abs(vd.cpu().numpy() - vr)) <= 1e-6


def test_training_reduces_loss(fmm_lib):
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, size=(4096, 12)).astype(np.float32)
    y = np.clip(0.6 * X[:, 0] - 0.4 * X[:, 3] + 0.2, math.log(0.25) + 0.05,
                math.log(8) - 0.05).astype(np.float32)
    blob, p, hist = stride_mod.train(fmm_lib, X, y, steps=400, lr=3e-3)
    assert hist[-1] < 0.25 * hist[0]
    assert blob.size == 1505 + 24


def _learned_blob(seed):
    rng = np.random.default_rng(seed)
    P = stride_mod.init_params(seed)
    mean = rng.uniform(0, 0.5, size=12).astype(np.float32)
    std = rng.uniform(0.5, 2.0, size=12).astype(np.float32)
    return stride_mod.pack_blob(P, mean, std)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_learned_stride_replays_bitwise_on_block_reference(fmm_lib, dtype):
    p = inputs.random_problem(600, shape=(32, 32, 32), nsrc=2, dtype=dtype, obstacles=0.02)
    F = _t(p.F)
    blob = _learned_blob(5)
    psi, st, rows = stride_mod.trace_solve(fmm_lib, F, p.h, p.sources, block=8, blob=_t(blob))
    got = psi.cpu().numpy()
    bounds = np.array([r["bound"] for r in rows])
    assert len(rows) == st["restarts"]
    assert np.all(np.diff(bounds) > 0)
    ref, rs = oracle.block_fmm(p.F, p.h, p.sources, block=8, stride=2 * p.h, bounds=bounds,
                               dtype=dtype, stats=True)
    assert np.array_equal(got, ref)
    assert rs["restarts"] == st["restarts"] and rs["pops"] == st["pops"]
    base = oracle.fmm(p.F, p.h, p.sources)
    fin = np.isfinite(base)
    tol = 1e-12 if dtype == np.float64 else 1e-5 * np.max(base[fin])
    assert np.max(np.abs(got[fin] - base[fin])) <= tol
    # the multiplier applied after restart r is the network on the features recorded then
    mu, sd = blob[1505:1517].astype(np.float64), blob[1517:].astype(np.float64)
    for r in range(len(rows) - 1):
        x = (rows[r]["feat"].astype(np.float64) - mu) / sd
        m = math.exp(oracle.mlp_forward(blob[:1505].astype(np.float64), x[None, :])[0])
        assert rows[r + 1]["stride_used"] == pytest.approx(m * 2 * p.h, rel=1e-5)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_bound_schedule_replays_bitwise_on_block_reference(fmm_lib, dtype):
    """A given bound sequence (irregular, with repeats, then the stride after it) gives
    bitwise the block reference run on the same sequence; the trace shows the bounds, and
    a solve stopped at the restart cap reports it instead of failing."""
    p = inputs.random_problem(605, shape=(40, 32, 24), nsrc=2, dtype=dtype, obstacles=0.02)
    F = _t(p.F)
    rng = np.random.default_rng(7)
    bounds = np.cumsum(rng.choice([0.0, 0.5, 1.0, 3.0], size=30) * p.h) + 0.5 * p.h
    trace = torch_zeros_trace(400)
    psi, st = fmm_lib.solve(F, p.h, p.sources, block=8, stride=2 * p.h, with_stats=True,
                            stride_mode="schedule", bounds=list(bounds), trace=trace)
    got = psi.cpu().numpy()
    ref, rs = oracle.block_fmm(p.F, p.h, p.sources, block=8, stride=2 * p.h, bounds=bounds,
                               dtype=dtype, stats=True)
    assert np.array_equal(got, ref)
    assert rs["restarts"] == st["restarts"] and rs["pops"] == st["pops"]
    rows = fmm_lib.trace_rows(trace, min(st["restarts"], 400))
    for r, row in enumerate(rows[:len(bounds)]):
        assert row["bound"] == bounds[r]
    if len(rows) > len(bounds):
        assert rows[len(bounds)]["bound"] == pytest.approx(bounds[-1] + 2 * p.h, rel=1e-12)
    cap = max(2, st["restarts"] // 2)
    _, sc = fmm_lib.solve(F, p.h, p.sources, block=8, stride=2 * p.h, with_stats=True,
                          stride_mode="schedule", bounds=list(bounds), max_restarts=cap,
                          stop_at_cap=True)
    assert sc.get("stopped_at_cap") and sc["restarts"] == cap


@pytest.mark.parametrize("block", [8, 16])
def test_stop_resume_and_saved_state_continue_exactly(fmm_lib, block):
    """A solve stopped at its restart cap and resumed, and two continuations from one saved
    state (one with another bound schedule that rejoins the same bounds), each give bitwise
    the uninterrupted solve's psi, and their restart and pop counts add up."""
    import torch
    p = inputs.random_problem(606, shape=(48, 48, 32), nsrc=2, dtype=np.float32, obstacles=0.02)
    F = _t(p.F)
    s = 2 * p.h
    full, sf = fmm_lib.solve(F, p.h, p.sources, block=block, stride=s, with_stats=True)
    k = max(2, sf["restarts"] // 3)
    part, sp = fmm_lib.solve(F, p.h, p.sources, block=block, stride=s, with_stats=True,
                             max_restarts=k, stop_at_cap=True)
    assert sp["stopped_at_cap"] and sp["restarts"] == k
    state = fmm_lib.workspace_save()
    rest, sr = fmm_lib.solve_resume(F, p.h, p.sources, k, block=block, stride=s, with_stats=True)
    assert torch.equal(rest, full)
    assert sr["restarts"] == sf["restarts"] and sp["pops"] + sr["pops"] == sf["pops"]
    # the same state again, continued through a bound schedule: the fixed bounds up to k,
    # then smaller steps, then the fixed stride from the last scheduled bound
    fmm_lib.workspace_restore(state)
    sched = [r * s for r in range(1, k + 1)] + [k * s + 0.5 * s * j for j in range(1, 5)]
    alt, sa = fmm_lib.solve_resume(F, p.h, p.sources, k, block=block, stride=s, with_stats=True,
                                   stride_mode="schedule", bounds=sched)
    ref, rs = oracle.block_fmm(p.F, p.h, p.sources, block=block, stride=s, bounds=np.array(sched),
                               dtype=np.float32, stats=True)
    assert np.array_equal(alt.cpu().numpy(), ref)
    assert sp["pops"] + sa["pops"] == rs["pops"] and sa["restarts"] == rs["restarts"]
    # a resume of another problem is refused
    G = _t(inputs.random_problem(607, shape=(48, 48, 32), nsrc=1, dtype=np.float32).F)
    with pytest.raises(fmm_lib.FmmError):
        fmm_lib.solve_resume(G, p.h, [(1, 2, 3, 0.0)], k, block=block, stride=s)


def torch_zeros_trace(rows):
    import torch
    return torch.zeros(rows * fmm_lib_row_bytes(), dtype=torch.uint8, device="cuda")


def fmm_lib_row_bytes():
    from paper_1811_00009_amd import fmm
    return fmm.TRACE_ROW_BYTES


def test_learned_stride_falls_back_without_usable_weights(fmm_lib):
    import torch
    p = inputs.random_problem(601, shape=(24, 24, 24), nsrc=1)
    F = _t(p.F)
    fixed, sf = fmm_lib.solve(F, p.h, p.sources, block=8, with_stats=True)
    none, sn = fmm_lib.solve(F, p.h, p.sources, block=8, with_stats=True, stride_mode="learned")
    bad = torch.full((1505 + 24,), float("nan"), dtype=torch.float32, device="cuda")
    nan, sb = fmm_lib.solve(F, p.h, p.sources, block=8, with_stats=True, stride_mode="learned",
                            mlp_weights=bad)
    for o, s in ((none, sn), (nan, sb)):
        assert torch.equal(o, fixed)
        assert s["restarts"] == sf["restarts"]


def test_trace_rows_are_consistent(fmm_lib):
    p = inputs.random_problem(602, shape=(32, 32, 32), nsrc=1)
    F = _t(p.F)
    psi, st, rows = stride_mod.trace_solve(fmm_lib, F, p.h, p.sources, block=8)
    assert len(rows) == st["restarts"]
    assert sum(r["pops"] for r in rows) == st["pops"]
    assert rows[0]["min_popped"] == 0.0  # the source is accepted first
    for r_i, r in enumerate(rows):
        assert r["bound"] == pytest.approx((r_i + 1) * 2 * p.h)
        if r["pops"] > 0:
            assert r["min_popped"] <= r["bound"]
        else:
            assert math.isinf(r["min_popped"])
        assert r["t_end"] >= r["t_start"]
        if r["next_active"] > 0:
            assert sum(r["feat"][2:10]) == pytest.approx(1.0, abs=1e-5)
            assert 0.25 <= r["feat"][11] <= 2.0
    assert rows[-1]["next_active"] == 0


def _trained_blob():
    import os
    import torch
    path = os.path.join(os.path.dirname(stride_mod.__file__), "weights", "stride_mlp_b16.f32")
    blob = np.fromfile(path, dtype="<f4")
    assert blob.size == 1505 + 24 and np.all(np.isfinite(blob))
    return torch.from_numpy(blob).cuda()


@pytest.mark.parametrize("seed", [100, 101])
def test_trained_network_keeps_psi_and_beats_fixed_2h(fmm_lib, seed):
    """The committed network on two unseen coarse-cell fields (the training family, 256^3):
    psi stays within the FP32 bar of the fixed-stride solve and of the single-heap oracle
    (on a box around the source), the solve is faster than the plain 2h stride, and the
    stride changes from restart to restart."""
    import torch
    from boxcut import box_origin, box_slices, exact_region
    blob = _trained_blob()
    n = 256
    p = inputs.stride_field([50, seed], n, materialize=False)
    F = inputs.expand_cells_device(p.meta["V"], n, torch)
    fixed_ms, learned_ms = [], []
    for _ in range(3):
        fixed, sf = fmm_lib.solve(F, p.h, p.sources, block=16, with_stats=True)
        fixed_ms.append(sf["elapsed_ms"])
        learned, sl = fmm_lib.solve(F, p.h, p.sources, block=16, with_stats=True,
                                    stride_mode="learned", mlp_weights=blob)
        learned_ms.append(sl["elapsed_ms"])
    tol = 1e-5 * float(fixed.max())
    assert float((learned - fixed).abs().max()) <= tol
    si, sj, sk = p.sources[0][:3]
    lo = box_origin((si, sj, sk), (n, n, n), 96)
    sl_ = box_slices(lo, 96)
    ref = oracle.fmm(np.ascontiguousarray(F[sl_].cpu().numpy()), p.h,
                     [(si - lo[0], sj - lo[1], sk - lo[2], 0.0)], dtype=np.float32)
    keep = exact_region(ref, lo, (n, n, n))
    got = learned[sl_].cpu().numpy()
    assert np.max(np.abs(got[keep].astype(np.float64) - ref[keep])) <= 1e-5 * ref[keep].max()
    # the gain: fewer device milliseconds than the method with its default stride
    assert min(learned_ms) < min(fixed_ms), (learned_ms, fixed_ms)
    assert sl["restarts"] != sf["restarts"]  # the network did choose other strides
    # and not one stride for the whole solve: the multiplier follows the restart features
    _, st, rows = stride_mod.trace_solve(fmm_lib, F, p.h, p.sources, block=16, blob=blob)
    used = {round(r["stride_used"] / p.h, 4) for r in rows}  # width is infinite: none is cut
    assert len(used) > 1, used
