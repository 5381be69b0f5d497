"""Python binding of the HIP library (include/fmm.h), argument marshalling only.

Every step of a solve runs in the library's HIP kernels; this module only
passes device pointers (torch CUDA tensors) and the current HIP stream through
ctypes.  There is no fallback: if ``libfmm_hip.so`` is missing or no GPU is
present, calls raise.

Arrays are torch tensors of shape (nz, ny, nx), C-contiguous, float32 or
float64 on the GPU: the linear index of point (i, j, k) is i + nx*(j + ny*k).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_SANITIZE=1: the build with the host code under AddressSanitizer and UBSan
# (build.py --sanitize; CPU tests with libasan preloaded); FMM_LIB=<file>: another build of
# the library in this directory (variants timed side by side)
LIB_PATH = os.path.join(_HERE, os.path.basename(os.environ["FMM_LIB"]) if os.environ.get("FMM_LIB")
                        else ("libfmm_hip_san.so" if os.environ.get("FMM_SANITIZE") == "1"
                              else "libfmm_hip.so"))

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EHIP, FMM_ENOCONV, FMM_ENOTSUP = 0, -1, -2, -3, -4, -5
FMM_F32, FMM_F64 = 0, 1
STRIDE_FIXED, STRIDE_LEARNED, STRIDE_SCHEDULE = 0, 1, 2
LAUNCH_PERSISTENT, LAUNCH_HOST = 0, 1
NFEAT = 12
MLP_NPARAMS = 1505
MLP_BLOB_FLOATS = MLP_NPARAMS + 2 * NFEAT


class FmmError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


class Source(C.Structure):
    _fields_ = [("i", C.c_int64), ("j", C.c_int64), ("k", C.c_int64), ("psi0", C.c_double)]


class Options(C.Structure):
    _fields_ = [("width", C.c_double), ("stride_mode", C.c_int32), ("mlp_weights", C.c_void_p),
                ("waves_per_block", C.c_int32), ("launch_mode", C.c_int32),
                ("max_restarts", C.c_int64), ("grid_limit", C.c_int32),
                ("trace_dev", C.c_void_p), ("trace_cap", C.c_int32), ("band_lds_cap", C.c_int32),
                ("bounds", C.POINTER(C.c_double)), ("nbounds", C.c_int32),
                ("per_problem_restarts", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("restarts", C.c_int64), ("pops", C.c_int64), ("march_calls", C.c_int64),
                ("exchange_calls", C.c_int64), ("tile_loads", C.c_int64),
                ("final_bound", C.c_double), ("elapsed_ms", C.c_double), ("loop_ms", C.c_double),
                ("grid", C.c_int32),
                ("block", C.c_int32), ("waves_per_block", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64), ("h", C.c_double),
                ("F_dev", C.c_void_p), ("psi_dev", C.c_void_p), ("src", C.POINTER(Source)),
                ("nsrc", C.c_int32), ("stride", C.c_double)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("waves_per_block", C.c_int32), ("ms", C.c_double)]


class TraceRow(C.Structure):
    _fields_ = [("feat", C.c_float * NFEAT), ("bound", C.c_double), ("stride_used", C.c_double),
                ("pops", C.c_int64), ("t_start", C.c_int64), ("t_end", C.c_int64),
                ("active", C.c_int32), ("next_active", C.c_int32), ("min_popped", C.c_double)]


TRACE_ROW_BYTES = C.sizeof(TraceRow)
_lib = None


def load():
    """Load libfmm_hip.so (built in-tree by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library's HIP runtime dependency (soname libamdhip64.so.7) then
    # binds to the runtime torch already mapped, so that both share one runtime, one
    # device context and the streams passed in.  Loaded the other way round, the
    # process maps two HIP runtimes and the second one to open the device finds none.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or paper_1811_00009_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.fmm_options_default.argtypes = [C.POINTER(Options)]
    lib.fmm_options_default.restype = None
    lib.fmm_solve.argtypes = [i64, i64, i64, dbl, i32, vp, C.POINTER(Source), i32, i32, dbl, vp,
                              vp, C.POINTER(Options), C.POINTER(Stats)]
    lib.fmm_solve.restype = C.c_int
    lib.fmm_solve_resume.argtypes = [i64, i64, i64, dbl, i32, vp, C.POINTER(Source), i32, i32,
                                     dbl, vp, vp, C.POINTER(Options), i64, C.POINTER(Stats)]
    lib.fmm_solve_resume.restype = C.c_int
    lib.fmm_workspace_save.argtypes = [vp, C.c_size_t, C.POINTER(C.c_size_t), vp]
    lib.fmm_workspace_save.restype = C.c_int
    lib.fmm_workspace_restore.argtypes = [vp, C.c_size_t, vp]
    lib.fmm_workspace_restore.restype = C.c_int
    lib.fmm_solve_noalloc.argtypes = [i64, i64, i64, dbl, i32, vp, C.POINTER(Source), i32, i32,
                                      dbl, vp, vp, C.POINTER(Options), C.POINTER(Stats)]
    lib.fmm_solve_noalloc.restype = C.c_int
    lib.fmm_solve_batched.argtypes = [i32, C.POINTER(Problem), i32, i32, C.POINTER(Options), vp,
                                      C.POINTER(Stats)]
    lib.fmm_solve_batched.restype = C.c_int
    lib.fmm_autotune.argtypes = [i32, C.POINTER(Problem), i32, C.c_char_p, vp, C.POINTER(Tuning)]
    lib.fmm_autotune.restype = C.c_int
    lib.fmm_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.fmm_mlp_forward.restype = C.c_int
    lib.fmm_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    lib.fmm_mlp_loss_grad.restype = C.c_int
    lib.fmm_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, i64, vp]
    lib.fmm_mlp_adam.restype = C.c_int
    lib.fmm_mlp_train.argtypes = [vp, vp, vp, i64, i64, C.c_float, vp, vp]
    lib.fmm_mlp_train.restype = C.c_int
    lib.fmm_selftest_wave_min.argtypes = [vp, vp, i32, vp]
    lib.fmm_selftest_wave_min.restype = C.c_int
    lib.fmm_selftest_band_argmin.argtypes = [i32, i32, vp, vp, i32, i32, vp, vp, vp]
    lib.fmm_selftest_band_argmin.restype = C.c_int
    lib.fmm_strerror.argtypes = [C.c_int]
    lib.fmm_strerror.restype = C.c_char_p
    lib.fmm_last_error_detail.argtypes = []
    lib.fmm_last_error_detail.restype = C.c_char_p
    lib.fmm_version.argtypes = []
    lib.fmm_version.restype = C.c_char_p
    lib.fmm_release.argtypes = []
    lib.fmm_release.restype = C.c_int
    _lib = lib
    # free the library's device memory and events before the interpreter (and with it the
    # HIP runtime) shuts down; registered after torch's import, so it runs before torch's
    import atexit
    atexit.register(lib.fmm_release)
    return lib


def _check(rc: int, where: str):
    if rc != FMM_OK:
        lib = load()
        detail = lib.fmm_last_error_detail().decode(errors="replace")
        raise FmmError(rc, where, f"{lib.fmm_strerror(rc).decode()}: {detail}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return FMM_F32
    if t.dtype == torch.float64:
        return FMM_F64
    raise TypeError("F must be float32 or float64")


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _sources(sources) -> "C.Array":
    arr = (Source * max(1, len(sources)))()
    for s, src in enumerate(sources):
        arr[s].i, arr[s].j, arr[s].k = int(src[0]), int(src[1]), int(src[2])
        arr[s].psi0 = float(src[3]) if len(src) > 3 else 0.0
    return arr


def make_options(width=math.inf, stride_mode="fixed", mlp_weights=None, waves_per_block=1,
                 launch="persistent", max_restarts=0, grid_limit=0, trace=None,
                 band_lds_cap=0, bounds=None, per_problem_restarts=False) -> Options:
    """Options for a solve.  stride_mode: "fixed", "learned" (mlp_weights) or "schedule"
    (bounds: the bound of each restart, then the last bound plus the stride)."""
    o = Options()
    load().fmm_options_default(C.byref(o))
    o.width = float(width)
    modes = {"fixed": STRIDE_FIXED, "learned": STRIDE_LEARNED, "schedule": STRIDE_SCHEDULE}
    if stride_mode not in modes:
        raise ValueError(f"stride_mode must be one of {sorted(modes)}")
    o.stride_mode = modes[stride_mode]
    if bounds is not None:
        arr = (C.c_double * len(bounds))(*[float(b) for b in bounds])
        o._bounds_keep = arr  # the array lives as long as the options
        o.bounds = C.cast(arr, C.POINTER(C.c_double))
        o.nbounds = len(bounds)
    if mlp_weights is not None:
        import torch
        # the device reads MLP_BLOB_FLOATS float32 values through this pointer
        if mlp_weights.dtype != torch.float32:
            raise ValueError("mlp_weights must be a float32 tensor")
        if mlp_weights.numel() < MLP_BLOB_FLOATS:
            raise ValueError(f"mlp_weights must hold at least {MLP_BLOB_FLOATS} values "
                             "(parameters, feature means, feature standard deviations)")
        _check_tensor(mlp_weights, "mlp_weights")
        o.mlp_weights = mlp_weights.data_ptr()
    o.waves_per_block = int(waves_per_block)
    o.launch_mode = LAUNCH_HOST if launch == "host" else LAUNCH_PERSISTENT
    o.max_restarts = int(max_restarts)
    o.grid_limit = int(grid_limit)
    o.band_lds_cap = int(band_lds_cap)
    o.per_problem_restarts = 1 if per_problem_restarts else 0
    if trace is not None:
        _check_tensor(trace, "trace")
        o.trace_dev = trace.data_ptr()
        o.trace_cap = trace.numel() * trace.element_size() // TRACE_ROW_BYTES
    return o


def solve(F, h: float, sources: Sequence, block: int = 16, stride: Optional[float] = None,
          out=None, with_stats: bool = False, stop_at_cap: bool = False, **opts):
    """psi for speed F (GPU tensor (nz, ny, nx)) and point sources [(i, j, k[, psi0])].
    stop_at_cap: a solve that reaches max_restarts returns (its stats get
    "stopped_at_cap": True) instead of raising; psi is then incomplete."""
    import torch
    lib = load()
    _check_tensor(F, "F")
    if F.dim() != 3:
        raise ValueError("F must have shape (nz, ny, nx)")
    nz, ny, nx = F.shape
    if out is None:
        out = torch.empty_like(F)
    _check_tensor(out, "out")
    if out.dtype != F.dtype or out.shape != F.shape:
        raise ValueError("out must match F in shape and dtype")
    stride = 2.0 * h if stride is None else float(stride)
    o = make_options(**opts)
    src = _sources(sources)
    st = Stats()
    rc = lib.fmm_solve(nx, ny, nz, float(h), _dtype_code(F), F.data_ptr(), src, len(sources),
                       int(block), stride, out.data_ptr(), _stream(), C.byref(o), C.byref(st))
    if stop_at_cap and rc == FMM_ENOCONV and b"restart cap" in lib.fmm_last_error_detail():
        d = st.as_dict()
        d["stopped_at_cap"] = True
        return (out, d) if with_stats else out
    _check(rc, "fmm_solve")
    return (out, st.as_dict()) if with_stats else out


def solve_resume(F, h: float, sources: Sequence, from_restart: int, block: int = 16,
                 stride: Optional[float] = None, out=None, with_stats: bool = False,
                 stop_at_cap: bool = False, **opts):
    """Continue the solve of the same problem last stopped on this device at its restart
    cap, from restart from_restart + 1 (fmm_solve_resume); arguments as solve()."""
    import torch
    lib = load()
    _check_tensor(F, "F")
    if F.dim() != 3:
        raise ValueError("F must have shape (nz, ny, nx)")
    nz, ny, nx = F.shape
    if out is None:
        out = torch.empty_like(F)
    _check_tensor(out, "out")
    if out.dtype != F.dtype or out.shape != F.shape:
        raise ValueError("out must match F in shape and dtype")
    stride = 2.0 * h if stride is None else float(stride)
    o = make_options(**opts)
    src = _sources(sources)
    st = Stats()
    rc = lib.fmm_solve_resume(nx, ny, nz, float(h), _dtype_code(F), F.data_ptr(), src,
                              len(sources), int(block), stride, out.data_ptr(), _stream(),
                              C.byref(o), int(from_restart), C.byref(st))
    if stop_at_cap and rc == FMM_ENOCONV and b"restart cap" in lib.fmm_last_error_detail():
        d = st.as_dict()
        d["stopped_at_cap"] = True
        return (out, d) if with_stats else out
    _check(rc, "fmm_solve_resume")
    return (out, st.as_dict()) if with_stats else out


def workspace_save(buf=None):
    """The state the last solve on this device left in the library workspace, copied into a
    uint8 GPU tensor (buf, reused when large enough); see fmm_workspace_save."""
    import torch
    lib = load()
    need = C.c_size_t(0)
    _check(lib.fmm_workspace_save(None, 0, C.byref(need), _stream()), "fmm_workspace_save")
    if buf is None or buf.numel() < need.value:
        buf = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    _check(lib.fmm_workspace_save(buf.data_ptr(), buf.numel(), C.byref(need), _stream()),
           "fmm_workspace_save")
    buf._fmm_state_bytes = need.value
    return buf


def workspace_restore(buf):
    """Copy a state saved by workspace_save back into the library workspace."""
    n = getattr(buf, "_fmm_state_bytes", buf.numel())
    _check(load().fmm_workspace_restore(buf.data_ptr(), n, _stream()), "fmm_workspace_restore")


def solve_noalloc(F, h: float, sources: Sequence, out, block: int = 16,
                  stride: Optional[float] = None, with_stats: bool = False, **opts):
    """solve() through fmm_solve_noalloc: the library allocates no device memory (its
    workspace is a fixed static array per GPU).  `out` is required (same shape and dtype
    as F); grids whose workspace exceeds the array raise FmmError (FMM_ENOMEM)."""
    lib = load()
    _check_tensor(F, "F")
    if F.dim() != 3:
        raise ValueError("F must have shape (nz, ny, nx)")
    nz, ny, nx = F.shape
    _check_tensor(out, "out")
    if out.dtype != F.dtype or out.shape != F.shape:
        raise ValueError("out must match F in shape and dtype")
    stride = 2.0 * h if stride is None else float(stride)
    o = make_options(**opts)
    src = _sources(sources)
    st = Stats()
    rc = lib.fmm_solve_noalloc(nx, ny, nz, float(h), _dtype_code(F), F.data_ptr(), src,
                               len(sources), int(block), stride, out.data_ptr(), _stream(),
                               C.byref(o), C.byref(st))
    _check(rc, "fmm_solve_noalloc")
    return (out, st.as_dict()) if with_stats else out


def solve_batched(problems: Sequence, block: int = 16, with_stats: bool = False, outs=None,
                  **opts):
    """problems: [(F, h, sources[, stride])]; one persistent launch for all of them."""
    import torch
    lib = load()
    n = len(problems)
    if n == 0:
        raise ValueError("solve_batched needs at least one problem")
    arr = (Problem * n)()
    keep = []
    if outs is None:
        outs = [torch.empty_like(p[0]) for p in problems]
    elif len(outs) != n:
        raise ValueError(f"outs holds {len(outs)} tensors for {n} problems")
    for q, p in enumerate(problems):
        F = p[0]
        if F.dim() != 3:
            raise ValueError(f"F[{q}] must have shape (nz, ny, nx)")
        # the library writes nx * ny * nz values of F's dtype through outs[q]
        if outs[q].shape != F.shape or outs[q].dtype != F.dtype:
            raise ValueError(f"outs[{q}] must match F[{q}] in shape and dtype")
    dtype = None
    for q, p in enumerate(problems):
        F, h, sources = p[0], p[1], p[2]
        stride = float(p[3]) if len(p) > 3 and p[3] is not None else 2.0 * h
        _check_tensor(F, f"F[{q}]")
        _check_tensor(outs[q], f"outs[{q}]")
        d = _dtype_code(F)
        if dtype is None:
            dtype = d
        elif d != dtype:
            raise ValueError("all problems of a batch must share the dtype")
        nz, ny, nx = F.shape
        src = _sources(sources)
        keep.append(src)
        arr[q].nx, arr[q].ny, arr[q].nz, arr[q].h = nx, ny, nz, float(h)
        arr[q].F_dev, arr[q].psi_dev = F.data_ptr(), outs[q].data_ptr()
        arr[q].src = C.cast(src, C.POINTER(Source))
        arr[q].nsrc = len(sources)
        arr[q].stride = stride
    o = make_options(**opts)
    stats = (Stats * n)()
    rc = lib.fmm_solve_batched(n, arr, dtype, int(block), C.byref(o), _stream(), stats)
    _check(rc, "fmm_solve_batched")
    if with_stats:
        return outs, [s.as_dict() for s in stats]
    return outs


def autotune(samples: Sequence, cache_path: Optional[str] = None):
    """Pick (block, waves_per_block) for problems like `samples` [(F, h, sources[, stride])]."""
    import torch
    lib = load()
    n = len(samples)
    arr = (Problem * n)()
    keep, outs = [], []
    dtype = None
    for q, p in enumerate(samples):
        F, h, sources = p[0], p[1], p[2]
        stride = float(p[3]) if len(p) > 3 and p[3] is not None else 2.0 * h
        if F.dim() != 3:
            raise ValueError(f"samples[{q}]: F must have shape (nz, ny, nx)")
        _check_tensor(F, f"samples[{q}] F")
        d = _dtype_code(F)
        if dtype is not None and d != dtype:
            raise ValueError("all autotune samples must share the dtype")
        dtype = d
        nz, ny, nx = F.shape
        src = _sources(sources)
        o = torch.empty_like(F)
        keep.append(src)
        outs.append(o)
        arr[q].nx, arr[q].ny, arr[q].nz, arr[q].h = nx, ny, nz, float(h)
        arr[q].F_dev, arr[q].psi_dev = F.data_ptr(), o.data_ptr()
        arr[q].src = C.cast(src, C.POINTER(Source))
        arr[q].nsrc = len(sources)
        arr[q].stride = stride
    t = Tuning()
    path = cache_path.encode() if cache_path else None
    rc = lib.fmm_autotune(n, arr, dtype, path, _stream(), C.byref(t))
    _check(rc, "fmm_autotune")
    return {"block": t.block, "waves_per_block": t.waves_per_block, "ms": t.ms}


# ------------------------------------------------------------------ stride network
def mlp_forward(params, x):
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    _check(load().fmm_mlp_forward(params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(),
                                  _stream()), "fmm_mlp_forward")
    return y


def mlp_loss_grad(params, x, t):
    import torch
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
    _check(load().fmm_mlp_loss_grad(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0],
                                    loss.data_ptr(), grad.data_ptr(), _stream()),
           "fmm_mlp_loss_grad")
    return loss, grad


def mlp_adam(params, grad, m, v, lr, beta1, beta2, eps, t):
    _check(load().fmm_mlp_adam(params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                               float(lr), float(beta1), float(beta2), float(eps), int(t),
                               _stream()), "fmm_mlp_adam")


def mlp_train(params, x, t, steps: int, lr: float, loss_hist=None):
    _check(load().fmm_mlp_train(params.data_ptr(), x.data_ptr(), t.data_ptr(), x.shape[0],
                                int(steps), float(lr),
                                loss_hist.data_ptr() if loss_hist is not None else None,
                                _stream()), "fmm_mlp_train")


def selftest_wave_min(x):
    """x: uint32 values as an int32 GPU tensor of 64*W elements -> W per-wave minima."""
    import torch
    nw = x.numel() // 64
    out = torch.empty(nw, dtype=torch.int32, device=x.device)
    _check(load().fmm_selftest_wave_min(x.data_ptr(), out.data_ptr(), nw, _stream()),
           "fmm_selftest_wave_min")
    return out


def selftest_band_argmin(psi_tile, band, block: int, cap: int = 0):
    """Locate_Min of a march by one wave on a given band: psi_tile is the (B+2)^3 tile of
    one block (float32 or float64 GPU tensor), band the tile indices (int16 GPU tensor).
    Returns (value, tile index, slot)."""
    import torch
    _check_tensor(psi_tile, "psi_tile")
    _check_tensor(band, "band")
    if band.dtype != torch.int16:
        raise TypeError("band must be an int16 tensor of tile indices")
    dt = _dtype_code(psi_tile)
    val = torch.empty(1, dtype=psi_tile.dtype, device=psi_tile.device)
    idx = torch.empty(2, dtype=torch.int32, device=psi_tile.device)
    _check(load().fmm_selftest_band_argmin(dt, int(block), psi_tile.data_ptr(), band.data_ptr(),
                                           int(band.numel()), int(cap), val.data_ptr(),
                                           idx.data_ptr(), _stream()),
           "fmm_selftest_band_argmin")
    i = idx.cpu().tolist()
    return val.item(), i[0], i[1]


def trace_rows(trace_tensor, count: int):
    """Decode the first `count` trace rows of a trace buffer (after a solve)."""
    import numpy as np
    raw = trace_tensor.detach().cpu().numpy().tobytes()
    rows = []
    for r in range(count):
        tr = TraceRow.from_buffer_copy(raw[r * TRACE_ROW_BYTES:(r + 1) * TRACE_ROW_BYTES])
        rows.append({"feat": np.array(tr.feat[:], dtype=np.float32), "bound": tr.bound,
                     "stride_used": tr.stride_used, "pops": tr.pops, "t_start": tr.t_start,
                     "t_end": tr.t_end, "active": tr.active, "next_active": tr.next_active,
                     "min_popped": tr.min_popped})
    return rows


def version() -> str:
    return load().fmm_version().decode()
