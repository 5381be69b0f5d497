"""CPU oracle for the block-based restarted narrow-band FMM -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``liboracle.so`` (plain C, built by ``oracle/build.py``).
Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package; the HIP product path never does.

Array convention: numpy arrays of shape (nz, ny, nx), C-contiguous, so the
linear index of grid point (i, j, k) is i + nx*(j + ny*k).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_SANITIZE=1 loads the AddressSanitizer / UBSan builds (build.py --sanitize)
_SAN = os.environ.get("FMM_SANITIZE") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if _SAN else "liboracle.so")
_lib = None

ORC_EINVAL, ORC_ENOMEM, ORC_ENOCONV = -1, -2, -3

_i64 = C.c_int64
_i32 = C.c_int32
_dbl = C.c_double
_vp = C.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build(sanitize=_SAN)
    lib = C.CDLL(_LIB_PATH)
    for sfx in ("f64", "f32"):
        f = getattr(lib, f"orc_fmm_{sfx}")
        f.restype = C.c_int
        f.argtypes = [_i64, _i64, _i64, _dbl, _vp, _i32, _vp, _vp, _dbl, _i32, _vp, _vp, _vp]
        f = getattr(lib, f"orc_block_fmm_{sfx}")
        f.restype = C.c_int
        f.argtypes = [_i64, _i64, _i64, _dbl, _vp, _i32, _vp, _vp, _i32, _dbl, _dbl, _vp, _i32,
                      _i32, _i64, _vp, _vp, _vp, _vp, _vp]
    for name in ("orc_gauss_seidel", "orc_jacobi"):
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = [_i64, _i64, _i64, _dbl, _vp, _i32, _vp, _vp, _i64, _vp, _vp]
    lib.orc_mlp_nparams.restype = C.c_int
    lib.orc_mlp_forward.restype = C.c_int
    lib.orc_mlp_forward.argtypes = [_vp, _vp, _i64, _vp]
    lib.orc_mlp_loss_grad.restype = C.c_int
    lib.orc_mlp_loss_grad.argtypes = [_vp, _vp, _vp, _i64, _vp, _vp]
    lib.orc_adam_step.restype = C.c_int
    lib.orc_adam_step.argtypes = [_vp, _vp, _vp, _vp, _i64, _dbl, _dbl, _dbl, _dbl, _i64]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def _sources(shape, sources, dtype):
    nz, ny, nx = shape
    idx = np.empty(len(sources), dtype=np.int64)
    val = np.empty(len(sources), dtype=dtype)
    for s, src in enumerate(sources):
        i, j, k = int(src[0]), int(src[1]), int(src[2])
        idx[s] = i + nx * (j + ny * k)
        val[s] = float(src[3]) if len(src) > 3 else 0.0
    return idx, val


def _speed(F: np.ndarray, dtype):
    F = np.ascontiguousarray(F, dtype=dtype)
    if F.ndim != 3:
        raise ValueError("F must have shape (nz, ny, nx)")
    return F


def fmm(F: np.ndarray, h: float, sources, width: float = math.inf, literal: bool = False,
        dtype=np.float64, stats: bool = False):
    """Baseline single-heap FMM (paper Sec. 2.1 + 2.2).  sources: [(i, j, k[, psi0]), ...]."""
    lib = _load()
    F = _speed(F, dtype)
    nz, ny, nx = F.shape
    idx, val = _sources(F.shape, sources, dtype)
    psi = np.empty_like(F)
    pops, nonmono = _i64(0), _i64(0)
    fn = lib.orc_fmm_f64 if dtype == np.float64 else lib.orc_fmm_f32
    rc = fn(nx, ny, nz, h, _ptr(F), len(idx), _ptr(idx), _ptr(val), width, int(literal), _ptr(psi),
            C.byref(pops), C.byref(nonmono))
    _check(rc, "orc_fmm")
    if stats:
        return psi, {"pops": pops.value, "nonmonotone_pops": nonmono.value}
    return psi


def block_fmm(F: np.ndarray, h: float, sources, block: int, stride: float, width: float = math.inf,
              bounds=None, literal: bool = False, dtype=np.float64, max_restarts: int = 0,
              stats: bool = False):
    """Multi-block restarted method, Alg. 6 executed literally on the CPU."""
    lib = _load()
    F = _speed(F, dtype)
    nz, ny, nx = F.shape
    idx, val = _sources(F.shape, sources, dtype)
    psi = np.empty_like(F)
    if bounds is not None:
        b = np.ascontiguousarray(bounds, dtype=np.float64)
        bp, nb = _ptr(b), len(b)
    else:
        bp, nb = None, 0
    r, pops, mc, ec = _i64(0), _i64(0), _i64(0), _i64(0)
    fn = lib.orc_block_fmm_f64 if dtype == np.float64 else lib.orc_block_fmm_f32
    rc = fn(nx, ny, nz, h, _ptr(F), len(idx), _ptr(idx), _ptr(val), block, stride, width, bp, nb,
            int(literal), max_restarts, _ptr(psi), C.byref(r), C.byref(pops), C.byref(mc),
            C.byref(ec))
    _check(rc, "orc_block_fmm")
    if stats:
        return psi, {"restarts": r.value, "pops": pops.value, "march_calls": mc.value,
                     "exchange_calls": ec.value}
    return psi


def gauss_seidel(F: np.ndarray, h: float, sources, max_sweeps: int = 100000, stats: bool = False):
    lib = _load()
    F = _speed(F, np.float64)
    nz, ny, nx = F.shape
    idx, val = _sources(F.shape, sources, np.float64)
    psi = np.empty_like(F)
    sw = _i64(0)
    rc = lib.orc_gauss_seidel(nx, ny, nz, h, _ptr(F), len(idx), _ptr(idx), _ptr(val), max_sweeps,
                              _ptr(psi), C.byref(sw))
    _check(rc, "orc_gauss_seidel")
    return (psi, {"sweeps": sw.value}) if stats else psi


def jacobi(F: np.ndarray, h: float, sources, max_iters: int = 100000, stats: bool = False):
    lib = _load()
    F = _speed(F, np.float64)
    nz, ny, nx = F.shape
    idx, val = _sources(F.shape, sources, np.float64)
    psi = np.empty_like(F)
    it = _i64(0)
    rc = lib.orc_jacobi(nx, ny, nz, h, _ptr(F), len(idx), _ptr(idx), _ptr(val), max_iters,
                        _ptr(psi), C.byref(it))
    _check(rc, "orc_jacobi")
    return (psi, {"iters": it.value}) if stats else psi


# ---------------------------------------------------------------- stride network (FP64)
MLP_NPARAMS = 1505


def mlp_forward(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    lib = _load()
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.empty(X.shape[0], dtype=np.float64)
    _check(lib.orc_mlp_forward(_ptr(P), _ptr(X), X.shape[0], _ptr(y)), "orc_mlp_forward")
    return y


def mlp_loss_grad(params: np.ndarray, X: np.ndarray, T: np.ndarray):
    lib = _load()
    P = np.ascontiguousarray(params, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.empty(MLP_NPARAMS, dtype=np.float64)
    loss = _dbl(0)
    _check(lib.orc_mlp_loss_grad(_ptr(P), _ptr(X), _ptr(T), X.shape[0], C.byref(loss), _ptr(g)),
           "orc_mlp_loss_grad")
    return loss.value, g


def adam_step(params, grad, m, v, lr, beta1, beta2, eps, t):
    """In-place Adam update of float64 arrays params, m, v."""
    lib = _load()
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    _check(lib.orc_adam_step(_ptr(params), _ptr(g), _ptr(m), _ptr(v), len(params), lr, beta1,
                             beta2, eps, t), "orc_adam_step")


# ------------------------------------------------------------------ parallel CPU baseline
_par = None


def _load_par():
    global _par
    if _par is not None:
        return _par
    path = os.path.join(_HERE, "libcpu_parallel_san.so" if _SAN else "libcpu_parallel.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build(sanitize=_SAN)
    lib = C.CDLL(path)
    for sfx in ("f64", "f32"):
        f = getattr(lib, f"cpu_block_fmm_par_{sfx}")
        f.restype = C.c_int
        f.argtypes = [_i64, _i64, _i64, _dbl, _vp, _i32, _vp, _vp, _i32, _dbl, _dbl, _i32, _i64,
                      _vp, _vp, _vp, _vp]
    _par = lib
    return lib


def block_fmm_parallel(F: np.ndarray, h: float, sources, block: int, stride: float,
                       width: float = math.inf, threads: int = 0, dtype=np.float64,
                       stats: bool = False):
    """The paper's parallel CPU solver (Sec. 2.7): the block method of block_fmm with
    each step's blocks spread over OpenMP threads, in FP64 or FP32 (bitwise the block
    reference of the same precision).  A comparison baseline, and the reference for
    grids too large for the sequential block reference."""
    lib = _load_par()
    F = _speed(F, dtype)
    nz, ny, nx = F.shape
    idx, val = _sources(F.shape, sources, dtype)
    psi = np.empty_like(F)
    r, pops, used = _i64(0), _i64(0), _i32(0)
    fn = lib.cpu_block_fmm_par_f64 if dtype == np.float64 else lib.cpu_block_fmm_par_f32
    rc = fn(nx, ny, nz, h, _ptr(F), len(idx), _ptr(idx), _ptr(val), block, stride, width,
            threads, 0, _ptr(psi), C.byref(r), C.byref(pops), C.byref(used))
    _check(rc, "cpu_block_fmm_par")
    if stats:
        return psi, {"restarts": r.value, "pops": pops.value, "threads": used.value}
    return psi
