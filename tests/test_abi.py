"""The C-ABI library builds, loads and exports what include/fmm.h declares; host-side
argument validation rejects bad input before any device work (no GPU needed)."""
import ctypes as C
import math
import os
import re

import pytest

from paper_1811_00009_amd import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(fmm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("fmm_solve", "fmm_solve_batched", "fmm_autotune", "fmm_mlp_forward",
                     "fmm_mlp_loss_grad", "fmm_mlp_adam", "fmm_mlp_train", "fmm_strerror",
                     "fmm_options_default"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = fmm.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    assert C.sizeof(fmm.Source) == 32
    assert C.sizeof(fmm.TraceRow) == 48 + 8 * 5 + 8 + 8
    assert C.sizeof(fmm.Stats) == 5 * 8 + 3 * 8 + 4 * 4
    assert C.sizeof(fmm.Options) == 80


def test_options_default():
    o = fmm.Options()
    fmm.load().fmm_options_default(C.byref(o))
    assert math.isinf(o.width) and o.stride_mode == 0 and o.waves_per_block == 1
    assert o.launch_mode == 0 and o.max_restarts == 0


def _solve_raw(nx=16, ny=16, nz=16, h=0.1, dtype=0, F=1, srcs=((1, 1, 1, 0.0),), block=8,
               stride=0.2, psi=1, opt=None):
    lib = fmm.load()
    arr = fmm._sources(list(srcs))
    st = fmm.Stats()
    return lib.fmm_solve(nx, ny, nz, h, dtype, C.c_void_p(F), arr, len(srcs), block, stride,
                         C.c_void_p(psi), None, C.byref(opt) if opt else None, C.byref(st))


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), fmm.FMM_EINVAL),
    (dict(h=0.0), fmm.FMM_EINVAL),
    (dict(h=float("nan")), fmm.FMM_EINVAL),
    (dict(h=float("inf")), fmm.FMM_EINVAL),
    (dict(stride=0.0), fmm.FMM_EINVAL),
    (dict(stride=-1.0), fmm.FMM_EINVAL),
    (dict(stride=float("nan")), fmm.FMM_EINVAL),
    (dict(block=64), fmm.FMM_ENOTSUP),
    (dict(block=5), fmm.FMM_ENOTSUP),
    (dict(nx=20), fmm.FMM_EINVAL),          # not divisible by the block
    (dict(F=0), fmm.FMM_EINVAL),            # NULL speed
    (dict(psi=0), fmm.FMM_EINVAL),          # NULL output
    (dict(srcs=()), fmm.FMM_EINVAL),        # no source
    (dict(srcs=((16, 0, 0, 0.0),)), fmm.FMM_EINVAL),   # outside the grid
    (dict(srcs=((0, 0, 0, -1.0),)), fmm.FMM_EINVAL),   # negative psi0
    (dict(srcs=((0, 0, 0, float("inf")),)), fmm.FMM_EINVAL),
    (dict(dtype=7), fmm.FMM_EINVAL),
])
def test_validation_rejects_bad_arguments(kw, code):
    assert _solve_raw(**kw) == code
    assert len(fmm.load().fmm_last_error_detail()) > 0


def test_validation_rejects_bad_options():
    o = fmm.Options()
    fmm.load().fmm_options_default(C.byref(o))
    o.waves_per_block = 3
    assert _solve_raw(opt=o) == fmm.FMM_EINVAL
    fmm.load().fmm_options_default(C.byref(o))
    o.width = 0.0
    assert _solve_raw(opt=o) == fmm.FMM_EINVAL
    fmm.load().fmm_options_default(C.byref(o))
    o.stride_mode = 5
    assert _solve_raw(opt=o) == fmm.FMM_EINVAL
    fmm.load().fmm_options_default(C.byref(o))
    o.stride_mode = fmm.STRIDE_LEARNED
    assert _solve_raw(stride=float("inf"), opt=o) == fmm.FMM_EINVAL


def test_bound_schedule_is_checked_on_the_host():
    """FMM_STRIDE_SCHEDULE needs a host array of finite, positive, non-decreasing bounds."""
    def opts(bounds, n=None):
        o = fmm.Options()
        fmm.load().fmm_options_default(C.byref(o))
        o.stride_mode = fmm.STRIDE_SCHEDULE
        if bounds is not None:
            arr = (C.c_double * len(bounds))(*bounds)
            o._keep = arr
            o.bounds = C.cast(arr, C.POINTER(C.c_double))
        o.nbounds = len(bounds) if n is None else n
        return o
    assert _solve_raw(opt=opts(None, 3)) == fmm.FMM_EINVAL
    assert _solve_raw(opt=opts([0.1, 0.2], 0)) == fmm.FMM_EINVAL
    assert _solve_raw(opt=opts([0.2, 0.1])) == fmm.FMM_EINVAL        # decreasing
    assert _solve_raw(opt=opts([0.0, 0.1])) == fmm.FMM_EINVAL        # not > 0
    assert _solve_raw(opt=opts([0.1, float("inf")])) == fmm.FMM_EINVAL
    assert _solve_raw(opt=opts([0.1, 0.2]), stride=float("inf")) == fmm.FMM_EINVAL
    with pytest.raises(ValueError):
        fmm.make_options(stride_mode="adaptive")


def test_block_32_takes_one_wave_per_block():
    """32^3 blocks march their tile in device memory with one wave; more waves are refused
    before any device work."""
    o = fmm.Options()
    fmm.load().fmm_options_default(C.byref(o))
    o.waves_per_block = 2
    assert _solve_raw(nx=32, ny=32, nz=32, block=32, opt=o) == fmm.FMM_ENOTSUP
    assert "one wave" in fmm.load().fmm_last_error_detail().decode()


def test_strerror_covers_codes():
    lib = fmm.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.fmm_strerror(code)
    assert fmm.version().startswith("fmm-mi355x")


def test_batched_and_mlp_reject_bad_arguments():
    lib = fmm.load()
    assert lib.fmm_solve_batched(0, None, 0, 16, None, None, None) == fmm.FMM_EINVAL
    assert lib.fmm_mlp_forward(None, None, 0, None, None) == fmm.FMM_EINVAL
    assert lib.fmm_mlp_adam(None, None, None, None, 0.1, 0.9, 0.99, 1e-8, 0, None) == fmm.FMM_EINVAL
    assert lib.fmm_autotune(0, None, 0, None, None, None) == fmm.FMM_EINVAL


def test_locate_min_probe_rejects_bad_arguments_on_the_host():
    lib = fmm.load()
    buf = C.create_string_buffer(64)  # never dereferenced: every case fails before device work
    p, b, v, i = (C.cast(buf, C.c_void_p),) * 4
    call = lib.fmm_selftest_band_argmin
    assert call(fmm.FMM_F32, 16, None, b, 1, 0, v, i, None) == fmm.FMM_EINVAL   # null psi
    assert call(fmm.FMM_F32, 16, p, None, 1, 0, v, i, None) == fmm.FMM_EINVAL   # null band
    assert call(fmm.FMM_F32, 16, p, b, 1, 100, v, i, None) == fmm.FMM_EINVAL    # cap % 512
    assert call(fmm.FMM_F32, 16, p, b, 1, -512, v, i, None) == fmm.FMM_EINVAL
    assert call(7, 16, p, b, 1, 0, v, i, None) == fmm.FMM_EINVAL                # dtype
    assert call(fmm.FMM_F32, 12, p, b, 1, 0, v, i, None) == fmm.FMM_EINVAL      # block size
    assert call(fmm.FMM_F32, 16, p, b, 0, 0, v, i, None) == fmm.FMM_EINVAL      # empty band
    assert call(fmm.FMM_F64, 8, p, b, 1000, 0, v, i, None) == fmm.FMM_EINVAL    # n >= (B+2)^3


def test_binding_checks_batched_outputs_and_weights_on_the_host():
    """The binding refuses buffers the library would write or read past: outs of the wrong
    count, shape or dtype, speed fields that are not 3-D, and stride weights that are not
    float32 or hold fewer values than the device reads.  CPU tensors suffice: every check
    fires before a pointer is passed."""
    import torch
    F = torch.ones(16, 16, 16, dtype=torch.float32)
    batch = [(F, 0.1, [(1, 1, 1)]), (F, 0.1, [(2, 2, 2)])]
    with pytest.raises(ValueError, match="outs holds"):
        fmm.solve_batched(batch, block=8, outs=[torch.empty_like(F)])
    with pytest.raises(ValueError, match="shape and dtype"):
        fmm.solve_batched(batch, block=8, outs=[torch.empty_like(F), torch.empty(8, 16, 16)])
    with pytest.raises(ValueError, match="shape and dtype"):
        fmm.solve_batched(batch, block=8, outs=[torch.empty_like(F), torch.empty_like(F).double()])
    with pytest.raises(ValueError, match=r"shape \(nz, ny, nx\)"):
        fmm.solve_batched([(F.reshape(16, 256), 0.1, [(1, 1, 1)])], block=8)
    with pytest.raises(ValueError, match="at least one"):
        fmm.solve_batched([], block=8)
    with pytest.raises(ValueError, match="float32"):
        fmm.make_options(mlp_weights=torch.zeros(fmm.MLP_BLOB_FLOATS, dtype=torch.float64))
    with pytest.raises(ValueError, match="at least"):
        fmm.make_options(mlp_weights=torch.zeros(fmm.MLP_NPARAMS, dtype=torch.float32))
