"""fmm_solve_noalloc: the entry point that allocates no device memory (its workspace is
one static device array per GPU) gives bitwise the result and counts of fmm_solve, on
two calls in a row with the second on a smaller grid (the array keeps the first call's
data, which the second must not see), and rejects grids that do not fit before any
device work."""
import ctypes as C

import numpy as np
import pytest

from paper_1811_00009_amd import fmm, inputs

SCRATCH_BYTES = 64 << 20


def _raw_noalloc(nx, ny, nz, block, dtype=fmm.FMM_F32, srcs=((1, 1, 1, 0.0),)):
    lib = fmm.load()
    buf = C.create_string_buffer(64)  # never dereferenced: rejected before device work
    arr = fmm._sources(list(srcs))
    st = fmm.Stats()
    return lib.fmm_solve_noalloc(nx, ny, nz, 0.01, dtype, C.cast(buf, C.c_void_p), arr,
                                 len(srcs), block, 0.02, C.cast(buf, C.c_void_p), None, None,
                                 C.byref(st))


def test_noalloc_rejects_grids_beyond_the_scratch_on_the_host():
    lib = fmm.load()
    assert _raw_noalloc(256, 256, 256, 16) == fmm.FMM_ENOMEM       # ~265 MB of workspace
    detail = lib.fmm_last_error_detail().decode()
    assert "bytes" in detail and str(SCRATCH_BYTES) in detail
    assert _raw_noalloc(192, 192, 192, 8, fmm.FMM_F64) == fmm.FMM_ENOMEM
    many = [(i % 16, i // 16, 0, 0.0) for i in range(257)]
    assert _raw_noalloc(16, 16, 16, 8, srcs=many) == fmm.FMM_EINVAL  # more than 256 sources
    assert _raw_noalloc(20, 16, 16, 8) == fmm.FMM_EINVAL              # not divisible
    assert _raw_noalloc(16, 16, 16, 5) == fmm.FMM_ENOTSUP


CASES = [
    # (shape of the first call, shape of the second, block, dtype, waves)
    ((96, 80, 64), (40, 32, 24), 8, np.float32, 1),
    ((128, 128, 112), (48, 32, 64), 16, np.float32, 1),
    ((64, 64, 48), (16, 24, 32), 8, np.float64, 2),
]


@pytest.mark.gpu
@pytest.mark.parametrize("big,small,block,dtype,waves", CASES)
def test_noalloc_equals_fmm_solve_on_two_calls(fmm_lib, big, small, block, dtype, waves):
    import torch
    for call, shape in enumerate((big, small)):
        p = inputs.random_problem(900 + call, shape=shape, nsrc=3, obstacles=0.02, dtype=dtype)
        F = torch.from_numpy(p.F).cuda()
        print(f"[noalloc] call {call}: {shape} block {block} {np.dtype(dtype).name} waves {waves}",
              flush=True)
        ref, rs = fmm_lib.solve(F, p.h, p.sources, block=block, with_stats=True,
                                waves_per_block=waves)
        out = torch.full_like(F, -1.0)
        got, st = fmm_lib.solve_noalloc(F, p.h, p.sources, out, block=block, with_stats=True,
                                        waves_per_block=waves)
        torch.cuda.synchronize()
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), float(np.nanmax(np.abs(a - b)))
        for k in ("restarts", "pops", "march_calls", "exchange_calls", "tile_loads"):
            assert st[k] == rs[k], (k, st[k], rs[k])
        assert st["elapsed_ms"] == 0.0


@pytest.mark.gpu
def test_noalloc_at_the_largest_grid_that_fits(fmm_lib):
    """A grid whose workspace nearly fills the array (160^3 FP32 at block 16: 1000 blocks)."""
    import torch
    p = inputs.coarse_cells(160, 16, seed=(77,), materialize=True)
    F = torch.from_numpy(p.F).cuda()
    ref = fmm_lib.solve(F, p.h, p.sources, block=16)
    out = torch.empty_like(F)
    got = fmm_lib.solve_noalloc(F, p.h, p.sources, out, block=16)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
