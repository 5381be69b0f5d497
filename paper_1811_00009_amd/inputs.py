"""Seeded synthetic inputs (speed fields and source points).

This module only draws random numbers and evaluates the speed formulas that
define the workloads; it holds none of the solver's arithmetic.  Both the CPU
oracle (in tests) and the HIP library are fed the same arrays from here.

Arrays are numpy, shape (nz, ny, nx), C-contiguous: the linear index of grid
point (i, j, k) is i + nx*(j + ny*k).  Node-centred grids on [0, 1]^3 with
x_i = i*h, h = 1/(n-1).

Workloads
---------
* ``smooth_point``   64^3, F = 1, source at (32, 32, 32), FP64, 8^3 blocks.
* ``smooth_sine``    256^3, F = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z),
                     source at the corner (0, 0, 0), 16^3 blocks.
* ``coarse_cells``   1024^3, F piecewise constant on 64^3 coarse cells with
                     i.i.d. U[0.5, 2.0] values, random interior source.
* ``batched``        512 cubes, sides uniform over {32, 48, ..., 192}, speed
                     1 + 0.75 g / max|g| with g a sum of 8 random Fourier modes.
* ``stride_fields``  coarse-cell fields used to train / evaluate the stride
                     network.
The paper's own test speeds (its Sec. 3.1, cases 1-4) are also provided.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    name: str
    F: np.ndarray                 # (nz, ny, nx)
    h: float
    sources: list                 # [(i, j, k, psi0)]
    block: int = 16
    stride: float = 0.0           # 0 -> 2h
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.F.shape

    @property
    def npoints(self):
        return int(np.prod(self.F.shape))

    def stride_or_default(self):
        return self.stride if self.stride > 0 else 2.0 * self.h


def _coords(n: int, dtype=np.float64):
    h = 1.0 / (n - 1)
    return np.arange(n, dtype=np.float64) * h, h


# --------------------------------------------------------------------------- configs
def smooth_point(n: int = 64, dtype=np.float64) -> Problem:
    """Constant speed, single source at index n/2 of every axis."""
    h = 1.0 / (n - 1)
    F = np.ones((n, n, n), dtype=dtype)
    c = n // 2
    return Problem("smooth_point", F, h, [(c, c, c, 0.0)], block=8, stride=2 * h,
                   meta={"n": n})


def sine_speed(n: int, dtype=np.float64) -> np.ndarray:
    x, _ = _coords(n)
    s = np.sin(2 * np.pi * x)
    F = 1.0 + 0.5 * s[:, None, None] * s[None, :, None] * s[None, None, :]
    return np.ascontiguousarray(F, dtype=dtype)


def smooth_sine(n: int = 256, dtype=np.float32) -> Problem:
    """F = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z), source at the corner."""
    h = 1.0 / (n - 1)
    return Problem("smooth_sine", sine_speed(n, dtype), h, [(0, 0, 0, 0.0)], block=16,
                   stride=2 * h, meta={"n": n})


def coarse_cell_values(seed_words, cells: int, lo: float = 0.5, hi: float = 2.0):
    """Coarse-cell speed values and the generator positioned after them."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_words)))
    V = rng.uniform(lo, hi, size=(cells, cells, cells))  # indexed [kc, jc, ic]
    return V, rng


def expand_cells(V: np.ndarray, n: int, dtype=np.float32) -> np.ndarray:
    """F[k, j, i] = V[k // r, j // r, i // r] with r = n / cells."""
    cells = V.shape[0]
    r = n // cells
    assert r * cells == n
    F = np.broadcast_to(V.astype(dtype)[:, None, :, None, :, None],
                        (cells, r, cells, r, cells, r)).reshape(n, n, n)
    return np.ascontiguousarray(F)


def coarse_cells(n: int = 1024, cells: int = 64, seed=(3,), dtype=np.float32,
                 materialize: bool = True) -> Problem:
    """Piecewise-constant speed on cells^3 coarse cells, U[0.5, 2.0], random source."""
    V, rng = coarse_cell_values(seed, cells)
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))  # uniform in [1, n-2]^3
    h = 1.0 / (n - 1)
    F = expand_cells(V, n, dtype) if materialize else None
    return Problem("coarse_cells", F, h, [(src[0], src[1], src[2], 0.0)], block=16,
                   stride=2 * h, meta={"n": n, "cells": cells, "seed": list(seed), "V": V})


BATCH_SIDES = tuple(range(32, 193, 16))  # 32, 48, ..., 192


def fourier_modes(rng, modes: int = 8):
    """Draw the random modes (k_m, a_m, phi_m) of the Fourier speed, in draw order."""
    out = []
    for _ in range(modes):
        kv = rng.integers(1, 5, size=3)            # wavenumbers 1..4 per axis
        a = float(rng.uniform(-1.0, 1.0))
        phi = float(rng.uniform(0.0, 2 * np.pi))
        out.append((kv, a, phi))
    return out


def fourier_speed(n: int, rng, modes: int = 8, amp: float = 0.75, dtype=np.float32):
    """F = 1 + amp * g / max|g|, g(x) = sum_m a_m cos(2 pi k_m . x + phi_m)."""
    x, _ = _coords(n)
    g = np.zeros((n, n, n), dtype=np.float64)
    for kv, a, phi in fourier_modes(rng, modes):
        ph = (2 * np.pi * kv[2] * x[:, None, None] + 2 * np.pi * kv[1] * x[None, :, None]
              + 2 * np.pi * kv[0] * x[None, None, :])
        g += a * np.cos(ph + phi)
    g /= np.abs(g).max()
    return np.ascontiguousarray(1.0 + amp * g, dtype=dtype)


def batched_problem(s: int, dtype=np.float32) -> Problem:
    rng = np.random.default_rng(np.random.SeedSequence([4, s]))
    n = int(rng.choice(BATCH_SIDES))
    h = 1.0 / (n - 1)
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))
    F = fourier_speed(n, rng, dtype=dtype)
    return Problem(f"batched[{s}]", F, h, [(src[0], src[1], src[2], 0.0)], block=16,
                   stride=2 * h, meta={"n": n, "seed": [4, s]})


# ------------------------------------------------------------------ the same fields built on a GPU
# Large workloads are evaluated on the device from the same random draws (FP64,
# then cast), which keeps multi-GiB host arrays out of the benchmark.  The values
# agree with the host versions to the last bit of the cast in all but rare cases
# (device and host cosines may differ in the last FP64 bit).
def expand_cells_device(V: np.ndarray, n: int, torch, dtype=None):
    """Device tensor F[k, j, i] = V[k // r, j // r, i // r], r = n / cells."""
    dtype = dtype or torch.float32
    c = V.shape[0]
    r = n // c
    assert r * c == n
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to("cuda").to(dtype)
    return Vd[:, None, :, None, :, None].expand(c, r, c, r, c, r).reshape(n, n, n).contiguous()


def fourier_speed_device(n: int, modes, torch, amp: float = 0.75, dtype=None):
    dtype = dtype or torch.float32
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (1.0 / (n - 1))
    g = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    for kv, a, phi in modes:
        ph = (2 * math.pi * float(kv[2]) * x[:, None, None]
              + 2 * math.pi * float(kv[1]) * x[None, :, None]
              + 2 * math.pi * float(kv[0]) * x[None, None, :])
        g += a * torch.cos(ph + phi)
    g /= g.abs().max()
    return (1.0 + amp * g).to(dtype).contiguous()


def batched_problem_device(s: int, torch) -> Problem:
    """batched_problem(s) with F built on the GPU (FP32)."""
    rng = np.random.default_rng(np.random.SeedSequence([4, s]))
    n = int(rng.choice(BATCH_SIDES))
    h = 1.0 / (n - 1)
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))
    F = fourier_speed_device(n, fourier_modes(rng), torch)
    return Problem(f"batched[{s}]", F, h, [(src[0], src[1], src[2], 0.0)], block=16,
                   stride=2 * h, meta={"n": n, "seed": [4, s]})


def batched_sides(count: int = 512):
    """Side of every batched problem without building its field."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(np.random.SeedSequence([4, s]))
        out.append(int(rng.choice(BATCH_SIDES)))
    return out


def stride_field(seed_words, n: int, cells: int = 64, dtype=np.float32,
                 materialize: bool = True) -> Problem:
    """Coarse-cell field with a random interior source (stride-network data)."""
    V, rng = coarse_cell_values(seed_words, cells)
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))
    h = 1.0 / (n - 1)
    F = expand_cells(V, n, dtype) if materialize else None
    return Problem(f"stride_field{list(seed_words)}", F, h, [(src[0], src[1], src[2], 0.0)],
                   block=16, stride=2 * h, meta={"n": n, "cells": cells, "V": V})


def fourier_field_device(seed_words, n: int, torch) -> Problem:
    """Stride-network family: Fourier speed as in the batched workload, on an n^3 grid."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_words)))
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))
    F = fourier_speed_device(n, fourier_modes(rng), torch)
    return Problem(f"fourier{list(seed_words)}", F, 1.0 / (n - 1),
                   [(src[0], src[1], src[2], 0.0)], block=16, meta={"n": n})


def sine_field_device(seed_words, n: int, torch) -> Problem:
    """Stride-network family: F = 1 + a sin(2 pi k x) sin(2 pi k y) sin(2 pi k z),
    a ~ U[0.2, 0.9], k uniform in {1, 2, 3}, random interior source."""
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_words)))
    src = tuple(int(v) for v in rng.integers(1, n - 1, size=3))
    a = float(rng.uniform(0.2, 0.9))
    k = int(rng.integers(1, 4))
    x = torch.arange(n, dtype=torch.float64, device="cuda") * (1.0 / (n - 1))
    s = torch.sin(2 * math.pi * k * x)
    F = 1.0 + a * s[:, None, None] * s[None, :, None] * s[None, None, :]
    return Problem(f"sine{list(seed_words)}", F.to(torch.float32).contiguous(), 1.0 / (n - 1),
                   [(src[0], src[1], src[2], 0.0)], block=16, meta={"n": n, "a": a, "k": k})


# --------------------------------------------------------------------------- the paper's cases
def paper_case(case: int, n: int, dtype=np.float64) -> Problem:
    """The four point-source problems of the paper's Sec. 3.1 on a cell-centred grid of
    the cube [-0.5, 0.5]^3 with the source at the grid point nearest the centre."""
    h = 1.0 / n
    x = -0.5 + (np.arange(n) + 0.5) * h
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    if case == 1:
        F = np.ones((n, n, n))
    elif case == 2:
        F = 1 + 0.5 * np.sin(20 * np.pi * X) * np.sin(20 * np.pi * Y) * np.sin(20 * np.pi * Z)
    elif case == 3:
        F = 1 - 0.99 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y) * np.sin(2 * np.pi * Z)
    elif case == 4:
        R = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
        r = np.sqrt(X ** 2 + Y ** 2) + 0 * Z
        w = 1.0 / 24
        F = np.ones((n, n, n))
        shells = [(0.15, 0.05, -1), (0.25, 0.10, 1), (0.35, 0.10, -1), (0.45, 0.10, 1)]
        for R0, rh, side in shells:
            wall = (R > R0) & (R < R0 + w)
            hole = (r < rh) & ((Z < 0) if side < 0 else (Z > 0))
            F = np.where(wall & ~hole, 0.0, F)
    else:
        raise ValueError(case)
    F = np.ascontiguousarray(np.broadcast_to(F, (n, n, n)), dtype=dtype)
    c = n // 2
    return Problem(f"paper_case{case}", F, h, [(c, c, c, 0.0)], block=16, stride=2 * h,
                   meta={"n": n, "case": case})


# --------------------------------------------------------------------------- small random
def random_problem(seed: int, shape=(16, 16, 16), nsrc: int = 2, flo: float = 0.25,
                   fhi: float = 2.0, dtype=np.float64, block: int = 8, obstacles: float = 0.0,
                   psi0_max: float = 0.0) -> Problem:
    """Random speed in [flo, fhi] per point, nsrc random sources, optional F=0 cells."""
    rng = np.random.default_rng(np.random.SeedSequence([1000, seed]))
    nz, ny, nx = shape
    F = rng.uniform(flo, fhi, size=shape)
    if obstacles > 0:
        F = np.where(rng.random(shape) < obstacles, 0.0, F)
    srcs = []
    for _ in range(nsrc):
        i, j, k = int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))
        v = float(rng.uniform(0, psi0_max)) if psi0_max > 0 else 0.0
        srcs.append((i, j, k, v))
        F[k, j, i] = max(F[k, j, i], flo)  # a source is never inside an obstacle
    h = 1.0 / (max(shape) - 1)
    return Problem(f"random[{seed}]", np.ascontiguousarray(F, dtype=dtype), h, srcs,
                   block=block, stride=2 * h, meta={"seed": seed})
