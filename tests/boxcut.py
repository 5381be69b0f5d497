"""Box restriction used to compare a large solve with the single-heap oracle.

The single-heap method accepts points in increasing psi, and a point's value is
computed only from accepted neighbours with smaller values (Sec. 2.1, Alg. 2-4).
Solve the same speed on a box that holds the sources: up to the first acceptance
of a point in the box's boundary layer (the cells next to a box face that is not
also a face of the grid) both runs perform the same operations, so every box
point whose box value is strictly below the smallest boundary-layer value has
the value the whole-grid solve gives it.
"""
import numpy as np


def box_origin(src, shape, box):
    """Lower corner (i, j, k) of a box of side `box` centred on src, clipped to the grid."""
    nz, ny, nx = shape
    return [min(max(c - box // 2, 0), n - box) for c, n in zip(src[:3], (nx, ny, nz))]


def box_slices(lo, box):
    return (slice(lo[2], lo[2] + box), slice(lo[1], lo[1] + box), slice(lo[0], lo[0] + box))


def exact_region(box_psi, lo, shape):
    """Mask of box points whose value equals the whole-grid single-heap value."""
    nz, ny, nx = shape
    box = box_psi.shape[0]
    layer = np.zeros(box_psi.shape, dtype=bool)
    for ax, o, n in ((2, lo[0], nx), (1, lo[1], ny), (0, lo[2], nz)):
        idx = [slice(None)] * 3
        if o > 0:
            idx[ax] = 0
            layer[tuple(idx)] = True
        if o + box < n:
            idx[ax] = box - 1
            layer[tuple(idx)] = True
    if not layer.any():
        return np.isfinite(box_psi)
    m = box_psi[layer].min()
    return box_psi < m
