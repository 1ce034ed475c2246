"""Coarse occupancy grid -- TEST INFRASTRUCTURE ONLY.

Not from the paper: the empty-space skip of this implementation proves a
stretch of ray empty with a 64^3 bit grid over the unit cube.  Cell
(x, y, z) is set iff some leaf overlaps the cell or one of its 26
neighbours.  Written here as that definition: mark covered cells, then take
the maximum over the 27 shifts.
"""
from __future__ import annotations

import numpy as np

RES = 64


def covered(leaf_dijk: np.ndarray) -> np.ndarray:
    """bool [64][64][64] indexed [z][y][x]: cells some leaf overlaps."""
    occ = np.zeros((RES, RES, RES), bool)
    for d, i, j, k in np.asarray(leaf_dijk, dtype=np.int64):
        # leaf [i, i+1) 2^-d per axis -> coarse cells [lo, hi]
        lo = [int(np.floor(v * RES / 2.0 ** d)) for v in (i, j, k)]
        hi = [int(np.ceil((v + 1) * RES / 2.0 ** d)) - 1 for v in (i, j, k)]
        occ[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    return occ


def dilated(leaf_dijk: np.ndarray) -> np.ndarray:
    occ = covered(leaf_dijk)
    pad = np.pad(occ, 1)
    out = np.zeros_like(occ)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out |= pad[dz:dz + RES, dy:dy + RES, dx:dx + RES]
    return out


def to_words(grid: np.ndarray) -> np.ndarray:
    """bool [z][y][x] -> uint32 [8192], bit (z 64 + y) 64 + x (LSB first)."""
    flat = grid.reshape(-1).astype(np.uint64)
    w = flat.reshape(-1, 32) << np.arange(32, dtype=np.uint64)
    return w.sum(axis=1).astype(np.uint32)
