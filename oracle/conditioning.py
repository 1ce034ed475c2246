"""Conditioning of the FP64 reference under sideways ray shifts -- TEST
INFRASTRUCTURE ONLY.

A ray that crosses a cell face at grazing incidence, or runs along one, has a
colour that is not determined to the parity tolerance by a ray known only to
FP32 accuracy (an FP32 ray from a camera 1.5 units away is placed to about
1e-7).  These helpers measure that from the oracle alone: the spread of a ray
at shift eps is the largest change of its FP64 colour when the ray is moved
sideways by eps.  Rays whose spread at 2e-7 exceeds the tolerance are the
ties of the colour contract; their error is bounded by the spread at 1e-6.
"""
from __future__ import annotations

import numpy as np


def perpendicular_pair(d: np.ndarray):
    """Two unit vectors perpendicular to each (unit) row of d and to each other."""
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    a = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    u = np.cross(d, a)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(d, u)
    return u, v


def conditioned_reference(oracle, otree, coeffs, params, times, o, d, t_idx, eps=(2e-7, 1e-6), n_threads=8,
                          snapshot=None):
    """Oracle render plus each ray's spread at each shift in `eps`: the
    largest change of its FP64 colour (over four sideways shifts of the ray by
    that distance, closest early-termination outcomes compared).
    ref["spread"] is the spread at eps[0], ref["spread_wide"] at eps[-1]."""
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    ref = oracle.render_rays(otree, coeffs, params, times, o, d, t_idx, n_threads=n_threads, snapshot=snapshot)
    u, v = perpendicular_pair(d)
    spreads = []
    for e in eps:
        spread = np.zeros(len(o))
        for s, w in ((1.0, u), (-1.0, u), (1.0, v), (-1.0, v)):
            alt = oracle.render_rays(otree, coeffs, params, times, o + s * e * w, d, t_idx,
                                     n_threads=n_threads, snapshot=snapshot)["rgb"]
            dist = np.full(len(o), np.inf)
            for i in range(2):
                for j in range(2):
                    dist = np.minimum(dist, np.max(np.abs(alt[:, i] - ref["rgb"][:, j]), axis=1))
            spread = np.maximum(spread, dist)
        spreads.append(spread)
    ref["spread"] = spreads[0]
    ref["spread_wide"] = spreads[-1]
    return ref
