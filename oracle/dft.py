"""Building a Fourier PlenOctree from per-frame PlenOctrees -- TEST
INFRASTRUCTURE ONLY.

Sec. 4.2: the per-frame octrees are unified (the union has equal or deeper
leaves than every frame; where a frame's leaf is divided in the union, the
new leaves copy its value), then every union leaf's per-frame values are
turned into Fourier coefficients by the DFT of Eq. 10-12.  Sec. 3: leaves
whose density stays below 1e-3 are filtered out.

Readings:
- frames t = 0 .. T-1 sit at times t (the basis is T-periodic, so the
  paper's t = 1 .. T is the same set);
- the DFT weight is 1/T for i = 0 and 2/T for i >= 1 (the printed 1/T for
  every i returns the non-DC terms at half amplitude, since
  sum_t IDFT_i(t)^2 = T/2 for i >= 1); literal=True keeps the printed 1/T;
- a union leaf that a frame leaves empty gets zeros in that frame;
- pruning drops a union leaf whose sigma is below 1e-3 in every frame.

Everything here is written as the plain definition: sets of cells, explicit
ancestor searches, FP64 sums.
"""
from __future__ import annotations

import numpy as np

N_VALUES = 28          # sigma + 27 SH coefficients per leaf and frame
PRUNE_SIGMA = 1e-3


def _children(cell):
    d, i, j, k = cell
    return [(d + 1, 2 * i + (o & 1), 2 * j + ((o >> 1) & 1), 2 * k + ((o >> 2) & 1)) for o in range(8)]


def _parent(cell):
    d, i, j, k = cell
    return (d - 1, i >> 1, j >> 1, k >> 1)


def union_leaves(frames):
    """frames: list of [n_f][4] (depth, i, j, k) arrays.  Returns the union
    leaves as a sorted list of tuples."""
    leaves = [set(map(tuple, np.asarray(f, dtype=np.int64).tolist())) for f in frames]
    internal = set()
    for L in leaves:
        for c in L:
            p = c
            while p[0] > 0:
                p = _parent(p)
                internal.add(p)
    out = set()
    for L in leaves:
        for c in L:
            stack = [c]
            while stack:
                x = stack.pop()
                if x in internal:
                    stack.extend(_children(x))
                else:
                    out.add(x)
    return sorted(out)


def frame_values_on_union(frame_leaves, frame_values, union):
    """The frame's value at every union leaf: the value of the frame leaf
    that is the union leaf or one of its ancestors, else zeros.
    frame_values [n_f][28].  Returns [n_union][28]."""
    lut = {tuple(c): v for c, v in zip(np.asarray(frame_leaves, dtype=np.int64).tolist(), np.asarray(frame_values))}
    out = np.zeros((len(union), N_VALUES))
    for u, c in enumerate(union):
        x = tuple(c)
        while x[0] > 0:
            if x in lut:
                out[u] = lut[x]
                break
            x = _parent(x)
    return out


def basis(t, period, n):
    """Eq. 8 in FP64."""
    i = np.arange(n)
    return np.where(i % 2 == 0, np.cos(i * np.pi * t / period), np.sin((i + 1) * np.pi * t / period))


def dft(values, n_sigma=31, n_sh_fourier=5, literal=False):
    """values [T][L][28] (sigma, z_{c,j}) at frames t = 0 .. T-1 -> Fourier
    coefficients [L][n_sigma + 27 n_sh_fourier] in the library's order
    (q < n_sigma: k^sigma_q; then 27 blocks of n_sh_fourier for z)."""
    v = np.asarray(values, dtype=np.float64)
    T = v.shape[0]
    B = np.stack([basis(t, float(T), n_sigma) for t in range(T)])        # [T][n_sigma]
    w = np.full(n_sigma, 1.0 / T if literal else 2.0 / T)
    w[0] = 1.0 / T
    ks = np.einsum("tl,ti->li", v[:, :, 0], B * w)
    kz = np.einsum("tlq,ti->lqi", v[:, :, 1:], B[:, :n_sh_fourier] * w[:n_sh_fourier])
    return np.concatenate([ks, kz.reshape(v.shape[1], -1)], axis=1)


def sigma_max(values):
    return np.asarray(values, dtype=np.float64)[:, :, 0].max(axis=0)


def prune(union, values):
    """Indices of the union leaves kept (sigma >= 1e-3 in some frame)."""
    return np.nonzero(sigma_max(values) >= PRUNE_SIGMA)[0]
