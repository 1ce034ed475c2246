"""Brute-force numpy checkers for the oracle -- TEST INFRASTRUCTURE ONLY.

These take a different route to the same quantities as the C oracle, so that
a mistake in one shows up as a disagreement:

* `slab_segments` intersects the ray with every leaf box separately (no DDA,
  no point location) and sorts the hits;
* `dense_render` approximates the volume-rendering integral by a midpoint
  Riemann sum over many tiny steps, locating each sample point by scanning the
  leaf boxes, instead of using the exact per-segment closed form.

Leaf evaluation here is written from the paper directly (Eq. 7, 8, 9 for
density and SH coefficients; Eq. 1 for colour, with the SH basis taken from
scipy's complex spherical harmonics).
"""
from __future__ import annotations

import math

import numpy as np


def leaf_boxes(dijk: np.ndarray):
    d = dijk[:, 0].astype(np.float64)
    size = 2.0 ** (-d)
    lo = dijk[:, 1:4].astype(np.float64) * size[:, None]
    hi = lo + size[:, None]
    return lo, hi


def slab_segments(dijk: np.ndarray, o, d):
    """Every leaf box the ray crosses with positive length, sorted by entry."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    lo, hi = leaf_boxes(dijk)
    tmin = np.zeros(len(dijk))
    tmax = np.full(len(dijk), np.inf)
    ok = np.ones(len(dijk), dtype=bool)
    for a in range(3):
        if d[a] == 0.0:
            ok &= (o[a] >= lo[:, a]) & (o[a] < hi[:, a])
            continue
        t1 = (lo[:, a] - o[a]) / d[a]
        t2 = (hi[:, a] - o[a]) / d[a]
        tmin = np.maximum(tmin, np.minimum(t1, t2))
        tmax = np.minimum(tmax, np.maximum(t1, t2))
    ok &= tmax > tmin
    idx = np.nonzero(ok)[0]
    order = np.argsort(tmin[idx], kind="stable")
    idx = idx[order]
    return idx, tmin[idx], tmax[idx]


def chord_length(lo, hi, o, d):
    """Length of a unit-direction ray inside one box (0 if it misses)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    t0, t1 = 0.0, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] <= o[a] <= hi[a]):
                return 0.0
            continue
        u = (lo[a] - o[a]) / d[a]
        v = (hi[a] - o[a]) / d[a]
        t0 = max(t0, min(u, v))
        t1 = min(t1, max(u, v))
    return max(0.0, t1 - t0)


def fourier_basis(t: float, period: float, n: int) -> np.ndarray:
    """Eq. 8: cos(i pi t / T) for even i, sin((i+1) pi t / T) for odd i."""
    i = np.arange(n)
    return np.where(i % 2 == 0, np.cos(i * np.pi * t / period), np.sin((i + 1) * np.pi * t / period))


def real_sh9_scipy(d) -> np.ndarray:
    """Real SH of degree <= 2 built from scipy's complex harmonics (which
    carry the Condon-Shortley phase): Y_l0 = Y_l^0, Y_lm = sqrt2 Re Y_l^m for
    m > 0 and sqrt2 Im Y_l^|m| for m < 0; index j = l^2 + l + m."""
    from scipy.special import sph_harm_y
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    theta = math.acos(max(-1.0, min(1.0, d[2])))
    phi = math.atan2(d[1], d[0])
    out = np.zeros(9)
    for l in range(3):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                v = y.real
            elif m > 0:
                v = math.sqrt(2.0) * y.real
            else:
                v = math.sqrt(2.0) * y.imag
            out[l * l + l + m] = v
    return out


def leaf_sigma_rgb(k: np.ndarray, t: float, d, period=60.0, n_sigma=31, n_sh_fourier=5,
                   sigma_scale=64.0):
    """sigma_eff and RGB of one leaf at time t, viewed along d."""
    b = fourier_basis(t, period, max(n_sigma, n_sh_fourier))
    sraw = float(np.dot(k[:n_sigma], b[:n_sigma]))                      # Eq. 7
    kz = k[n_sigma:].reshape(3, 9, n_sh_fourier)
    z = kz @ b[:n_sh_fourier]                                           # Eq. 9
    Y = real_sh9_scipy(d)
    rgb = 1.0 / (1.0 + np.exp(-(z @ Y)))                                # Eq. 1
    return sigma_scale * max(sraw, 0.0), rgb


def dense_render(dijk: np.ndarray, coeffs: np.ndarray, o, d, t: float, h: float,
                 bg=(0.0, 0.0, 0.0), **kw):
    """Midpoint Riemann sum of the volume-rendering integral with step h."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    idx, t0s, t1s = slab_segments(dijk, o, d)
    if len(idx) == 0:
        return np.asarray(bg, dtype=np.float64).copy(), 1.0
    lo, hi = leaf_boxes(dijk)
    cache = {}
    a, b = t0s.min(), t1s.max()
    n = max(1, int(math.ceil((b - a) / h)))
    step = (b - a) / n
    T = 1.0
    C = np.zeros(3)
    for s in range(n):
        tm = a + (s + 0.5) * step
        p = o + tm * d
        inside = np.nonzero(np.all((p >= lo[idx]) & (p < hi[idx]), axis=1))[0]
        if len(inside) == 0:
            continue
        l = int(idx[inside[0]])
        if l not in cache:
            cache[l] = leaf_sigma_rgb(coeffs[l].astype(np.float64), t, d, **kw)
        sigma, rgb = cache[l]
        alpha = 1.0 - math.exp(-sigma * step)
        C += T * alpha * rgb
        T *= 1.0 - alpha
    return C + T * np.asarray(bg, dtype=np.float64), T
