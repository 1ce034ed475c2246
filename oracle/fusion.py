"""PlenOctree fusion (Sec. 3, fine stage; Eq. 3-5) -- TEST INFRASTRUCTURE ONLY.

In the fine stage of the construction, the PlenOctree is rendered from many
views; the points met with transmittance T > 1e-3 are queried from the
radiance field, and every leaf is updated with the transmittance as weight:
    sigma_i = (W_{i-1} sigma_{i-1} + T_i sigma_obs) / (W_{i-1} + T_i)          (Eq. 3)
    z_i     = (W_{i-1} z_{i-1} + T_i SH(d) c(d)) / (W_{i-1} + T_i)             (Eq. 4)
    C_i = C_{i-1} + 1,  W_i = (C_i - 1) / C_i W_{i-1} + T_i / C_i               (Eq. 5)

Readings (the paper leaves these open):
- views are fused one after another; within one view, the transmittance of
  each leaf segment comes from the current values, front to back;
- the points are the leaf segments: a segment [t0, t1) entered with
  transmittance T > tau is observed at its midpoint, and counts with weight
  proportional to its length delta (a sampler that steps along the ray puts
  that many points into the leaf);
- all observations of one leaf in one view make one update: T_i is their
  length-weighted mean transmittance sum(T delta) / sum(delta), and
  T_i sigma_obs, T_i SH c are sum(T delta sigma) / sum(delta) and
  sum(T delta Y c) / sum(delta);
- z_{c,j} is updated with Y_j(d) c_c, the colour projected on the SH basis
  of the view direction (the product SH(theta, phi) c(theta, phi) of Eq. 4);
- the walk stops at the first segment entered with T <= tau.

The radiance field is the analytic stand-in of the library's synthetic
inputs (density and view-dependent colour as closed forms), since the
generalizable network itself is out of scope.

Everything is FP64, one ray and one segment at a time.
"""
from __future__ import annotations

import numpy as np

N_VALUES = 28       # sigma_raw, then z_{c,j} at 1 + 9 c + j
N_ACC = 30          # sum T delta, sum T delta sigma, 27 x sum T delta Y_j c_c, sum delta


def field_sigma(field, x) -> float:
    x = np.asarray(x, dtype=np.float64)
    r2 = ((x[None, :] - np.asarray(field.mu, dtype=np.float64)) ** 2).sum(axis=1)
    w = np.asarray(field.w, dtype=np.float64)
    return float((np.asarray(field.a, dtype=np.float64) * np.exp(-r2 / (2.0 * w * w))).sum())


def field_colour(field, x, d) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    h = np.asarray(field.u, dtype=np.float64) @ x + np.asarray(field.v, dtype=np.float64) @ d \
        + np.asarray(field.b, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-h))


def observe_rays(oracle, tree, values, o, d, field, sigma_scale: float, tau: float):
    """Observation sums of a set of rays (o [n][3], d [n][3]): acc [L][30];
    per leaf, whether one of its segments was entered with T within a
    relative 1e-4 of tau (an FP32 walk may decide that segment the other
    way); and each ray's transmittance where its walk ended."""
    values = np.asarray(values, dtype=np.float64)
    o = np.atleast_2d(np.asarray(o, dtype=np.float64))
    d = np.atleast_2d(np.asarray(d, dtype=np.float64))
    L = values.shape[0]
    acc = np.zeros((L, N_ACC))
    near_tau = np.zeros(L, dtype=bool)
    T_end = np.ones(len(o))
    for r in range(len(o)):
        dn = d[r] / np.linalg.norm(d[r])
        leaf, t0, t1 = tree.trace(o[r], dn)
        if len(leaf) == 0:
            continue
        Y = oracle.sh9(dn)
        T = 1.0
        for l, a, b in zip(leaf, t0, t1):
            if abs(T - tau) <= 1e-4 * tau:
                near_tau[l] = True
            if not T > tau:
                break
            delta = b - a
            x = o[r] + 0.5 * (a + b) * dn
            sig = field_sigma(field, x)
            col = field_colour(field, x, dn)
            w = T * delta
            acc[l, 0] += w
            acc[l, 1] += w * sig
            acc[l, 2:29] += w * np.outer(col, Y).reshape(-1)
            acc[l, 29] += delta
            T *= np.exp(-sigma_scale * max(values[l, 0], 0.0) * delta)
        T_end[r] = T
    return acc, near_tau, T_end


def observe_view(oracle, tree, values, cam, field, sigma_scale: float, tau: float):
    """observe_rays over every pixel ray of a pinhole camera."""
    o, d = oracle.camera_rays(cam)
    acc, near, _ = observe_rays(oracle, tree, values, o, d, field, sigma_scale, tau)
    return acc, near


def apply_view(values, weight, count, acc):
    """Eq. 3-5 once for every leaf observed in the view (sum delta > 0).
    Returns new (values, weight, count)."""
    values = np.array(values, dtype=np.float64, copy=True)
    weight = np.array(weight, dtype=np.float64, copy=True)
    count = np.array(count, dtype=np.int64, copy=True)
    for l in np.nonzero(acc[:, 29] > 0.0)[0]:
        n = acc[l, 29]
        Ti = acc[l, 0] / n
        W = weight[l]
        values[l, 0] = (W * values[l, 0] + acc[l, 1] / n) / (W + Ti)
        values[l, 1:29] = (W * values[l, 1:29] + acc[l, 2:29] / n) / (W + Ti)
        count[l] += 1
        C = count[l]
        weight[l] = (C - 1) / C * W + Ti / C
    return values, weight, count


def fuse_view(oracle, tree, values, weight, count, cam, field, sigma_scale: float, tau: float):
    """One view: observe with the current values, then update.  Returns
    (values, weight, count, acc, near_tau)."""
    acc, near = observe_view(oracle, tree, values, cam, field, sigma_scale, tau)
    v, w, c = apply_view(values, weight, count, acc)
    return v, w, c, acc, near
