"""Reference Adam update -- TEST INFRASTRUCTURE ONLY.

Adam as stated by Kingma and Ba (ICLR 2015, Algorithm 1), in FP64 numpy.  The
paper fine-tunes the coefficients by back-propagation (Sec. 4.3) without
naming an optimiser; Adam is this implementation's reading.
"""
from __future__ import annotations

import numpy as np


def adam(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One step; returns (p, m, v) as new FP64 arrays."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adam_touched(p, g, m, v, step: int, lr: float, record: int, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
    """Lazy Adam over records of `record` values: a record whose gradient is
    zero everywhere keeps its parameters and moments; every other record takes
    the step above (with the global step count).  Returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, record)
    g = np.asarray(g, dtype=np.float64).reshape(-1, record)
    m = np.asarray(m, dtype=np.float64).reshape(-1, record)
    v = np.asarray(v, dtype=np.float64).reshape(-1, record)
    hit = np.any(g != 0.0, axis=1)
    p2, m2, v2 = p.copy(), m.copy(), v.copy()
    p2[hit], m2[hit], v2[hit] = adam(p[hit], g[hit], m[hit], v[hit], step, lr, beta1, beta2, eps)
    return p2.ravel(), m2.ravel(), v2.ravel()
