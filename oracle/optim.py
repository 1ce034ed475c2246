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
