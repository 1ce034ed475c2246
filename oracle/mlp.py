"""Reference proposal network -- TEST INFRASTRUCTURE ONLY.

The paper has no proposal network; this is the learned empty-space skipper
of this implementation, written plainly in FP64 numpy so that the GPU
forward, backward and training kernels can be checked against it.

Network: positional encoding gamma(x) = (sin(2^f pi x), cos(2^f pi x)),
f < 6, of 7 inputs -- the ray's entry point into the unit cube (3), its unit
direction (3) and t / T wrapped to [0, 1) (1) -- feature index
12 c + 2 f + {0: sin, 1: cos}; then 84 -> 64 -> 64 -> 3 with ReLU on the
hidden layers.  Output 0 is a hit logit, outputs 1 and 2 pass through a
sigmoid to give s_in and s_out, fractions of the ray's chord through the
cube.

Loss per ray (mean over the batch): binary cross-entropy on the hit logit;
for rays that hit, pinball losses rho_q(y - yhat) = (y - yhat)(q - [y < yhat])
with q = 0.1 on s_in and q = 0.9 on s_out (an early entry and a late exit are
the cheap mistakes).
"""
from __future__ import annotations

import numpy as np

N_IN = 7
N_FREQ = 6
N_PE = N_IN * 2 * N_FREQ      # 84
HIDDEN = 64
N_OUT = 3
Q_IN = 0.1
Q_OUT = 0.9


def init_weights(seed: int = 7):
    """He-normal weights, zero biases; W stored as [in][out]."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_PE, HIDDEN)) * np.sqrt(2.0 / N_PE)
    W2 = rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN)
    W3 = rng.standard_normal((HIDDEN, N_OUT)) * np.sqrt(2.0 / HIDDEN)
    return {"W1": W1, "b1": np.zeros(HIDDEN), "W2": W2, "b2": np.zeros(HIDDEN),
            "W3": W3, "b3": np.zeros(N_OUT)}


def encode(inputs: np.ndarray) -> np.ndarray:
    """inputs [n][7] -> gamma [n][84]."""
    x = np.asarray(inputs, dtype=np.float64)
    out = np.zeros((x.shape[0], N_PE))
    for c in range(N_IN):
        for f in range(N_FREQ):
            a = (2.0 ** f) * np.pi * x[:, c]
            out[:, 12 * c + 2 * f] = np.sin(a)
            out[:, 12 * c + 2 * f + 1] = np.cos(a)
    return out


def forward(w, inputs: np.ndarray):
    """Returns (outputs [n][3], cache)."""
    g = encode(inputs)
    z1 = g @ w["W1"] + w["b1"]
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ w["W2"] + w["b2"]
    a2 = np.maximum(z2, 0.0)
    o = a2 @ w["W3"] + w["b3"]
    return o, (g, z1, a1, z2, a2)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def loss_and_grad_out(o: np.ndarray, labels: np.ndarray):
    """labels [n][3] = (hit, s_in, s_out).  Returns (mean loss, dL/do [n][3])."""
    n = o.shape[0]
    y = labels[:, 0]
    hit = y > 0.5
    l0 = np.maximum(o[:, 0], 0.0) - y * o[:, 0] + np.log1p(np.exp(-np.abs(o[:, 0])))
    g = np.zeros_like(o)
    g[:, 0] = sigmoid(o[:, 0]) - y
    loss = l0.copy()
    for j, q in ((1, Q_IN), (2, Q_OUT)):
        s = sigmoid(o[:, j])
        u = labels[:, j] - s
        w = q - (u < 0).astype(np.float64)
        loss += np.where(hit, u * w, 0.0)
        g[:, j] = np.where(hit, -w * s * (1.0 - s), 0.0)
    return float(loss.mean()), g / n


def backward(w, cache, g_out: np.ndarray):
    """Gradients of sum(g_out * o) w.r.t. every weight."""
    g, z1, a1, z2, a2 = cache
    grads = {"W3": a2.T @ g_out, "b3": g_out.sum(0)}
    d2 = (g_out @ w["W3"].T) * (z2 > 0)
    grads["W2"] = a1.T @ d2
    grads["b2"] = d2.sum(0)
    d1 = (d2 @ w["W2"].T) * (z1 > 0)
    grads["W1"] = g.T @ d1
    grads["b1"] = d1.sum(0)
    return grads


def round_fp16(w):
    """The weights as FP16 values (the inference precision), back in FP64."""
    return {k: np.asarray(v, dtype=np.float16).astype(np.float64) for k, v in w.items()}


def ray_inputs(o: np.ndarray, d: np.ndarray, t: np.ndarray, period: float = 60.0):
    """Network inputs of rays: entry point into [0,1]^3 (the origin if inside),
    unit direction, t / T mod 1.  Rays that miss the cube get their origin."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (0.0 - o) / d
        t2 = (1.0 - o) / d
    lo = np.where(d == 0, -np.inf, np.minimum(t1, t2))
    lo = np.nanmax(np.where(np.isnan(lo), -np.inf, lo), axis=1)
    t_in = np.maximum(lo, 0.0)
    e = o + t_in[:, None] * d
    tau = np.mod(np.asarray(t, dtype=np.float64) / period, 1.0)
    return np.concatenate([e, d, tau[:, None]], axis=1)


# Flat parameter vector: [85][64], [65][64], [65][3] row-major matrices end to
# end (input index major), the last row of each the layer's bias.
N_PARAMS = (N_PE + 1) * HIDDEN + (HIDDEN + 1) * HIDDEN + (HIDDEN + 1) * N_OUT   # 9795


def to_flat(w) -> np.ndarray:
    parts = [np.vstack([w["W1"], w["b1"][None]]), np.vstack([w["W2"], w["b2"][None]]),
             np.vstack([w["W3"], w["b3"][None]])]
    return np.concatenate([p.ravel() for p in parts])


def from_flat(p: np.ndarray):
    p = np.asarray(p, dtype=np.float64)
    a = (N_PE + 1) * HIDDEN
    b = a + (HIDDEN + 1) * HIDDEN
    L1 = p[:a].reshape(N_PE + 1, HIDDEN)
    L2 = p[a:b].reshape(HIDDEN + 1, HIDDEN)
    L3 = p[b:b + (HIDDEN + 1) * N_OUT].reshape(HIDDEN + 1, N_OUT)
    return {"W1": L1[:-1].copy(), "b1": L1[-1].copy(), "W2": L2[:-1].copy(), "b2": L2[-1].copy(),
            "W3": L3[:-1].copy(), "b3": L3[-1].copy()}


def _f16(x):
    return np.asarray(x, dtype=np.float16).astype(np.float64)


def forward_fp16(w, inputs: np.ndarray):
    """Inference-precision forward: FP16 weights (round to nearest even), FP16
    layer inputs (the encoding and each hidden activation after ReLU), biases
    as given, exact accumulation."""
    g = _f16(encode(inputs))
    a1 = _f16(np.maximum(g @ _f16(w["W1"]) + w["b1"], 0.0))
    a2 = _f16(np.maximum(a1 @ _f16(w["W2"]) + w["b2"], 0.0))
    return a2 @ _f16(w["W3"]) + w["b3"]


def magnitude(w, inputs: np.ndarray) -> np.ndarray:
    """Per-output scale sum |terms| propagated through the layers with
    absolute weights: the quantity FP rounding errors are proportional to."""
    g = np.abs(encode(inputs))
    m1 = g @ np.abs(w["W1"]) + np.abs(w["b1"])
    m2 = m1 @ np.abs(w["W2"]) + np.abs(w["b2"])
    return m2 @ np.abs(w["W3"]) + np.abs(w["b3"])
