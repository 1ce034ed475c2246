"""Shared helpers for the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np

from oracle.conditioning import conditioned_reference, perpendicular_pair  # noqa: F401


def note(msg: str):
    """Name the case before a GPU step, so that a crash log says what ran."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def straddle_err(gpu_rgb: np.ndarray, oracle_rgb2: np.ndarray) -> np.ndarray:
    """Per-ray max-abs error against the closer of the oracle's two
    early-termination outcomes (they coincide unless the FP64 transmittance
    straddles the threshold)."""
    e0 = np.max(np.abs(gpu_rgb - oracle_rgb2[:, 0]), axis=-1)
    e1 = np.max(np.abs(gpu_rgb - oracle_rgb2[:, 1]), axis=-1)
    return np.minimum(e0, e1)


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)


def check_parity(gpu_rgb: np.ndarray, ref: dict, tol: float = 1e-4, max_exempt_frac: float = 0.01):
    """Every well-conditioned ray (spread at 2e-7 within tol) within tol of
    the oracle; ill-conditioned rays rare and within their 1e-6 spread + tol."""
    err = straddle_err(gpu_rgb, ref["rgb"])
    exempt = ref["spread"] > tol
    bad = np.nonzero((~exempt) & (err > tol))[0]
    assert len(bad) == 0, f"{len(bad)} rays above {tol}: worst {err[bad].max():.3e} at ray {bad[np.argmax(err[bad])]}"
    assert exempt.mean() <= max_exempt_frac, f"{exempt.sum()} ill-conditioned rays of {len(err)}"
    if exempt.any():
        over = err[exempt] > ref["spread_wide"][exempt] + tol
        assert not over.any(), "an ill-conditioned ray is further off than its FP64 spread at 1e-6"
    return err, exempt
