"""Reference codecs for coefficient storage -- TEST INFRASTRUCTURE ONLY.

The paper never states a precision; storage in BF16 or FP8 with a per-leaf
FP32 scale is this implementation's reading.  Both codecs are written from
their definitions:

* FP8 E4M3FN (OCP 8-bit floating point, v1.0): 1 sign, 4 exponent bits with
  bias 7, 3 mantissa bits; exponent field 0 is subnormal (2^-6 * m/8); no
  infinities; S.1111.111 is NaN; the largest finite magnitude is 448.
  Encoding rounds to nearest, ties to an even mantissa, and saturates at 448.
* BF16: the upper 16 bits of binary32; rounding to nearest, ties to even.

Per-leaf scale: s = max |k| over the leaf's coefficients (BF16) or
max |k| / 448 (E4M3); an all-zero leaf has s = 1.  The scaled value k / s is
formed in FP32 (IEEE division) before rounding.  Dequantised value = s * q.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_table() -> np.ndarray:
    """Value of each of the 256 codes (NaN for 0x7F and 0xFF)."""
    vals = np.zeros(256, dtype=np.float64)
    for code in range(256):
        s = (code >> 7) & 1
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            v = np.nan
        elif e == 0:
            v = 2.0 ** (-6) * (m / 8.0)
        else:
            v = 2.0 ** (e - 7) * (1.0 + m / 8.0)
        vals[code] = -v if s else v
    return vals


def e4m3_encode(x: np.ndarray) -> np.ndarray:
    """Round to nearest E4M3FN code, ties to even mantissa, saturating at 448."""
    x = np.asarray(x, dtype=np.float64)
    table = e4m3_table()
    pos = table[:0x7F]                  # non-negative finite codes 0x00..0x7E, increasing
    mag = np.minimum(np.abs(x), E4M3_MAX)
    hi_i = np.searchsorted(pos, mag, side="left")      # first code >= mag
    hi_i = np.minimum(hi_i, len(pos) - 1)
    lo_i = np.maximum(hi_i - 1, 0)
    exact = pos[hi_i] == mag
    dlo = mag - pos[lo_i]
    dhi = pos[hi_i] - mag
    pick_hi = dhi < dlo
    tie = dhi == dlo
    pick_hi = np.where(tie, (hi_i & 1) == 0, pick_hi)
    code = np.where(exact, hi_i, np.where(pick_hi, hi_i, lo_i)).astype(np.uint8)
    neg = np.signbit(x)
    code = np.where(neg, code | 0x80, code).astype(np.uint8)
    code = np.where(np.isnan(x), np.uint8(0x7F), code).astype(np.uint8)
    return code


def e4m3_decode(code: np.ndarray) -> np.ndarray:
    return e4m3_table()[np.asarray(code, dtype=np.uint8)]


def bf16_encode(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 (ties to even) of float32 values, as uint16 bit patterns."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    lo = (bits >> 16).astype(np.uint32)                # truncation toward zero in magnitude
    lo_val = (lo << 16).view(np.float32).astype(np.float64)
    hi = lo + 1
    hi_val = (hi.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    dlo = np.abs(xv - lo_val)
    dhi = np.abs(hi_val - xv)
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ((lo & 1) == 1))
    out = np.where(pick_hi, hi, lo)
    out = np.where(np.isnan(x), np.uint32(0x7FC0), out)
    return out.astype(np.uint16)


def bf16_decode(code: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(code, dtype=np.uint16).astype(np.uint32) << 16
    return c.view(np.float32).astype(np.float64)


def leaf_scales(coeffs: np.ndarray, kind: str) -> np.ndarray:
    """Per-leaf FP32 scale for coeffs [L][n]."""
    m = np.max(np.abs(coeffs.astype(np.float32)), axis=1).astype(np.float32)
    if kind == "fp8":
        s = (m / np.float32(E4M3_MAX)).astype(np.float32)
    elif kind == "bf16":
        s = m
    else:
        raise ValueError(kind)
    return np.where(m == 0, np.float32(1.0), s).astype(np.float32)


def quantize(coeffs: np.ndarray, kind: str):
    """(codes [L][n], scale [L]).  codes: uint16 (bf16) or uint8 (fp8)."""
    c = np.ascontiguousarray(coeffs, dtype=np.float32)
    s = leaf_scales(c, kind)
    y = (c / s[:, None]).astype(np.float32)
    if kind == "fp8":
        return e4m3_encode(y), s
    return bf16_encode(y), s


def dequantize(codes: np.ndarray, scale: np.ndarray, kind: str) -> np.ndarray:
    q = e4m3_decode(codes) if kind == "fp8" else bf16_decode(codes)
    return scale.astype(np.float64)[:, None] * q
