"""Low-precision edge codes (an extension: the paper stores its per-edge
projections as float, Supplementary F).  Test infrastructure only.

Each rounding is written from the number format itself, in float64:

* bfloat16: 1 sign, 8 exponent, 7 stored mantissa bits (8 significant
  bits); round to nearest, ties to even.
* OCP FP8 E4M3: 1 sign, 4 exponent bits with bias 7, 3 stored mantissa bits;
  normals 2^(e-7) (1 + m/8) for e = 1..15 except the NaN code e = 15, m = 7,
  so the largest finite value is 448; subnormals 2^-6 (m/8); no infinities.
  Round to nearest, ties to even; magnitudes beyond 448 saturate to 448.
* Per-node scale for FP8: s_c = max |u| over the node's codes / 448 (1 when
  all are zero); the stored code is E4M3(u / s_c) and decodes to s_c * value.
"""
from __future__ import annotations

import numpy as np


def _round_to_grid(x: np.ndarray, mant_bits: int, min_exp: int) -> np.ndarray:
    """Nearest value with `mant_bits` stored mantissa bits (exponents below
    min_exp use min_exp's spacing), ties to even."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = x != 0
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # guard log2 rounding at exact powers of two
    e = np.where(2.0 ** e > ax, e - 1, e)
    e = np.where(2.0 ** (e + 1) <= ax, e + 1, e)
    e = np.maximum(e, min_exp)
    q = 2.0 ** (e - mant_bits)
    out[nz] = np.sign(x[nz]) * np.rint(ax / q) * q   # rint: ties to even
    return out


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value of x (finite range only)."""
    return _round_to_grid(x, 7, -126)


E4M3_MAX = 448.0


def round_e4m3(x) -> np.ndarray:
    """Nearest OCP E4M3 value of x, saturating at +-448."""
    y = _round_to_grid(x, 3, -6)
    return np.clip(y, -E4M3_MAX, E4M3_MAX)


def e4m3_values() -> np.ndarray:
    """Value of each of the 256 E4M3 byte codes (NaN for 0x7f and 0xff)."""
    vals = np.empty(256)
    for b in range(256):
        s, e, m = b >> 7, (b >> 3) & 15, b & 7
        if e == 15 and m == 7:
            vals[b] = np.nan
            continue
        v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
        vals[b] = -v if s else v
    return vals


def fp8_node_scale(U: np.ndarray) -> float:
    """Per-node scale of the node's code rows U [deg, r]."""
    amax = float(np.max(np.abs(U))) if U.size else 0.0
    return amax / E4M3_MAX if amax > 0 else 1.0


def quantize_codes(U: np.ndarray, code: str) -> np.ndarray:
    """The decoded value of each stored code for one node's rows U
    [deg, r]: 'f32' rounds to float32, 'bf16' and 'fp8' as above."""
    U = np.asarray(U, dtype=np.float64)
    if code == "f32":
        return U.astype(np.float32).astype(np.float64)
    if code == "bf16":
        return round_bf16(U)
    if code == "fp8":
        s = fp8_node_scale(U)
        return round_e4m3(U / s) * s
    raise ValueError(code)
