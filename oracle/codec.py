"""Bit-width reduction of recorded fields (Section 2) written from the format definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper converts each recorded value to a smaller floating-point type and
converts it back before it is used, so the only error is the conversion
error (Section 2).  This module states that conversion plainly: build the
set of finite values a format can represent from its field widths, then map
every input to the nearest member of that set, ties going to the code with
an even last mantissa bit (IEEE round-to-nearest-even).  Beyond the largest
finite value the format's overflow rule applies (infinity for IEEE-style
formats, the NaN code for the "fn" FP8 format, which has no infinity).

Storage modes used by the gradient oracle:
    fp64                 keep FP64 values (oracle-only reference mode)
    fp32                 round to float32
    fp16, bf16           round to float32, then to the 16-bit format
    fp8_e4m3fn_scaled    round to float32; per block a power-of-two scale
                         s = 2^e, e the smallest integer with 448 * 2^e >= max|x|
                         (clamped to the normal float32 exponent range), codes
                         q = e4m3fn(x / s); decode float32(value(q) * s)
    fp8_e4m3b11fnuz, fp8_e5m2fnuz, fp8_e4m3fnuz, fp8_e4m3, fp8_e3m4, fp8_e4m3fn
                         the unscaled 8-bit types of Section 3 (Fig. 3): round to
                         float32, then straight to the format (no scale).  Names:
                         eXmY = exponent / mantissa bits; "fn" finite with NaN,
                         "fnuz" finite, NaN, unsigned zero; b11 = exponent bias
                         11 (the others use 2^(X-1) - 1, fnuz types one more).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FloatFormat:
    name: str
    exp_bits: int
    man_bits: int
    bias: int
    kind: str        # "ieee": top exponent = inf/nan; "fn": only S.1111.111 is NaN (no inf);
                     # "fnuz": only 1.0000.000 (negative zero) is NaN, no inf, no negative zero

    @property
    def bits(self) -> int:
        return 1 + self.exp_bits + self.man_bits


FP16 = FloatFormat("fp16", 5, 10, 15, "ieee")
BF16 = FloatFormat("bf16", 8, 7, 127, "ieee")
FP8_E4M3FN = FloatFormat("fp8_e4m3fn", 4, 3, 7, "fn")
# the unscaled 8-bit family compared in Section 3 / Fig. 3
FP8_E4M3B11FNUZ = FloatFormat("fp8_e4m3b11fnuz", 4, 3, 11, "fnuz")
FP8_E5M2FNUZ = FloatFormat("fp8_e5m2fnuz", 5, 2, 16, "fnuz")
FP8_E4M3FNUZ = FloatFormat("fp8_e4m3fnuz", 4, 3, 8, "fnuz")
FP8_E4M3 = FloatFormat("fp8_e4m3", 4, 3, 7, "ieee")
FP8_E3M4 = FloatFormat("fp8_e3m4", 3, 4, 3, "ieee")
UNSCALED_FP8 = {f.name: f for f in (FP8_E4M3B11FNUZ, FP8_E5M2FNUZ, FP8_E4M3FNUZ, FP8_E4M3, FP8_E3M4, FP8_E4M3FN)}

STORAGE_BITS = {"fp64": 64, "fp32": 32, "fp16": 16, "bf16": 16, "fp8_e4m3fn_scaled": 8,
                **{name: 8 for name in UNSCALED_FP8}}
FP8_MAX = 448.0


def code_value(fmt: FloatFormat, code: int) -> float:
    """Value of one code from the sign / exponent / mantissa fields (nan / inf for specials)."""
    m_mask = (1 << fmt.man_bits) - 1
    e_max = (1 << fmt.exp_bits) - 1
    sign = -1.0 if (code >> (fmt.exp_bits + fmt.man_bits)) & 1 else 1.0
    e = (code >> fmt.man_bits) & e_max
    m = code & m_mask
    if fmt.kind == "ieee" and e == e_max:
        return sign * math.inf if m == 0 else math.nan
    if fmt.kind == "fn" and e == e_max and m == m_mask:
        return math.nan
    if fmt.kind == "fnuz" and code == 1 << (fmt.exp_bits + fmt.man_bits):
        return math.nan
    if e == 0:
        return sign * (m / (1 << fmt.man_bits)) * 2.0 ** (1 - fmt.bias)
    return sign * (1.0 + m / (1 << fmt.man_bits)) * 2.0 ** (e - fmt.bias)


def _positive_table(fmt: FloatFormat):
    """Non-negative finite codes and values in increasing order, plus the overflow code."""
    half = 1 << (fmt.exp_bits + fmt.man_bits)
    codes, vals = [], []
    for code in range(half):
        v = code_value(fmt, code)
        if math.isfinite(v):
            codes.append(code)
            vals.append(v)
    order = np.argsort(vals, kind="stable")
    codes = np.asarray(codes, np.int64)[order]
    vals = np.asarray(vals, np.float64)[order]
    # the code just above the largest finite one: inf (ieee) or the NaN pattern (fn)
    overflow_code = int(codes[-1]) + 1
    ulp_top = vals[-1] - vals[-2]
    overflow_value = vals[-1] + ulp_top
    return codes, vals, overflow_code, overflow_value


_TABLES = {}


def _table(fmt):
    if fmt.name not in _TABLES:
        _TABLES[fmt.name] = _positive_table(fmt)
    return _TABLES[fmt.name]


def encode(x, fmt: FloatFormat) -> np.ndarray:
    """Round-to-nearest-even codes of x (any float array) in the given format."""
    codes, vals, ov_code, ov_val = _table(fmt)
    x = np.asarray(x, np.float64)
    sign_bit = 1 << (fmt.exp_bits + fmt.man_bits)
    a = np.abs(x)
    # candidate neighbours in the extended table (finite values + the overflow value)
    ext_vals = np.append(vals, ov_val)
    ext_codes = np.append(codes, ov_code)
    hi = np.searchsorted(ext_vals, a, side="left")
    hi = np.clip(hi, 1, ext_vals.size - 1)
    lo = hi - 1
    d_lo = a - ext_vals[lo]
    d_hi = ext_vals[hi] - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (ext_codes[hi] % 2 == 0))
    out = np.where(pick_hi, ext_codes[hi], ext_codes[lo])
    out = np.where(a >= ov_val, ov_code, out)                # at or past the overflow value
    if fmt.kind == "fnuz":                                    # no negative zero; the sign bit alone is NaN
        out = np.where(np.signbit(x) & (out != 0), out | sign_bit, out)
        nan_code = sign_bit
    else:
        out = np.where(np.signbit(x), out | sign_bit, out)
        nan_code = (1 << (fmt.exp_bits + fmt.man_bits)) - 1 if fmt.kind == "fn" else \
            (((1 << fmt.exp_bits) - 1) << fmt.man_bits) | (1 << (fmt.man_bits - 1))
    out = np.where(np.isnan(x), nan_code, out)
    return out.astype(np.int64)


_LUTS = {}


def decode(codes, fmt: FloatFormat) -> np.ndarray:
    """Exact FP64 values of codes."""
    if fmt.name not in _LUTS:
        _LUTS[fmt.name] = np.array([code_value(fmt, c) for c in range(1 << fmt.bits)], np.float64)
    return _LUTS[fmt.name][np.asarray(codes, np.int64)]


# ----------------------------------------------------------------------------
# Per-block power-of-two scale for FP8
# ----------------------------------------------------------------------------

def fp8_scale_exponent(m: float) -> int:
    """Smallest integer e with 448 * 2^e >= m (m >= 0), clamped to [-126, 127]; 0 if m == 0."""
    if m == 0.0:
        return 0
    e = math.ceil(math.log2(m / FP8_MAX))
    # guard the floating log against off-by-one near powers of two
    while FP8_MAX * 2.0 ** (e - 1) >= m:
        e -= 1
    while FP8_MAX * 2.0 ** e < m:
        e += 1
    return max(-126, min(127, e))


def encode_block(x32: np.ndarray, mode: str):
    """Encode one (slice, face, component) block of float32 values.  Returns (codes, scale)."""
    x32 = np.asarray(x32, np.float32)
    if mode == "fp32":
        return x32.copy(), 1.0
    if mode == "fp16":
        return encode(x32, FP16), 1.0
    if mode == "bf16":
        return encode(x32, BF16), 1.0
    if mode == "fp8_e4m3fn_scaled":
        m = float(np.max(np.abs(x32))) if x32.size else 0.0
        s = 2.0 ** fp8_scale_exponent(m)
        return encode(x32.astype(np.float64) / s, FP8_E4M3FN), s
    if mode in UNSCALED_FP8:
        return encode(x32, UNSCALED_FP8[mode]), 1.0
    raise ValueError(mode)


def decode_block(codes, scale: float, mode: str) -> np.ndarray:
    """Decode one block back to float32 values (returned as float64 holding float32 values)."""
    if mode == "fp32":
        return np.asarray(codes, np.float32).astype(np.float64)
    if mode == "fp16":
        return decode(codes, FP16).astype(np.float32).astype(np.float64)
    if mode == "bf16":
        return decode(codes, BF16).astype(np.float32).astype(np.float64)
    if mode == "fp8_e4m3fn_scaled":
        return (decode(codes, FP8_E4M3FN) * scale).astype(np.float32).astype(np.float64)
    if mode in UNSCALED_FP8:
        return decode(codes, UNSCALED_FP8[mode]).astype(np.float32).astype(np.float64)
    raise ValueError(mode)


def roundtrip_block(x: np.ndarray, mode: str) -> np.ndarray:
    """What the reverse pass sees of a recorded block: encode then decode (FP64 mode: identity)."""
    if mode == "fp64":
        return np.asarray(x, np.float64).copy()
    x32 = np.asarray(x, np.float64).astype(np.float32)
    codes, s = encode_block(x32, mode)
    return decode_block(codes, s, mode)
