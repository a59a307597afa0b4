"""Bit-level rounding emulators for the reduced storage formats.

TEST INFRASTRUCTURE ONLY (see ofrr_oracle.py).  Written from the IEEE-754 /
OCP format definitions; round-to-nearest, ties to even, for every
conversion (the paper does not name a rounding mode; RNE is the IEEE
default).

* bfloat16: the upper 16 bits of an FP32 word (8 exponent bits, 7 stored
  mantissa bits).
* float16: IEEE binary16 (numpy's own conversion is RNE).
* float8 e4m3fn (OCP 8-bit floating point): 1 sign, 4 exponent (bias 7),
  3 mantissa bits, no infinities, S.1111.111 is NaN, largest finite 448,
  subnormals m/8 * 2^-6; out-of-range values saturate to +-448.
"""
from __future__ import annotations

import numpy as np


def f32_to_bf16_bits(x) -> np.ndarray:
    """FP32 -> bfloat16 bit patterns (uint16), round to nearest even."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x0040, r)  # keep NaN quiet
    return r.astype(np.uint16)


def bf16_bits_to_f32(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 and return the value as FP32 (shape kept)."""
    x = np.asarray(x, dtype=np.float32)
    return bf16_bits_to_f32(f32_to_bf16_bits(x).ravel(order="K")).reshape(x.shape)


def round_f16(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def _e4m3_table():
    """All 127 non-negative finite e4m3fn values, ascending, with codes."""
    codes = np.arange(0, 0x7F, dtype=np.int64)  # 0x7F is NaN
    e = codes >> 3
    m = codes & 7
    val = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))
    return val, codes


_E4M3_VAL, _E4M3_CODE = _e4m3_table()
E4M3_MAX = float(_E4M3_VAL[-1])  # 448


def f32_to_e4m3_bits(x) -> np.ndarray:
    """FP32 -> e4m3fn codes (uint8), nearest value, ties to the even code,
    saturating to +-448; NaN -> 0x7F."""
    f = np.asarray(x, dtype=np.float64)
    a = np.abs(f)
    sign = (np.signbit(f)).astype(np.uint8) << 7
    a_sat = np.minimum(a, E4M3_MAX)
    hi = np.searchsorted(_E4M3_VAL, a_sat, side="left")
    hi = np.clip(hi, 0, _E4M3_VAL.size - 1)
    lo = np.clip(hi - 1, 0, _E4M3_VAL.size - 1)
    dlo = a_sat - _E4M3_VAL[lo]
    dhi = _E4M3_VAL[hi] - a_sat
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (_E4M3_CODE[hi] % 2 == 0))
    code = np.where(pick_hi, _E4M3_CODE[hi], _E4M3_CODE[lo]).astype(np.uint8)
    code = np.where(np.isnan(f), np.uint8(0x7F), code | sign)
    return code.astype(np.uint8)


# Smallest and largest exponent of a block scale: 2^k with k in [-126, 127]
# is a normal FP32 number, its reciprocal too, and it is an E8M0 scale
# byte (OCP microscaling formats: bias 127, 0xFF reserved for NaN).
SCALE_EXP_MIN, SCALE_EXP_MAX = -126, 127


def e4m3_block_scale(amax: float) -> float:
    """Power-of-two scale of one FP8 block: the smallest 2^k, k >= -126,
    with amax / 2^k <= 448 (the largest finite e4m3fn value), so that every
    scaled entry is in range and the division by the scale is exact; 1 for
    an all-zero block.  Found by walking k from an exact starting point
    (frexp gives amax = m 2^e with m in [0.5, 1), so amax <= 2^e)."""
    amax = float(amax)
    if not amax > 0.0:
        return 1.0
    _, e = np.frexp(amax)
    k = max(int(e), SCALE_EXP_MIN)  # amax / 2^k <= amax / 2^e <= 1 <= 448
    while k - 1 >= SCALE_EXP_MIN and amax / 2.0 ** (k - 1) <= E4M3_MAX:
        k -= 1
    assert k <= SCALE_EXP_MAX
    return 2.0 ** k


def fp8_block_quantize(A, block: int = 32):
    """Per-block e4m3fn quantisation of a 2-D FP32 array: each block x block
    tile gets the scale e4m3_block_scale(amax of the tile) and the codes
    e4m3fn(A / scale).  Returns (codes uint8, scales float32 of shape
    (ceil(rows/block), ceil(cols/block)))."""
    A = np.asarray(A, dtype=np.float32)
    rows, cols = A.shape
    br, bc = -(-rows // block), -(-cols // block)
    scales = np.ones((br, bc), dtype=np.float32)
    codes = np.zeros((rows, cols), dtype=np.uint8)
    for i in range(br):
        for j in range(bc):
            t = A[i * block:(i + 1) * block, j * block:(j + 1) * block]
            s = e4m3_block_scale(np.max(np.abs(t)) if t.size else 0.0)
            scales[i, j] = s
            codes[i * block:(i + 1) * block, j * block:(j + 1) * block] = \
                f32_to_e4m3_bits(t.astype(np.float64) / s)
    return codes, scales


def fp8_colblock_quantize(V, block: int = 32):
    """e4m3fn quantisation of a 2-D FP32 array with one scale per `block`
    consecutive rows of each column (e4m3_block_scale of the segment's
    amax).  Returns the dequantised values (codes * scale) as float64."""
    V = np.asarray(V, dtype=np.float32)
    out = np.zeros(V.shape, dtype=np.float64)
    rows, cols = V.shape
    for j in range(cols):
        for r0 in range(0, rows, block):
            seg = V[r0:r0 + block, j]
            s = e4m3_block_scale(np.max(np.abs(seg)) if seg.size else 0.0)
            codes = f32_to_e4m3_bits(seg.astype(np.float64) / s)
            out[r0:r0 + block, j] = e4m3_bits_to_f32(codes).astype(np.float64) * s
    return out


def e4m3_bits_to_f32(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    mag = b & 0x7F
    out = np.where(mag == 0x7F, np.nan, _E4M3_VAL[np.minimum(mag, 0x7E)])
    out = np.where(b & 0x80, -out, out)
    return out.astype(np.float32)
