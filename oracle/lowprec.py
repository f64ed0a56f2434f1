"""Exact emulation, in float64, of the low-precision operand formats used by
the sketch.

The paper computes in FP64 only (Section 5, setup).  The low-precision sketch
is this project's addition, so the oracle reproduces the operand values the
GPU feeds its matrix units, and then does all arithmetic on them in FP64:

  * bf16: 1 sign, 8 exponent, 7 stored mantissa bits; round to nearest,
    ties to even (RNE);
  * fp8 e4m3 (OCP "e4m3fn"): 4 exponent bits (bias 7), 3 mantissa bits,
    subnormals down to 2^-9, largest finite 448, no infinities; RNE with
    saturation to +-448;
  * a residual split of FP32 data into bf16 terms: hi = bf16(a), then each
    further term rounds what is left, a - hi - mid - ..., computed exactly;
  * fp8 block quantisation with power-of-two scales: for each block,
    scale = 2^ceil(log2(amax / 448)) so that a / scale fits e4m3 and
    dequantisation q * scale is exact; the FP32 residual a - q * scale is
    then exact as well;
  * the same block quantisation carried on as T e4m3 terms: term t
    quantises what the earlier terms left, r_t / (scale 16^-t), so that
    a ~ sum_t q_t scale 16^-t (every term an e4m3 value times a power of
    two, every r_t exact in FP32).

All rounding here is from the exact (float64) value in a single step.
"""
from __future__ import annotations

import numpy as np


def round_sig(x, bits):
    """Round float64 values to ``bits`` significant bits, RNE; no exponent
    range limit (bf16 shares the float32 exponent range, so for the values
    that arise here this is the bf16 rounding when bits = 8)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                     # x = m * 2^e, 0.5 <= |m| < 1
    scaled = np.ldexp(m, bits)             # exact
    r = np.rint(scaled)                    # ties to even
    return np.ldexp(r, e - bits)


def round_bf16(x):
    """RNE to bf16 (8 significant bits), exact in float64."""
    return round_sig(x, 8)


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


E4M3_MAX = 448.0
E4M3_MIN_NORMAL_EXP = -6          # smallest normal is 2^-6
E4M3_MANT = 3


def round_e4m3(x):
    """RNE to OCP fp8 e4m3fn, saturating at +-448; subnormal spacing 2^-9."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    m, e = np.frexp(ax)                      # ax = m 2^e, 0.5 <= m < 1
    # exponent of the leading bit is e-1; normals have e-1 >= -6
    lead = np.maximum(e - 1, E4M3_MIN_NORMAL_EXP)
    quantum = np.ldexp(1.0, lead - E4M3_MANT)     # spacing at this binade
    r = np.rint(ax / quantum) * quantum           # ax/quantum exact (power of 2)
    r = np.minimum(r, E4M3_MAX)
    r = np.where(ax == 0, 0.0, r)
    return np.copysign(r, x)


def split_bf16(a32, terms):
    """Split FP32 data into ``terms`` bf16 terms.  a32 must hold FP32 values
    (as float64 or float32).  Returns a list of float64 arrays; the sum of the
    terms equals a32 up to the part below the last term's rounding."""
    a = np.asarray(a32, dtype=np.float64)
    if not np.array_equal(a, a.astype(np.float32).astype(np.float64)):
        raise ValueError("split_bf16 expects values exactly representable in FP32")
    out = []
    rem = a.copy()
    for _ in range(terms):
        t = round_bf16(rem)
        out.append(t)
        rem = rem - t          # exact: both are FP32 values, difference fits FP32
    return out


def pow2_scale(amax):
    """Power-of-two scale s with amax / s <= 448: s = 2^ceil(log2(amax/448));
    s = 1 for an all-zero block."""
    amax = np.asarray(amax, dtype=np.float64)
    with np.errstate(divide="ignore"):
        e = np.ceil(np.log2(np.where(amax > 0, amax / E4M3_MAX, 1.0)))
    # log2 of a float64 may be off by an ulp at exact powers of two: fix up
    s = np.ldexp(1.0, e.astype(np.int64))
    too_small = amax / s > E4M3_MAX
    s = np.where(too_small, s * 2.0, s)
    half = s / 2.0
    can_halve = (amax > 0) & (amax / half <= E4M3_MAX)
    s = np.where(can_halve, half, s)
    return np.where(amax > 0, s, 1.0)


def quantize_e4m3_blocks(a, block_rows, block_cols):
    """Quantise a 2-D float64 array (FP32-exact values) to e4m3 with one
    power-of-two scale per (block_rows x block_cols) tile.  Returns
    (dequantised values, scales with shape (ceil(m/br), ceil(n/bc)))."""
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    gm, gn = -(-m // block_rows), -(-n // block_cols)
    pad = np.zeros((gm * block_rows, gn * block_cols))
    pad[:m, :n] = np.abs(a)
    amax = pad.reshape(gm, block_rows, gn, block_cols).max(axis=(1, 3))
    scales = pow2_scale(amax)
    s_full = np.repeat(np.repeat(scales, block_rows, axis=0), block_cols, axis=1)[:m, :n]
    q = round_e4m3(a / s_full)
    return q * s_full, scales


E4M3_TERM_SHIFT = 16.0             # term t of the multi-term split uses scale * 16^-t


def quantize_e4m3_terms(a, block_rows, block_cols, terms):
    """Quantise a 2-D float64 array (FP32-exact values) to ``terms`` e4m3
    terms with one power-of-two scale s per (block_rows x block_cols) tile:
    r_0 = a, q_t = e4m3(r_t / (s 16^-t)) (RNE), r_{t+1} = r_t - q_t s 16^-t.
    After term 0, |r_1| <= 16 s (half a step of e4m3 at 448), so
    r_1 / (s / 16) <= 256 and no later term saturates.  Returns (the list of
    dequantised terms q_t s 16^-t, the tile scales)."""
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    gm, gn = -(-m // block_rows), -(-n // block_cols)
    pad = np.zeros((gm * block_rows, gn * block_cols))
    pad[:m, :n] = np.abs(a)
    amax = pad.reshape(gm, block_rows, gn, block_cols).max(axis=(1, 3))
    scales = pow2_scale(amax)
    s_full = np.repeat(np.repeat(scales, block_rows, axis=0), block_cols, axis=1)[:m, :n]
    out = []
    rem = a.copy()
    for t in range(terms):
        st = s_full / E4M3_TERM_SHIFT ** t          # exact: powers of two
        d = round_e4m3(rem / st) * st
        out.append(d)
        rem = rem - d                                # exact in FP32 (and here)
    return out, scales


def round_dtype(x, dtype):
    """Round exact values to the named operand format."""
    if dtype == "f64":
        return np.asarray(x, dtype=np.float64)
    if dtype == "f32":
        return round_f32(x)
    if dtype == "bf16":
        return round_bf16(x)
    if dtype in ("fp8", "fp8x"):
        return round_e4m3(x)
    raise ValueError(dtype)
