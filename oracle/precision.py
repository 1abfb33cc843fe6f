"""Rounding to reduced-precision leaf formats, for emulating reduced-precision leaves.

These set tolerances for the reduced-precision paths; they are never the
parity reference.  Each is the plain definition of round-to-nearest-even onto
the format's grid:

  bf16:  1 sign, 8 exponent, 7 fraction bits (float32 with the low 16 bits
         cleared after rounding to nearest even on bit 16);
  f16:   IEEE binary16 (numpy's float16 conversion is correctly rounded);
  e4m3:  OCP FP8 E4M3FN: bias 7, 3 fraction bits, largest finite 448, no
         infinities, subnormal spacing 2^-9; values beyond 448 saturate here.

split_hi_lo(x, fmt) returns hi = rn(x), lo = rn(x - hi) (the residual computed
in float64, which is exact for float32 x and these formats).

Pins: tests compare bf16 / f16 / e4m3 rounding with torch's CPU casts
(an independent implementation) on random and edge values.
"""

import numpy as np


def round_bf16(x):
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32)


def round_f16(x):
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float32)


def round_e4m3(x, saturate=True):
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    out = np.zeros_like(a)
    nz = a > 0
    e = np.floor(np.log2(np.where(nz, a, 1.0)))
    e = np.maximum(e, -6.0)              # below 2^-6 the grid is the subnormal one
    step = 2.0 ** (e - 3)
    q = a / step
    r = np.floor(q)
    frac = q - r
    r = r + ((frac > 0.5) | ((frac == 0.5) & (np.mod(r, 2) == 1)))
    out = np.where(nz, r * step, 0.0)
    if saturate:
        out = np.minimum(out, 448.0)
    return (np.sign(x) * out).astype(np.float32)


ROUND = {"bf16": round_bf16, "f16": round_f16, "e4m3": round_e4m3}


def decode_e4m3(codes):
    """Values of OCP E4M3FN byte codes: sign bit 7, exponent bits 6..3 (bias 7), fraction
    bits 2..0; exponent 0 is subnormal (f * 2^-9); 0x7F and 0xFF are NaN."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    e = (c >> 3) & 15
    f = c & 7
    mag = np.where(e == 0, f * 2.0 ** -9, (8 + f) * 2.0 ** (e - 10))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return np.where(c & 0x80, -mag, mag)


def split_e4m3_scaled(y):
    """The fp8 leaf split of an already scaled operand y (|y| <= 448): hi = rn_e4m3(y) and
    lo = rn_e4m3(16 (y - hi)), so that y ~ hi + lo / 16 (y - hi computed in float64, exact
    for float32 y)."""
    y = np.asarray(y, dtype=np.float64)
    hi = round_e4m3(y).astype(np.float64)
    lo = round_e4m3(16.0 * (y - hi)).astype(np.float64)
    return hi, lo


def split_hi_lo(x, fmt="bf16"):
    rn = ROUND[fmt]
    x = np.asarray(x, dtype=np.float32)
    hi = rn(x)
    lo = rn((x.astype(np.float64) - hi.astype(np.float64)).astype(np.float32))
    return hi, lo


def path_norms(schemes, side):
    """Per leaf (r_0 slowest), the product over levels of the 1-norm of the coefficient
    column of U (side "A") or V (side "B") used at that level.  Folding only permutes
    and flips signs, so this bounds |leaf operand| / max|input| for every draw."""
    norms = [np.sum(np.abs(np.asarray(s[0 if side == "A" else 1], np.float64)), axis=(0, 1)) for s in schemes]
    g = np.ones(1)
    for nr in norms:
        g = (g[:, None] * nr[None, :]).reshape(-1)
    return g


def leaf_exponent(maxabs, G, target=32768.0):
    """e = floor(log2(target / (G maxabs))) evaluated in float32 (0 when the bound is 0),
    clamped to [-120, 120]: the power-of-two scale of an f16 leaf operand."""
    bound = np.float32(G) * np.float32(maxabs)
    if not (bound > 0 and np.isfinite(bound)):
        return 0
    q = np.float32(target) / bound
    _, x = np.frexp(q)
    return int(min(max(int(x) - 1, -120), 120))

