"""FP32 -> FP16 quantisation rules, modelled exactly.

Paper passages followed:
  * Round-to-nearest-even (RN), the hardware conversion (Section 2.3; Section
    4.2, first rounding approach).
  * Exact stochastic rounding (SR): x in [x-, x+] goes to x+ with probability
    (x - x-)/(x+ - x-) (Section 2.3).  Realised as in Section 4.2: take the
    FP16 values rounded down and up, their gap D and the distance E of x above
    the lower one; draw u from 24 random bits, u' = u * 2**-24 in [0, 1); the
    result is the upper value when u' * D < E, else the lower one.
  * Dithered rounding: Q(x + xi) with zero-mean uniform xi of about one ULP,
    scaled with x (Section 2.3; Section 4.2, dithering paragraph):
        noise  = (u' - 1/2) * (x * F)
        result = RN16(x + noise)   with the add done as one FMA
    The paper leaves F (its ULP scale factor) unset; this library reads it as
    F = 2**-10, the FP16 machine epsilon, so |noise| < |x| 2**-11 <= 1 ULP.

Readings where the paper is silent:
  * SR when |x| > 65504 (largest finite FP16): behave as RN (the up/down
    construction degenerates at the overflow boundary).
  * NaN stays NaN under every rule; +-inf stays +-inf.
  * FP16 subnormals are kept (no flush to zero) on both sides.

Everything is computed with integers on the FP32 bit pattern (no floating
point decides a rounding), so results are exact.  Pinned by: numpy's
float32 -> float16 cast for RN (library conversion, all rounding cases);
directed rounding bracketing (rd <= x <= ru, adjacent FP16 values); the
exhaustive count of u values that round up (SR is unbiased to 2**-24); libm
fmaf for the fused multiply-add of the dither; the closed-form mean of the
dither over u.
"""
from __future__ import annotations

from fractions import Fraction
import math

import numpy as np

F16_MAX = 65504.0
DITHER_F = 2.0 ** -10
U24 = 0xFFFFFF
NEAREST, TRUNC, CEIL = 0, 1, 2


def _parts(x):
    """Split FP32 or FP64 values into sign, |x| = M * 2**E (M integer) and the
    FP16 spacing exponent te at |x|; shift = te - E low bits of M to drop."""
    x = np.asarray(x)
    if x.dtype == np.float64:
        bits = x.view(np.uint64)
        neg = (bits >> np.uint64(63)).astype(np.int64)
        ex = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64)
        f = (bits & np.uint64((1 << 52) - 1)).astype(np.int64)
        M = np.where(ex > 0, f | (1 << 52), f)
        E = np.maximum(ex, 1) - 1075
        binade = ex - 1023
        top = 0x7FF
    else:
        x = x.astype(np.float32)
        bits = x.view(np.uint32).astype(np.int64)
        neg = (bits >> 31) & 1
        ex = (bits >> 23) & 0xFF
        f = bits & 0x7FFFFF
        M = np.where(ex > 0, f | (1 << 23), f)
        E = np.maximum(ex, 1) - 150
        binade = ex - 127
        top = 0xFF
    te = np.maximum(binade, -14) - 10
    shift = te - E                                   # >= 13 for FP32, >= 42 for FP64
    special = ex == top
    return neg, special, f, M, te, shift


def _round_mag(M, shift, how):
    """Round M / 2**shift to an integer: how = NEAREST (ties even), TRUNC, CEIL.
    M < 2**53 and shift >= 1, so a shift of 60 already means "everything"."""
    sh = np.minimum(shift, 60)
    q = M >> sh
    r = M - (q << sh)
    half = np.left_shift(np.int64(1), sh - 1)
    up_near = (r > half) | ((r == half) & ((q & 1) == 1))
    up_ceil = r > 0
    return q + np.where(how == NEAREST, up_near, np.where(how == CEIL, up_ceil, False))


def _to_f16(x, mode_pos, mode_neg):
    """Round FP32 or FP64 x to FP16; magnitude rounding `mode_pos` for
    non-negative x and `mode_neg` for negative x.  Returns a float16 array."""
    neg, special, f, M, te, shift = _parts(x)
    how = np.where(neg == 1, mode_neg, mode_pos)
    k = _round_mag(M, shift, how)
    mag = k.astype(np.float64) * np.exp2(te.astype(np.float64))   # exact
    over = mag > F16_MAX
    mag = np.where(over, np.where(how == TRUNC, F16_MAX, np.inf), mag)
    mag = np.where(special, np.where(f == 0, np.inf, np.nan), mag)
    val = np.where(neg == 1, -mag, mag)
    # Every finite value here is an FP16 number, so this cast does not round.
    return val.astype(np.float16)


def rn16(x):
    """Round-to-nearest-even to FP16 of FP32 (or FP64) values."""
    return _to_f16(x, NEAREST, NEAREST)


def rd16(x):
    """Largest FP16 <= x (toward -inf)."""
    return _to_f16(x, TRUNC, CEIL)


def ru16(x):
    """Smallest FP16 >= x (toward +inf)."""
    return _to_f16(x, CEIL, TRUNC)


def sr16(x, u):
    """Exact stochastic rounding of FP32 x with 24-bit random integers u."""
    x, u = np.broadcast_arrays(np.asarray(x, dtype=np.float32),
                               np.asarray(u, dtype=np.uint64) & np.uint64(U24))
    lo = rd16(x).astype(np.float64)
    hi = ru16(x).astype(np.float64)
    xd = x.astype(np.float64)
    with np.errstate(invalid="ignore"):
        D = hi - lo                                   # power of two, or 0 (exact)
        Edist = xd - lo                               # exact
        t = u.astype(np.float64) * 2.0 ** -24         # exact
        take_hi = (t * D) < Edist
    out = np.where(take_hi, hi, lo)
    big = np.abs(xd) > F16_MAX
    out = np.where(big | np.isnan(xd), rn16(x).astype(np.float64), out)
    return out.astype(np.float16)


def sr16_up_probability(x):
    """Exact probability (over u uniform on [0, 2**24)) that SR rounds x up."""
    x = np.float32(x)
    lo = float(rd16(x))
    hi = float(ru16(x))
    if hi == lo:
        return Fraction(0)
    D = Fraction(hi) - Fraction(lo)
    E = Fraction(float(x)) - Fraction(lo)
    # u' * D < E  <=>  u < 2**24 * E / D ; count integers u in [0, 2**24).
    bound = Fraction(2 ** 24) * E / D
    count = math.ceil(bound)
    return Fraction(min(max(count, 0), 2 ** 24), 2 ** 24)


def rn32(fr):
    """Round an exact rational to the nearest FP32 (ties even), as float."""
    fr = Fraction(fr)
    if fr == 0:
        return 0.0
    neg = fr < 0
    a = -fr if neg else fr
    # exponent e with 2**e <= a < 2**(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    q_exp = max(e, -126) - 23                         # FP32 spacing at a
    scaled = a / Fraction(2) ** q_exp
    k = scaled.numerator // scaled.denominator
    rem = scaled - k
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and k % 2 == 1):
        k += 1
    val = math.ldexp(float(k), q_exp) if k < 2 ** 25 else math.inf
    if val > 3.4028234663852886e38:
        val = math.inf
    return -val if neg else val


def fma32(a, b, c):
    """Single-rounding FP32 fused multiply-add a*b + c, exact model.

    An exactly-zero result follows IEEE 754 (round to nearest): the sum of two
    zeros of the same sign keeps that sign, every other exact zero is +0."""
    a, b, c = (float(np.float32(v)) for v in (a, b, c))
    if any(math.isinf(v) or math.isnan(v) for v in (a, b, c)):
        return float(np.float32(a) * np.float32(b) + np.float32(c))
    exact = Fraction(a) * Fraction(b) + Fraction(c)
    if exact == 0:
        prod_neg = (math.copysign(1.0, a) < 0) != (math.copysign(1.0, b) < 0)
        prod_zero = a == 0 or b == 0
        if prod_zero and c == 0 and prod_neg and math.copysign(1.0, c) < 0:
            return -0.0
        return 0.0
    return rn32(exact)


def dither16(x, u):
    """Dithered rounding of FP32 x with 24-bit random integers u."""
    x = np.asarray(x, dtype=np.float32)
    u = np.asarray(u, dtype=np.uint64) & np.uint64(U24)
    x, u = np.broadcast_arrays(x, u)
    y = np.empty(x.shape, dtype=np.float32)
    xf_all = x * np.float32(DITHER_F)                            # fl32(x * F), one FP32 multiply
    for idx in np.ndindex(x.shape):
        xv = float(x[idx])
        if math.isnan(xv) or math.isinf(xv):
            y[idx] = xv
            continue
        t = int(u[idx]) * 2.0 ** -24 - 0.5                        # exact in FP32
        y[idx] = np.float32(fma32(t, float(xf_all[idx]), xv))
    return rn16(y)


def dither16_mean(x):
    """E over u of dither16(x, u), exactly (sums the FP16 outcomes over u).

    The noise t = u*2**-24 - 1/2 takes 2**24 equally likely values; the FP32
    FMA result is monotone in t, so the FP16 outcome changes at most twice
    and the outcome counts are found by bisection on u.
    """
    x = np.float32(x)

    def q(u):
        return float(dither16(np.float32(x), np.uint64(u)))

    lo_u, hi_u = 0, U24
    vals = []
    # Partition [0, 2**24) into maximal runs of equal outcome.
    start = lo_u
    while start <= hi_u:
        v = q(start)
        a, b = start, hi_u
        while a < b:                                  # last u with outcome v
            mid = (a + b + 1) // 2
            if q(mid) == v:
                a = mid
            else:
                b = mid - 1
        vals.append((v, a - start + 1))
        start = a + 1
    total = sum(Fraction(v) * c for v, c in vals)
    return total / 2 ** 24


def quantize(mode, x, u=None):
    """Dispatch: mode 1 = RN, 2 = SR, 3 = dither (library rounding codes)."""
    if mode == 1:
        return rn16(x)
    if mode == 2:
        return sr16(x, u)
    if mode == 3:
        return dither16(x, u)
    raise ValueError("mode must be 1 (RN), 2 (SR) or 3 (dither)")


# ---- BF16 (the high 16 bits of an FP32: 8 significant bits, FP32's exponent
# range).  The same three rules, with the BF16 neighbours; the dither's noise
# scale is read as the BF16 machine epsilon 2**-7 (about one BF16 ULP), by the
# same reading as F = 2**-10 for FP16.  Values are returned as float64 arrays
# (every BF16 number is exact in FP64); bf16_bits gives the bit patterns.

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127
DITHER_F_BF16 = 2.0 ** -7


def _to_bf16(x, mode_pos, mode_neg):
    """Round FP32 x to BF16 (magnitude rounding per sign), as float64."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32).astype(np.int64)
    neg = (bits >> 31) & 1
    ex = (bits >> 23) & 0xFF
    f = bits & 0x7FFFFF
    M = np.where(ex > 0, f | (1 << 23), f)
    E = np.maximum(ex, 1) - 150                       # |x| = M * 2**E
    te = np.maximum(ex - 127, -126) - 7               # BF16 spacing exponent at |x|
    how = np.where(neg == 1, mode_neg, mode_pos)
    k = _round_mag(M, te - E, how)
    mag = k.astype(np.float64) * np.exp2(te.astype(np.float64))
    over = mag > BF16_MAX
    mag = np.where(over, np.where(how == TRUNC, BF16_MAX, np.inf), mag)
    mag = np.where(ex == 0xFF, np.where(f == 0, np.inf, np.nan), mag)
    return np.where(neg == 1, -mag, mag)


def rnb16(x):
    """Round-to-nearest-even to BF16."""
    return _to_bf16(x, NEAREST, NEAREST)


def rdb16(x):
    """Largest BF16 <= x."""
    return _to_bf16(x, TRUNC, CEIL)


def rub16(x):
    """Smallest BF16 >= x."""
    return _to_bf16(x, CEIL, TRUNC)


def srb16(x, u):
    """Exact stochastic rounding of FP32 x to BF16 with 24-bit integers u."""
    x, u = np.broadcast_arrays(np.asarray(x, dtype=np.float32),
                               np.asarray(u, dtype=np.uint64) & np.uint64(U24))
    lo, hi = rdb16(x), rub16(x)
    xd = x.astype(np.float64)
    with np.errstate(invalid="ignore"):
        take_hi = (u.astype(np.float64) * 2.0 ** -24) * (hi - lo) < (xd - lo)    # all exact in FP64
    out = np.where(take_hi, hi, lo)
    return np.where((np.abs(xd) > BF16_MAX) | np.isnan(xd), rnb16(x), out)


def ditherb16(x, u):
    """Dithered rounding to BF16: RN_bf16(fma32(u*2**-24 - 1/2, fl32(x*2**-7), x))."""
    x = np.asarray(x, dtype=np.float32)
    u = np.asarray(u, dtype=np.uint64) & np.uint64(U24)
    x, u = np.broadcast_arrays(x, u)
    y = np.empty(x.shape, dtype=np.float32)
    xf_all = x * np.float32(DITHER_F_BF16)
    for idx in np.ndindex(x.shape):
        xv = float(x[idx])
        if math.isnan(xv) or math.isinf(xv):
            y[idx] = xv
            continue
        t = int(u[idx]) * 2.0 ** -24 - 0.5
        y[idx] = np.float32(fma32(t, float(xf_all[idx]), xv))
    return rnb16(y)


def quantize_bf16(mode, x, u=None):
    """Dispatch for the BF16 rounding codes: 4 = RN, 5 = SR, 6 = dither."""
    if mode == 4:
        return rnb16(x)
    if mode == 5:
        return srb16(x, u)
    if mode == 6:
        return ditherb16(x, u)
    raise ValueError("mode %r is not a BF16 rounding code" % (mode,))


def bf16_bits(v):
    """Bit patterns (uint16) of BF16 values held in float64 (NaN -> quiet NaN)."""
    b = (np.asarray(v, dtype=np.float64).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return np.where(np.isnan(v), (b | np.uint16(0x40)).astype(np.uint16), b)
