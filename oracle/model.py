"""What one sketch_apply call computes, as a model the GPU result is held to.

The paper forms SA by scattering every contribution sign * A[i, c] (times
1/sqrt(zeta)) into SA with atomic adds, either in FP32 or, for the FP16
variants, after quantising each contribution with the chosen rounding rule and
accumulating with FP16 atomics (Section 4.1, explicit SparseStack
accumulation; Section 4.2, vectorised 16-bit accumulation and the three
rounding rules).

Reading adopted by this library (the paper's per-contribution FP16 scheme
loses about 2% at a 4M-row input, far above a 4e-3 budget): rows are cut into
consecutive *units* of `chunk_rows` rows; inside a unit the contributions are
summed in FP32; the unit's partial P_u is then scaled by c_s = fl32(1/sqrt(s))
and, in the FP16 modes, quantised once per entry with the rounding rule and
added into the FP16 result with round-to-nearest FP16 additions.  In FP32 mode
the partials are added in FP32 and c_s is applied once to the total.

Both orders of summation (inside a unit and across units) are unspecified on
the GPU; the model fixes unit order.  Results therefore agree exactly when
every sum is exact (integer-valued A, a single unit per entry, ...) and to a
tolerance otherwise.

Rounding-noise stream (the paper calls an unspecified random_uint(), Section
4.2): for the entry (b, c) of the unit whose first global row is r0,
    q       = r0 * (d * n) + b * n + c
    counter = (lo32(q >> 2), hi32(q >> 2), epoch, TAG_ROUND)
    u       = word (q & 3) of Philox4x32-10(counter, (lo32(seed), hi32(seed)))
              & 0xFFFFFF.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from .philox import philox, split64
from .quant import rn16, quantize
from .sketch import TAG_ROUND, apply_f64, check_shape

ACC_F32, ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER = 0, 1, 2, 3


def c_s32(s):
    """fl32(1/sqrt(s)): the value scale as the FP32 library applies it."""
    return np.float32(1.0 / np.sqrt(np.float64(s)))


def round_u24(seed, epoch, q):
    """24-bit rounding noise for quantisation sites q (uint64 array)."""
    q = np.asarray(q, dtype=np.uint64)
    call = q >> np.uint64(2)
    lo, hi = split64(call)
    k0, k1 = split64(np.uint64(seed))
    w = philox(lo, hi, np.uint64(epoch) & np.uint64(0xFFFFFFFF), TAG_ROUND, k0, k1)
    sel = (q & np.uint64(3)).astype(np.int64)
    stacked = np.stack(w, axis=0)
    u = np.take_along_axis(stacked, sel[None, ...], axis=0)[0]
    return u.astype(np.uint64) & np.uint64(0xFFFFFF)


def units(rows, chunk_rows):
    """[(first, last+1)] of the consecutive row units of one call."""
    return [(r, min(r + chunk_rows, rows)) for r in range(0, rows, chunk_rows)]


def apply_f32_exact_int(A, d, s, seed, row_offset=0, SA0=None):
    """FP32-mode result when every partial sum is an integer below 2**24.

    expected = fl32(c_s32 * sum) (+ SA0 in FP32 when accumulating), where
    sum = sum of sign * A[i, c] over the rows hashed to the entry (exact).
    """
    check_shape(d, s)
    tot = apply_f64(A, d, s, seed, row_offset, scale=1.0)
    if np.any(np.abs(tot) >= 2.0 ** 24) or np.any(tot != np.round(tot)):
        raise ValueError("sums are not exactly representable integers")
    out = (c_s32(s) * tot.astype(np.float32)).astype(np.float32)
    if SA0 is not None:
        out = (np.asarray(SA0, dtype=np.float32) + out).astype(np.float32)
    return out


def f16_add(a, b):
    """Round-to-nearest FP16 addition (the exact sum of two FP16 numbers fits
    in FP64, so only one rounding happens)."""
    return rn16(np.asarray(a, dtype=np.float16).astype(np.float64)
                + np.asarray(b, dtype=np.float16).astype(np.float64))


def unit_partials(A, d, s, seed, chunk_rows, row_offset=0):
    """[(r0_global, P_u)] with P_u the unscaled FP64 partial of each unit."""
    A = np.asarray(A)
    out = []
    for a, b in units(A.shape[0], chunk_rows):
        P = apply_f64(A[a:b], d, s, seed, row_offset + a, scale=1.0)
        out.append((row_offset + a, P))
    return out


def apply_f16_model(A, d, s, seed, mode, epoch, chunk_rows, row_offset=0, SA0=None):
    """FP16-mode result, units added in order.

    Each unit partial is taken as fl32 of its exact value (exact for integer
    A with |sums| < 2**24), scaled by c_s32 in FP32, quantised per entry with
    rounding `mode` and noise from round_u24, then added with FP16 RN adds.
    """
    check_shape(d, s)
    A = np.asarray(A)
    n = A.shape[1]
    acc = (np.zeros((d, n), dtype=np.float16) if SA0 is None
           else np.asarray(SA0, dtype=np.float16).copy())
    cs = c_s32(s)
    site = (np.arange(d, dtype=np.uint64)[:, None] * np.uint64(n)
            + np.arange(n, dtype=np.uint64)[None, :])
    for r0, P in unit_partials(A, d, s, seed, chunk_rows, row_offset):
        v = (cs * P.astype(np.float32)).astype(np.float32)
        u = None
        if mode in (ACC_F16_SR, ACC_F16_DITHER):
            u = round_u24(seed, epoch, np.uint64(r0) * np.uint64(d * n) + site)
        qv = quantize(mode, v, u)
        acc = f16_add(acc, qv)
    return acc


def contribution_sites(rows, j, n, s):
    """Rounding-noise sites of the per-contribution scheme: q = (i*s + j)*n + c
    for global rows i (array), block j and every column c."""
    rows = np.asarray(rows, dtype=np.uint64)
    return ((rows[:, None] * np.uint64(s) + np.uint64(j)) * np.uint64(n)
            + np.arange(n, dtype=np.uint64)[None, :])


def apply_per_contribution_model(A, d, s, seed, mode, epoch=0, row_offset=0, SA0=None):
    """The paper's own kernel scheme (Section 4.1 scatter; Section 4.2
    quantise-then-add), rows taken in order.

    Every contribution is the FP32 product v = fl32(sv * x) of the stored S
    value sv = +-fl32(1/sqrt(s)) and the element x.  mode 0 (FP32 output):
    SA[b, c] += v in FP32.  Modes 1..3 (FP16 output): v is rounded to FP16
    with the rule (noise from site q = (i*s + j)*n + c of the rounding
    stream) and added with an FP16 round-to-nearest addition.  The GPU adds
    in an unspecified order, so the two agree exactly only where every sum is
    exact or each entry receives one contribution.

    Zero contributions: each rule maps +-0 to a zero (dither's exact FMA
    t*(x*2^-10) + x gives -0 only for x = -0 and t >= 0), and adding a zero
    to an FP16 sum changes it only if the sum is -0; a sum that starts
    without -0 never becomes -0 under round-to-nearest additions, so rows
    whose contributions are all zero are skipped (SA0 must hold no -0).
    """
    from .sketch import hash_rows
    check_shape(d, s)
    A = np.asarray(A)
    m, n = A.shape
    f16 = mode != ACC_F32
    dt = np.float16 if f16 else np.float32
    acc = np.zeros((d, n), dtype=dt) if SA0 is None else np.asarray(SA0, dtype=dt).copy()
    if np.any((acc == 0) & np.signbit(acc)):
        raise ValueError("SA0 holds -0")
    rows = np.arange(m, dtype=np.uint64) + np.uint64(row_offset)
    buckets, signs = hash_rows(seed, rows, d, s)
    cs = c_s32(s)
    x32 = A.astype(np.float32)
    for j in range(s):
        sv = np.where(signs[:, j] < 0, -cs, cs).astype(np.float32)
        v = (sv[:, None] * x32).astype(np.float32)               # [m, n], one FP32 product each
        if f16:
            u = None
            if mode in (ACC_F16_SR, ACC_F16_DITHER):
                u = round_u24(seed, epoch, contribution_sites(rows, j, n, s))
            qv = np.zeros(v.shape, dtype=np.float16)
            nz = v != 0
            qv[nz] = quantize(mode, v[nz], None if u is None else u[nz])
            zs = np.signbit(v) & ~nz
            if mode == ACC_F16_DITHER:
                zs &= u >= np.uint64(1 << 23)
            qv[zs] = np.float16(-0.0)
        else:
            qv = v
        b = buckets[:, j]
        live = np.nonzero(np.any(qv != 0, axis=1))[0]
        for i in live:
            if f16:
                acc[b[i]] = f16_add(acc[b[i]], qv[i])
            else:
                acc[b[i]] = (acc[b[i]] + qv[i]).astype(np.float32)
    return acc


ACC_BF16_RN, ACC_BF16_SR, ACC_BF16_DITHER = 4, 5, 6


def apply_bf16_model(A, d, s, seed, mode, epoch, row_offset=0, SA0=None):
    """BF16 output: the whole call is summed in FP32 and each entry rounded
    once (BF16 keeps 8 significant bits, so adding unit partials in BF16 would
    lose about 2**-9 per addition; the library keeps FP32 global partials).

    The sum is taken as fl32 of the exact FP64 sum (exact for integer A whose
    sums stay below 2**24), scaled by c_s32 in FP32, rounded with the BF16
    rule (noise site q = row_offset*d*n + b*n + c), and stored, or added to
    SA0 with one BF16 round-to-nearest addition.  Returns float64 BF16 values.
    """
    from .quant import quantize_bf16
    check_shape(d, s)
    A = np.asarray(A)
    n = A.shape[1]
    P = apply_f64(A, d, s, seed, row_offset, scale=1.0).astype(np.float32)
    v = (c_s32(s) * P).astype(np.float32)
    u = None
    if mode in (ACC_BF16_SR, ACC_BF16_DITHER):
        site = (np.uint64(row_offset) * np.uint64(d * n) + np.arange(d, dtype=np.uint64)[:, None] * np.uint64(n)
                + np.arange(n, dtype=np.uint64)[None, :])
        u = round_u24(seed, epoch, site)
    q = quantize_bf16(mode, v, u)
    if SA0 is None:
        return q
    # two BF16 numbers sum exactly in FP64 unless their exponents differ by
    # more than 44, and then the smaller cannot affect the BF16 rounding
    return rnb16_from_f64(np.asarray(SA0, dtype=np.float64) + q)


def rnb16_from_f64(s):
    """Round-to-nearest-even to BF16 of FP64 values, by exact rationals."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty_like(s)
    for idx in np.ndindex(s.shape):
        v = float(s[idx])
        if v == 0 or math.isinf(v) or math.isnan(v):
            out[idx] = v
            continue
        _, e = math.frexp(abs(v))                     # 2**(e-1) <= |v| < 2**e
        te = max(e - 1, -126) - 7                     # BF16 spacing exponent at |v|
        fr = Fraction(abs(v)) / Fraction(2) ** te
        k = fr.numerator // fr.denominator
        rem = fr - k
        if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and k % 2 == 1):
            k += 1
        mag = math.ldexp(float(k), te)
        out[idx] = -mag if v < 0 else mag
    return out
