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
summed in fixed point (`work_item_partial` below: per column an exponent from
a sample of the unit's first rows, contributions rounded to a grid of
2**(E_c + h - 19) below 2**(E_c + 1), the rare larger ones kept in FP32 and
added after the exact fixed-point sum is rounded to FP32); the unit's partial
P_u is then scaled by c_s = fl32(1/sqrt(s)) and, in the FP16 modes, quantised
once per entry with the rounding rule and added into the FP16 result with
round-to-nearest FP16 additions.  In FP32 mode the partials are added in FP32
and c_s is applied once to the total.

Both orders of summation (inside a unit and across units) are unspecified on
the GPU; the model fixes unit order.  Results therefore agree exactly when
every sum is exact or one unit covers the rows (one quantisation per entry)
and each entry receives at most one outlier, and to a tolerance otherwise.

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


# Fixed-point accumulation of one work item (unit x tile of nt columns x group
# of block_group SparseStack blocks), as the apply kernel computes it.
LIST_CAP = 1024        # outlier records per work item
SAMPLE_RANK = 4        # rank of the lane maximum that sets a column's exponent
HEADROOM = 2           # binades of the exponent above that lane maximum
TILE_COLS = 32
WAVE_ROWS = 64


def binade(v):
    """floor(log2 v) for v > 0, elementwise; -1000 for v == 0."""
    v = np.asarray(v, dtype=np.float64)
    _, e = np.frexp(v)
    return np.where(v > 0, e.astype(np.int64) - 1, -1000)


def default_plan(s, elem_bytes=2, n=64):
    """(block_group, waves, col_tile) the planner picks when a 32-column tile
    (an 8-column one for n <= 16) with the most blocks fits in LDS."""
    nt = 8 if n <= 16 else 32
    bg = next(b for b in ((8, 4, 2, 1) if nt == 32 else (4, 2, 1)) if s % b == 0)
    return bg, (8 if elem_bytes == 4 else 16), nt


def work_item_partial(X, bk, sg, W, waves, dual, nt=TILE_COLS):
    """Unscaled FP32 partial of one work item.

    X: the unit's rows of the tile's live columns as stored values upcast
    exactly (R x C, C <= 32, float64); bk, sg: bucket offsets within each
    block (R x BG, in [0, W)) and signs (+-1) of the rows for the group's
    blocks; waves: waves per workgroup; dual: the FP32 mode's two fields.
    Returns (P, h, n_out, redone): P is BG*W x C float32 (block-major).

    1. Sample: with L = nt/2 lanes per row slot and K = 64/L slots, the lane
       of slot k in wave w sees rows 64w + K g + k, g < L, of the unit's first
       64*waves rows; its largest |x| per column is one sample value, and
       E_c = binade(4th largest of the K*waves values) + 2.
    2. A contribution with |x| >= 2**(E_c + 1) is an outlier; the others are
       rounded to q = rne(x * 2**S_c), S_c = 19 - h - E_c (E_c clamped to
       [-108 - h, 145 - h]); the FP32 mode adds the residual's
       z = rne((x * 2**S_c - q) * 2**21) at 2**(S_c + 21).
    3. The count headroom starts at h0 = the smallest h with
       3a/2 + 64 < 2**(10 + h), a = ceil(R / W) (at most 16): a bucket row's
       average count with room to spare.  If more than LIST_CAP outlier records
       (elements x BG) arise, E_c becomes binade(max |x| of the column); if a
       bucket row takes K >= 2**(10 + h) contributions, h grows; the item is
       then recomputed.
    4. P = fl32(exact signed sum * 2**-S_c), then each outlier sign * x is
       added in FP32 (rows in order).
    """
    X = np.asarray(X, dtype=np.float64)
    R, C = X.shape
    bg = bk.shape[1]
    if not np.all(np.isfinite(X)):
        raise ValueError("non-finite input takes the float path; not modelled")
    absX = np.abs(X)
    rows = WAVE_ROWS * waves
    Xs = np.zeros((rows, C))
    Xs[:min(R, rows)] = absX[:rows]
    L = nt // 2
    K = 64 // L
    lane_max = Xs.reshape(waves, L, K, C).max(axis=1).reshape(K * waves, C)
    M = -np.sort(-lane_max, axis=0)[SAMPLE_RANK - 1]
    E = binade(M) + HEADROOM
    kall = max(int(np.bincount(bk[:, j], minlength=W).max()) if R else 0 for j in range(bg))
    h = 0
    while h < 16 and 3 * (-(-R // W)) // 2 + 64 >= (1 << (10 + h)):
        h += 1
    redone = False
    for attempt in range(2):
        Ec = np.clip(E, -108 - h, 145 - h)
        thr = np.ldexp(1.0, Ec + 1)
        out = absX >= thr[None, :]
        n_out = int(out.sum()) * bg
        if kall < (1 << (10 + h)) and n_out <= LIST_CAP:
            break
        if attempt == 1:
            raise AssertionError("the second attempt always succeeds")
        redone = True
        if n_out > LIST_CAP:
            E = binade(absX.max(axis=0) if R else np.zeros(C))
        while kall >= (1 << (10 + h)):
            h += 1
        if h > 16:
            raise ValueError("a bucket row with 2**26 rows or more takes the float path; not modelled")
    S = 19 - h - Ec
    scaled = np.where(out, 0.0, X) * np.ldexp(1.0, S)[None, :]
    q = np.rint(scaled)
    if dual:
        z = np.rint((scaled - q) * 2.0 ** 21)
        val = q.astype(np.int64) * (1 << 21) + z.astype(np.int64)
        shift = S + 21
    else:
        val = q.astype(np.int64)
        shift = S
    acc = np.zeros((bg * W, C), dtype=np.int64)
    for j in range(bg):
        np.add.at(acc, j * W + bk[:, j], sg[:, j:j + 1].astype(np.int64) * val)
    if dual:
        P = (acc.astype(np.float64) * np.ldexp(1.0, -shift)[None, :]).astype(np.float32)
    else:
        P = (acc.astype(np.float32).astype(np.float64) * np.ldexp(1.0, -shift)[None, :]).astype(np.float32)
    for i, c in zip(*np.nonzero(out)):
        for j in range(bg):
            e = j * W + bk[i, j]
            P[e, c] = np.float32(P[e, c] + np.float32(sg[i, j] * X[i, c]))
    return P, h, n_out, redone


def unit_partial_fixed(A, d, s, seed, r0, waves=None, block_group=None, dual=False, col_tile=None):
    """Unscaled FP32 partial (d x n) of one unit of rows A (first global row
    r0), assembled from its work items."""
    from .sketch import hash_rows
    check_shape(d, s)
    A = np.asarray(A)
    R, n = A.shape
    bgd, wd, ntd = default_plan(s, n=n)
    bg = block_group or bgd
    waves = waves or wd
    nt = col_tile or ntd
    W = d // s
    b, g = hash_rows(seed, np.arange(R, dtype=np.uint64) + np.uint64(r0), d, s)
    off = b - (np.arange(s, dtype=np.int64) * W)[None, :]
    X = A.astype(np.float64)
    P = np.zeros((d, n), dtype=np.float32)
    for j0 in range(0, s, bg):
        for c0 in range(0, n, nt):
            c1 = min(c0 + nt, n)
            Pi, _, _, _ = work_item_partial(X[:, c0:c1], off[:, j0:j0 + bg], g[:, j0:j0 + bg], W, waves, dual, nt)
            P[j0 * W:(j0 + bg) * W, c0:c1] = Pi
    return P


def apply_f16_model(A, d, s, seed, mode, epoch, chunk_rows, row_offset=0, SA0=None, waves=None,
                    block_group=None, col_tile=None):
    """FP16-mode result, units added in order.

    Each unit partial is `unit_partial_fixed` (the exact sum when every
    contribution sits on its column's grid, e.g. integer A with
    |sums| < 2**24), scaled by c_s32 in FP32, quantised per entry with
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
    for a, b in units(A.shape[0], chunk_rows):
        r0 = row_offset + a
        P = unit_partial_fixed(A[a:b], d, s, seed, r0, waves, block_group, col_tile=col_tile)
        v = (cs * P).astype(np.float32)
        u = None
        if mode in (ACC_F16_SR, ACC_F16_DITHER):
            u = round_u24(seed, epoch, np.uint64(r0) * np.uint64(d * n) + site)
        qv = quantize(mode, v, u)
        acc = f16_add(acc, qv)
    return acc


def apply_f32_one_unit_model(A, d, s, seed, row_offset=0, waves=None, block_group=None, col_tile=None):
    """FP32-mode result when one unit covers the rows: fl32(c_s32 * P) with P
    the two-field fixed-point partial (c_s32 is applied to the FP32 partial,
    exactly, when it is a power of two, else once to the FP32 total)."""
    P = unit_partial_fixed(A, d, s, seed, row_offset, waves, block_group, dual=True, col_tile=col_tile)
    return (c_s32(s) * P).astype(np.float32)


def apply_whole_call_model(A, d, s, seed, mode, epoch=0, row_offset=0, SA0=None):
    """Result of a call summed as ONE unit whose partial is fl32 of the exact
    sum (the bucket-sorted gather path: every entry of SA is the signed sum of
    the rows hashed to it, Section 2.2's definition read by bucket).

    P = fl32(sum of sign * A[i, c] over the rows hashed to (b, c)), taken from
    the FP64 sum; v = fl32(c_s32 * P).  FP32 mode: v, or fl32(SA0 + v) when
    accumulating.  FP16 modes: v quantised once per entry with rounding `mode`
    (noise site q = row_offset*d*n + b*n + c, as for any unit starting at
    global row row_offset), added to SA0 (zeros) with one FP16 RN addition.
    """
    check_shape(d, s)
    A = np.asarray(A)
    n = A.shape[1]
    P = apply_f64(A, d, s, seed, row_offset, scale=1.0).astype(np.float32)
    v = (c_s32(s) * P).astype(np.float32)
    if mode == ACC_F32:
        if SA0 is None:
            return v
        return (np.asarray(SA0, dtype=np.float32) + v).astype(np.float32)
    u = None
    if mode in (ACC_F16_SR, ACC_F16_DITHER):
        site = (np.uint64(row_offset) * np.uint64(d * n) + np.arange(d, dtype=np.uint64)[:, None] * np.uint64(n)
                + np.arange(n, dtype=np.uint64)[None, :])
        u = round_u24(seed, epoch, site)
    qv = quantize(mode, v, u)
    acc = np.zeros((d, n), dtype=np.float16) if SA0 is None else np.asarray(SA0, dtype=np.float16)
    return f16_add(acc, qv)


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
