"""The sketching operator S (d x m) and its application, in FP64.

Paper passages followed:
  * CountSketch: one nonzero per column, S e_i = rho_i e_{b_i}, rho Rademacher,
    b uniform over the d rows (Section 2.2, CountSketch paragraph).
  * SparseStack: zeta stacked CountSketch blocks; the j-th nonzero of a column
    lies in block j, i.e. in rows [j d/zeta, (j+1) d/zeta), with its own
    Rademacher sign (Section 2.2, Definition "SparseStack"; the block ranges
    and the 1/sqrt(zeta) value scale are stated in Section 4.1).  zeta is
    called ``s`` here.
  * The distortion eta(S,U) = max(|sigma_max(SU) - 1|, |1 - sigma_min(SU)|)
    for orthonormal U (Section 2.2, last display; Section 5.1).
  * The coherence mu(U) = (m/n) max_i ||U_{i,:}||^2 (Section 5.2, coherence
    sweep).

The paper draws row indices and signs i.i.d. but names no generator (Section
4.1).  This library fixes one: a counter-based hash, so S never has to be
stored.  Hash version 1:
    key     = (lo32(seed), hi32(seed))
    counter = (lo32(i), hi32(i), floor(j/4), TAG_SKETCH)   for global row i,
                                                          block j
    w       = word (j mod 4) of Philox4x32-10(counter, key)
    W       = d / s                                     (block height)
    bucket  = j*W + floor(w * W / 2**32)                (multiply-shift)
    sign    = -1 if (w & 1) else +1
Both halves are exact and uniform when W is a power of two.  d must be a
multiple of s (Section 4.1 assumes it).
"""
from __future__ import annotations

import numpy as np

from .philox import philox, split64

HASH_VERSION = 1
TAG_SKETCH = 0x534B4348   # counter word 3 of the S hash stream
TAG_ROUND = 0x524E4446    # counter word 3 of the rounding-noise stream


def check_shape(d, s):
    if s < 1 or d < 1 or d % s != 0:
        raise ValueError("need s >= 1, d >= 1 and d % s == 0")


def hash_rows(seed, rows, d, s):
    """Buckets and signs of the given global rows.

    rows: integer array of global row indices.  Returns (buckets int64 [r, s],
    signs int8 [r, s]).

    Pinned by: chi-square uniformity per block, sign balance, block-pair
    independence, E||Sx||^2 = ||x||^2 and its variance law over seeds, and
    bit-equality with the C oracle.
    """
    check_shape(d, s)
    rows = np.asarray(rows, dtype=np.uint64).reshape(-1)
    W = d // s
    k0, k1 = split64(np.uint64(seed))
    r_lo, r_hi = split64(rows)
    out_b = np.empty((rows.size, s), dtype=np.int64)
    out_s = np.empty((rows.size, s), dtype=np.int8)
    for g in range((s + 3) // 4):
        words = philox(r_lo, r_hi, g, TAG_SKETCH, k0, k1)
        for t in range(4):
            j = 4 * g + t
            if j >= s:
                break
            w = words[t].astype(np.uint64)
            out_b[:, j] = j * W + ((w * np.uint64(W)) >> np.uint64(32)).astype(np.int64)
            out_s[:, j] = np.where((w & np.uint64(1)) != 0, -1, 1)
    return out_b, out_s


def value_scale(s):
    """c_s = 1/sqrt(s) in FP64 (Section 4.1: values are +-1/sqrt(zeta))."""
    return 1.0 / np.sqrt(float(s))


def dense_S(m, d, s, seed, row_offset=0):
    """Explicit d x m matrix S[:, row_offset:row_offset+m] in FP64 (tiny m only).

    Built column by column from the definition: column i has the value
    sign*c_s at row bucket, one entry per block.
    """
    b, g = hash_rows(seed, np.arange(row_offset, row_offset + m), d, s)
    S = np.zeros((d, m))
    c = value_scale(s)
    for i in range(m):
        for j in range(s):
            S[b[i, j], i] += g[i, j] * c
    return S


def apply_f64(A, d, s, seed, row_offset=0, scale=None):
    """S[:, row_offset : row_offset+rows] @ A in FP64 by scatter-add.

    A: (rows, n) array of any float dtype; it is upcast exactly to FP64.
    scale: value multiplying each +-1 entry; default c_s = 1/sqrt(s).  Pass
    1.0 for the unscaled signed sums.

    Pinned by: equality with dense_S(...) @ A (numpy matmul) on tiny inputs;
    S e_k = column k of dense_S; column norms of S equal to 1.
    """
    A = np.asarray(A)
    A64 = A.astype(np.float64)
    rows, n = A64.shape
    b, g = hash_rows(seed, np.arange(row_offset, row_offset + rows, dtype=np.uint64), d, s)
    c = value_scale(s) if scale is None else float(scale)
    SA = np.zeros((d, n))
    for j in range(s):
        np.add.at(SA, b[:, j], (g[:, j].astype(np.float64) * c)[:, None] * A64)
    return SA


def singular_values(M):
    return np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)


def distortion(SU):
    """eta(S,U) from the singular values of SU (Section 2.2 / 5.1)."""
    sv = singular_values(SU)
    return max(abs(sv[0] - 1.0), abs(1.0 - sv[-1]))


def orthonormal_basis(A):
    """U from an FP64 QR of A (numpy / LAPACK Householder)."""
    q, _ = np.linalg.qr(np.asarray(A, dtype=np.float64))
    return q


def coherence(U):
    """mu(U) = (m/n) max_i ||U_{i,:}||^2 (Section 5.2)."""
    U = np.asarray(U, dtype=np.float64)
    m, n = U.shape
    return (m / n) * float(np.max(np.sum(U * U, axis=1)))


def condition_number(M):
    """kappa = sigma_max / sigma_min (Section 5.1, reported for SA)."""
    sv = singular_values(M)
    return float(sv[0] / sv[-1])
