"""Pins of the oracle's sketch operator (CPU only).

What fixes the hash and S independently of the oracle's own code: the block
structure of SparseStack (Section 2.2 definition, Section 4.1 block ranges),
explicit S @ A by numpy matmul, column norms, uniformity and independence
statistics, and E||Sx||^2 = ||x||^2 with its variance
(2/d)(||x||_2^4 - ||x||_4^4), derived for sign-hashed sketches whose buckets
are pairwise independent and signs 4-wise independent.
"""
import numpy as np
import pytest

import workloads
from oracle import native
from oracle.sketch import (apply_f64, coherence, dense_S, distortion, hash_rows,
                           orthonormal_basis)


@pytest.mark.parametrize("d,s", [(64, 1), (64, 4), (64, 8), (48, 3), (1024, 16)])
def test_buckets_stay_in_their_block(d, s):
    b, g = hash_rows(7, np.arange(5000), d, s)
    W = d // s
    for j in range(s):
        assert np.all(b[:, j] >= j * W) and np.all(b[:, j] < (j + 1) * W)
    assert set(np.unique(g)) <= {-1, 1}


def test_hash_c_and_python_agree():
    for d, s, seed, r0 in [(256, 4, 0, 0), (1024, 8, 2 ** 40 + 3, 2 ** 33 - 7), (30, 5, 9, 0)]:
        bp, gp = hash_rows(seed, np.arange(r0, r0 + 3000, dtype=np.uint64), d, s)
        bc, gc = native.hash_rows(seed, r0, 3000, d, s)
        assert np.array_equal(bp, bc) and np.array_equal(gp, gc)


def test_hash_uniform_balanced_and_independent():
    d, s, rows = 256, 4, 200_000
    b, g = hash_rows(3, np.arange(rows), d, s)
    W = d // s
    for j in range(s):
        counts = np.bincount(b[:, j] - j * W, minlength=W)
        exp = rows / W
        chi2 = float(((counts - exp) ** 2 / exp).sum())
        assert chi2 < W + 6 * np.sqrt(2 * W)           # ~6 sigma for W-1 dof
        assert abs(float(g[:, j].mean())) < 6 / np.sqrt(rows)
    # block pair (0, 1): joint histogram of the top 3 bits is uniform
    a = (b[:, 0] * 8) // W
    c = ((b[:, 1] - W) * 8) // W
    joint = np.bincount(a * 8 + c, minlength=64)
    exp = rows / 64
    assert float(((joint - exp) ** 2 / exp).sum()) < 64 + 6 * np.sqrt(128)
    # signs of different blocks are uncorrelated
    assert abs(float((g[:, 0].astype(float) * g[:, 1]).mean())) < 6 / np.sqrt(rows)


@pytest.mark.parametrize("d,s", [(16, 1), (16, 4), (24, 8), (12, 3)])
def test_scatter_equals_explicit_matmul(d, s):
    m, n = 200, 5
    A = workloads.gaussian(m, n, 4).astype(np.float64)
    S = dense_S(m, d, s, 99, row_offset=17)
    assert np.allclose(apply_f64(A, d, s, 99, row_offset=17), S @ A, rtol=0, atol=1e-12)
    # A = I gives S itself; a spike e_k picks column k
    assert np.allclose(apply_f64(np.eye(m), d, s, 99, row_offset=17), S, atol=0)
    e = np.zeros((m, 1))
    e[31, 0] = 1.0
    assert np.allclose(apply_f64(e, d, s, 99, row_offset=17)[:, 0], S[:, 31], atol=0)


@pytest.mark.parametrize("s", [1, 2, 4, 8])
def test_columns_have_unit_norm_and_s_nonzeros(s):
    S = dense_S(300, 32, s, 5)
    assert np.all((S != 0).sum(axis=0) == s)
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=1e-15)
    if s == 1:                                       # CountSketch: a signed one-hot
        assert set(np.unique(np.abs(S[S != 0]))) == {1.0}


def test_norm_preserved_in_expectation_with_closed_form_variance():
    d, s, K = 64, 4, 2000
    x = workloads.gaussian(400, 1, 8).astype(np.float64)[:, 0]
    x2 = float(x @ x)
    vals = np.array([np.sum(apply_f64(x[:, None], d, s, seed)[:, 0] ** 2) / x2
                     for seed in range(K)])
    var = (2.0 / d) * (x2 ** 2 - float(np.sum(x ** 4))) / x2 ** 2
    assert abs(vals.mean() - 1.0) < 4 * np.sqrt(var / K)
    # sample variance within ~15% of the closed form (K = 2000)
    assert abs(vals.var() / var - 1.0) < 0.15


def test_c_oracle_matches_python_oracle():
    for dt in (np.float32, np.float16):
        A = workloads.gaussian(3000, 7, 1, dt)
        for d, s in [(64, 4), (40, 8), (33, 1)]:
            p = apply_f64(A, d, s, 21, row_offset=1000)
            c = native.sketch_f64(A, d, s, 21, row_offset=1000)
            assert np.allclose(p, c, rtol=1e-12, atol=1e-12)
    # strided A (lda > n) and thread count 1
    big = workloads.gaussian(500, 12, 2)
    sub = big[:, :9]
    assert np.allclose(native.sketch_f64(sub, 64, 4, 3, nthreads=1),
                       apply_f64(sub, 64, 4, 3), rtol=1e-12, atol=1e-12)


def test_row_chunks_with_offsets_sum_to_whole():
    A = workloads.integers(5000, 6, 3).astype(np.float64)
    whole = apply_f64(A, 128, 4, 77)
    parts = sum(apply_f64(A[a:a + 1300], 128, 4, 77, row_offset=a) for a in range(0, 5000, 1300))
    assert np.array_equal(whole, parts)


def test_distortion_special_cases():
    # spikes with s = 1: eta = 1 exactly iff two spikes share a bucket, else 0
    m, n, d = 4096, 16, 64
    U = workloads.spikes(m, n).astype(np.float64)
    for seed in range(20):
        b, _ = hash_rows(seed, np.arange(0, m, m // n), d, 1)
        collide = len(np.unique(b[:, 0])) < n
        eta = distortion(apply_f64(U, d, 1, seed))
        assert (abs(eta - 1.0) < 1e-12) if collide else (eta < 1e-12)
    # Gaussian subspace: eta of the order sqrt(n/d) (Section 5.1 reference curve)
    A = workloads.gaussian(16384, 32, 0, np.float64)
    eta = distortion(apply_f64(orthonormal_basis(A), 256, 4, 0))
    assert 0.3 * np.sqrt(32 / 256) < eta < 2.5 * np.sqrt(32 / 256)


def test_coherence_of_the_input_families():
    m, n = 4096, 16
    assert coherence(orthonormal_basis(workloads.spikes(m, n))) == pytest.approx(m / n)
    assert coherence(orthonormal_basis(workloads.coherent(m, n, 1))) == pytest.approx(m / n, rel=1e-6)
    assert coherence(orthonormal_basis(workloads.gaussian(m, n, 1))) < 4.0
