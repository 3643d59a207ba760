"""Pins of the per-contribution model (the paper's own kernel scheme, Sections
4.1 and 4.2) against things other than itself: the FP64 scatter on inputs
whose every sum is exact, a direct sequential FP16 sum when every row lands
in the same entry, and the unbiasedness of stochastic rounding over epochs."""
import numpy as np
import pytest

import workloads
from oracle import model, quant
from oracle.sketch import apply_f64, hash_rows


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("s", [1, 4])
def test_exact_sums_equal_the_fp64_scatter(mode, s):
    # c_s is a power of two and every partial sum a small half-integer: all exact
    A = workloads.integers(2000, 6, seed=11, lim=5).astype(np.float16 if mode else np.float32)
    got = model.apply_per_contribution_model(A, 64, s, 7, mode, epoch=3)
    assert np.array_equal(got.astype(np.float64), apply_f64(A, 64, s, 7))


def test_single_bucket_is_a_sequential_fp16_sum():
    # d = s = 1: every row adds into row 0 of SA, in row order
    g = workloads.rng(5)
    A = (g.standard_normal((400, 3)) * 30).astype(np.float16)
    got = model.apply_per_contribution_model(A, 1, 1, 9, 1)
    _, signs = hash_rows(9, np.arange(400, dtype=np.uint64), 1, 1)
    acc = np.zeros(3, dtype=np.float64)
    for i in range(400):
        v = np.float32(signs[i, 0]) * A[i].astype(np.float32)          # c_s = 1
        acc = quant.rn16(acc + quant.rn16(v).astype(np.float64)).astype(np.float64)
    assert np.array_equal(got[0].astype(np.float64), acc)
    # and FP16 accumulation loses accuracy against the FP64 sum, as Section 4.2 warns
    exact = apply_f64(A, 1, 1, 9)[0]
    assert np.max(np.abs(acc - exact)) > 0


def test_sr_contributions_are_unbiased_over_epochs():
    # one spike, s = 8: each of its 8 contributions is +-fl32(1/sqrt(8)), not an FP16 value
    A = np.zeros((4, 2), dtype=np.float16)
    A[1, 0] = 1.0
    cs = float(model.c_s32(8))
    _, signs = hash_rows(3, np.arange(4, dtype=np.uint64), 16, 8)
    K = 1500
    tot = np.zeros(8)
    for e in range(K):
        SA = model.apply_per_contribution_model(A, 16, 8, 3, 2, epoch=e).astype(np.float64)
        b, _ = hash_rows(3, np.array([1], dtype=np.uint64), 16, 8)
        tot += SA[b[0], 0] * signs[1]
    mean = tot / K
    rd, ru = float(quant.rd16(np.float32(cs))), float(quant.ru16(np.float32(cs)))
    p = (cs - rd) / (ru - rd)
    sd = (ru - rd) * np.sqrt(p * (1 - p))
    assert np.all(np.abs(mean - cs) <= 4 * sd / np.sqrt(K))
    # round-to-nearest is biased by a fixed amount instead
    rn = model.apply_per_contribution_model(A, 16, 8, 3, 1).astype(np.float64)
    assert abs(abs(rn[b[0][0], 0]) - cs) > 10 * sd / np.sqrt(K)
