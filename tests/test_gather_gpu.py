"""The bucket-sorted gather path of sketch_apply against the oracle (needs an MI355X).

The gather lists every row under each of its s buckets (the hash of paper
Section 2.2) and sums each SA row from its list in FP64, so a call's result is
the one-unit model with partial fl32(exact sum): `model.apply_whole_call_model`.
Integer input makes every sum exact, so those cases are bit for bit; Gaussian
input may differ from the model only where an FP64 sum taken in another order
rounds to the other side of an FP32 (or FP16) rounding boundary, which the
tests allow for at most one unit in the last place on a tiny fraction of the
entries.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import model
from oracle.sketch import apply_f64
from paper_2606_20195_amd import (ACC_BF16_RN, ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, Sketch,
                                  SketchError)

pytestmark = pytest.mark.gpu

GATHER = dict(gather=1)


def to_dev(A, dtype=None, pad=0):
    A = np.ascontiguousarray(A)
    rows, n = A.shape
    t = torch.from_numpy(A.astype(np.float32) if dtype == torch.bfloat16 else A)
    if dtype is not None:
        t = t.to(dtype)
    if pad:
        big = torch.zeros((rows, n + pad), dtype=t.dtype)
        big[:, :n] = t
        return big.cuda()[:, :n]
    return t.cuda()


def gather_apply(A_dev, m, d, s, seed, rounding, row_offset=0, epoch=0, SA=None, accumulate=False, sched=GATHER):
    sk = Sketch(m, d, s, seed, rounding)
    if sched is not None:
        sk.set_schedule(**sched)
    out = sk.apply(A_dev, SA=SA, row_offset=row_offset, epoch=epoch, accumulate=accumulate)
    torch.cuda.synchronize()
    return (out.float() if out.dtype == torch.bfloat16 else out).cpu().numpy()


def ulp_diff16(a, b):
    """|difference| in FP16 units in the last place (same-sign finite values)."""
    ia = a.view(np.int16).astype(np.int64)
    ib = b.view(np.int16).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFF), ib)
    return np.abs(ia - ib)


def ulp_diff32(a, b):
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


@pytest.mark.parametrize("dt", [torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("rows,n,d,s,pad,r0", [
    (30000, 64, 4096, 1, 0, 0),          # CountSketch, one 16-byte group per lane, whole chunks
    (20000, 70, 16384, 4, 0, 77),        # ragged last chunk
    (12000, 300, 6000, 3, 5, 1000),      # two chunks (FP32), odd lda: per-element loads
    (5000, 1, 512, 8, 0, 0),             # one column, s = 8 (two hash calls per row)
    (777, 1030, 2048, 2, 0, 3),          # rows wider than a 64-lane chunk of 16-bit groups
])
def test_gather_fp32_integer_is_bit_exact(rows, n, d, s, pad, r0, dt):
    A = workloads.integers(rows, n, seed=rows + n, lim=6)
    got = gather_apply(to_dev(A, dt, pad), rows + r0, d, s, 21, ACC_F32, row_offset=r0)
    assert np.array_equal(got, model.apply_f32_exact_int(A, d, s, 21, row_offset=r0))


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER])
def test_gather_fp16_integer_is_one_quantisation(rounding):
    d, s, m, n = 8192, 2, 20000, 40
    A = workloads.integers(m, n, seed=52, lim=5).astype(np.float16)
    sa0 = workloads.integers(d, n, seed=53, lim=3).astype(np.float16)
    SA = torch.from_numpy(sa0).cuda()
    got = gather_apply(to_dev(A), m + 500, d, s, 13, rounding, row_offset=500, epoch=6, SA=SA, accumulate=True)
    ref = model.apply_whole_call_model(A, d, s, 13, rounding, epoch=6, row_offset=500, SA0=sa0)
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_gather_fp32_gaussian_is_fl32_of_the_exact_sum():
    d, s, m, n = 16384, 4, 60000, 96
    A = workloads.gaussian(m, n, 54, np.float32)
    got = gather_apply(to_dev(A), m, d, s, 14, ACC_F32)
    ref = model.apply_whole_call_model(A, d, s, 14, ACC_F32)
    diff = ulp_diff32(got, ref)
    assert diff.max() <= 1
    assert np.count_nonzero(diff) <= 1e-4 * diff.size


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR])
def test_gather_fp16_gaussian_matches_the_one_unit_model(rounding):
    d, s, m, n = 16384, 4, 60000, 128
    A = workloads.gaussian(m, n, 55, np.float16)
    got = gather_apply(to_dev(A), m, d, s, 15, rounding, epoch=2)
    ref = model.apply_whole_call_model(A, d, s, 15, rounding, epoch=2)
    diff = ulp_diff16(got, ref)
    assert diff.max() <= 1
    assert np.count_nonzero(diff) <= 1e-4 * diff.size
    # and against FP64: one FP16 rounding per entry
    f64 = apply_f64(A, d, s, 15)
    err = np.linalg.norm(got.astype(np.float64) - f64) / np.linalg.norm(f64)
    assert err <= 4e-4


def test_gather_bf16_output_is_the_bf16_model():
    d, s, m, n = 4096, 4, 30000, 64
    A = workloads.integers(m, n, seed=56, lim=4)
    got = gather_apply(to_dev(A), m, d, s, 16, ACC_BF16_RN)
    ref = model.apply_bf16_model(A, d, s, 16, ACC_BF16_RN, 0)
    assert np.array_equal(got.astype(np.float64), ref)


def test_gather_shards_accumulate_to_the_whole():
    # two row shards with SK_ACCUMULATE equal one call (FP32 mode, integer input)
    d, s, m, n = 16384, 4, 40000, 80
    A = workloads.integers(m, n, seed=57, lim=5)
    sk = Sketch(m, d, s, 18, ACC_F32)
    sk.set_schedule(gather=1)
    Ad = to_dev(A)
    SA = sk.apply(Ad[:15000])
    sk.apply(Ad[15000:], SA=SA, row_offset=15000, accumulate=True)
    torch.cuda.synchronize()
    assert np.array_equal(SA.cpu().numpy(), model.apply_f32_exact_int(A, d, s, 18))


def test_gather_is_deterministic_on_exact_sums_and_empty_input_clears():
    d, s, m, n = 4096, 4, 50000, 64
    A = to_dev(workloads.integers(m, n, seed=58, lim=7))
    a = gather_apply(A, m, d, s, 19, ACC_F32)
    b = gather_apply(A, m, d, s, 19, ACC_F32)
    assert np.array_equal(a, b)
    SA = torch.full((d, n), 3.0, device="cuda")
    out = gather_apply(A[:0], m, d, s, 19, ACC_F32, SA=SA)
    assert np.count_nonzero(out) == 0
    SA16 = torch.full((d, n), 2.0, dtype=torch.float16, device="cuda")
    out = gather_apply(A[:0].half(), m, d, s, 19, ACC_F16_RN, SA=SA16, accumulate=True)
    assert np.all(out == 2.0)


def test_planner_takes_the_gather_for_large_ds_and_wide_rows():
    # Table 1 at n = 1024, FP32 A: FP16 partials at d/n = 2 and 4 fit 32-column
    # tiles; d/n = 8, 16 and 24 leave narrow tiles only, CountSketch at d/n = 2
    # too, and FP32 partials at d/n = 2 one block per tile: the gather
    assert Sketch(100000, 2048, 4, 3, ACC_F16_RN).plan(0, 100000, 1024)["col_tile"] == 32
    assert Sketch(100000, 4096, 4, 3, ACC_F16_RN).plan(0, 100000, 1024)["col_tile"] == 32
    for d, s in ((2048, 4), (8192, 4), (16384, 4), (24576, 4), (2048, 1)):
        p = Sketch(100000, d, s, 3, ACC_F32).plan(0, 100000, 1024)
        assert p["gather"] == 1 and p["global_atomics"] == 0 and p["block_group"] == 0, (d, s)
    # narrow rows keep the tiles, or the atomics when no tile fits
    assert Sketch(100000, 4096, 1, 3, ACC_F16_RN).plan(1, 100000, 64)["gather"] == 0
    p = Sketch(100000, 1 << 17, 1, 3, ACC_F16_RN).plan(1, 100000, 16)
    assert p["global_atomics"] == 1 and p["gather"] == 0
    # a forced schedule is taken as given
    sk = Sketch(100000, 16384, 4, 3, ACC_F32)
    sk.set_schedule(col_tile=2)
    assert sk.plan(0, 100000, 1024)["col_tile"] == 2


def test_gather_noalloc_falls_back_or_refuses_beyond_the_scratch():
    # the planner's gather with lists beyond the scratch falls back to atomics;
    # a forced gather refuses
    d, s, m, n = 16384, 4, 1 << 20, 80
    A = torch.zeros((m, n), device="cuda")
    sk = Sketch(m, d, s, 0, ACC_F32)
    assert sk.plan(0, m, n)["gather"] == 1
    SA = torch.ones((d, n), device="cuda")
    sk.apply(A, SA=SA, noalloc=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(SA).item() == 0
    sk.set_schedule(gather=1)
    with pytest.raises(SketchError, match="scratch"):
        sk.apply(A, SA=SA, noalloc=True)


def test_full_size_gather_at_the_table1_shape_on_sampled_rows():
    # The paper's Table 1 shape (2^21 x 1024 FP32, d/n = 16, SparseStack s = 4),
    # the launch the gather leg of bench.py times: 48 sampled rows of SA, each
    # the oracle's FP64 sum over the rows its hash sends there (found with the
    # C oracle's hash), rounded to FP32 once and scaled by fl32(1/2).
    from oracle import native
    m, n, d, s, seed = 1 << 21, 1024, 16384, 4, 3
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    A = torch.randn((m, n), generator=gen, device="cuda", dtype=torch.float32)
    sk = Sketch(m, d, s, seed, ACC_F32)
    assert sk.plan(0, m, n)["gather"] == 1
    SA = sk.apply(A)
    torch.cuda.synchronize()
    b, g = native.hash_rows(seed, 0, m, d, s)
    picks = np.random.default_rng(8).choice(d, size=48, replace=False)
    got = SA[torch.from_numpy(picks).cuda()].cpu().numpy()
    for k, bucket in enumerate(picks):
        rows, blk = np.nonzero(b == bucket)
        X = A[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        exact = (g[rows, blk].astype(np.float64)[:, None] * X).sum(axis=0)
        want = (np.float32(0.5) * exact.astype(np.float32)).astype(np.float32)
        diff = ulp_diff32(got[k].copy(), want)
        assert diff.max() <= 1, (bucket, diff.max())
    del A, SA
    torch.cuda.empty_cache()


def test_tuner_weighs_the_gather_and_records_the_path(tmp_path):
    # A large-d/s sketch of wide rows: the single-apply tuner times the LDS
    # tiles, the FP32 atomics and the bucket-sorted gather, keeps the fastest
    # (the gather here), writes every schedule field of it to the JSON file,
    # and the planner then follows the table; the result stays exact.
    import json
    from paper_2606_20195_amd import clear_tuning, load_tuning
    clear_tuning()
    m, n, d, s = 200000, 256, 16384, 4
    A = workloads.integers(m, n, seed=60, lim=4)
    Ad = to_dev(A)
    sk = Sketch(m, d, s, 22, ACC_F32)
    path = str(tmp_path / "tune.json")
    tuned = sk.tune(Ad, cache_path=path)
    assert tuned["gather"] == 1 and tuned["global_atomics"] == 0
    entry = json.load(open(path))["entries"][-1]
    assert entry["gather"] == 1 and "col_tile" in entry and "global_atomics" in entry
    clear_tuning()
    assert load_tuning(path) >= 1
    assert sk.plan(0, m, n)["gather"] == 1
    got = sk.apply(Ad)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), model.apply_f32_exact_int(A, d, s, 22))
    clear_tuning()
