"""GPU parity of the per-contribution schedule (one global atomic per
contribution, the paper's Section 4 kernel scheme) through the C ABI.

Bars: bit-exact wherever every sum is exact (small-integer A with c_s a power
of two, any atomic order) and wherever each SA entry receives one
contribution (spikes: the rounding rule and its noise site are then visible
bit for bit); otherwise the FP16 accumulation error against the FP64 oracle
is held to the FP16 summation model (1.5e-4 sqrt(K) + 2e-4 per entry for K
contributions, relative) and to the same order as the sequential model's."""
import numpy as np
import pytest
import torch

import workloads
from oracle import model
from oracle.sketch import apply_f64
from paper_2606_20195_amd import ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, Sketch

pytestmark = pytest.mark.gpu

PC = dict(per_contribution=1)


def run(A, m, d, s, seed, rounding, epoch=0, SA0=None, row_offset=0):
    sk = Sketch(m, d, s, seed, rounding)
    sk.set_schedule(**PC)
    assert sk.plan(1 if A.dtype == np.float16 else 0, A.shape[0], A.shape[1])["per_contribution"] == 1
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    n = A.shape[1]
    dt = torch.float32 if rounding == ACC_F32 else torch.float16
    # FP16 output needs an even leading dimension (packed FP16 atomics)
    SA = torch.zeros((d, n + (n & 1)), dtype=dt, device="cuda")[:, :n]
    if SA0 is not None:
        SA.copy_(torch.from_numpy(SA0))
        sk.apply(Ad, SA=SA, accumulate=True, epoch=epoch, row_offset=row_offset)
    else:
        sk.apply(Ad, SA=SA, epoch=epoch, row_offset=row_offset)
    torch.cuda.synchronize()
    return SA.cpu().numpy()


@pytest.mark.parametrize("rounding", [ACC_F32, ACC_F16_RN, ACC_F16_SR])
@pytest.mark.parametrize("s,n", [(4, 32), (1, 7), (4, 33)])
def test_exact_sums_are_bit_exact(rounding, s, n):
    dt = np.float32 if rounding == ACC_F32 else np.float16
    A = workloads.integers(20000, n, seed=21, lim=4).astype(dt)
    got = run(A, 20000, 512, s, 5, rounding, epoch=2)
    assert np.array_equal(got.astype(np.float64), apply_f64(A, 512, s, 5))


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER])
def test_one_contribution_per_entry_is_bit_exact(rounding):
    # spikes in distinct columns, s = 8 (c_s not an FP16 value): every entry
    # gets at most one nonzero contribution, so the result is its rounding
    m, n, d, s = 16384, 16, 1024, 8
    A = workloads.spikes(m, n, np.float16)
    got = run(A, m, d, s, 17, rounding, epoch=9)
    ref = model.apply_per_contribution_model(A, d, s, 17, rounding, epoch=9)
    assert np.count_nonzero(ref) == n * s
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_row_offset_and_accumulate():
    A = workloads.integers(3000, 16, seed=2, lim=3).astype(np.float16)
    SA0 = workloads.integers(256, 16, seed=3, lim=50).astype(np.float16)
    got = run(A, 100000, 256, 4, 8, ACC_F16_RN, SA0=SA0, row_offset=50000)
    ref = apply_f64(A, 256, 4, 8, row_offset=50000) + SA0.astype(np.float64)
    assert np.array_equal(got.astype(np.float64), ref)


def fp16_bound(K):
    """Twice the FP16 summation model: 1.5e-4 sqrt(K) + 2e-4 relative."""
    return 2.0 * (1.5e-4 * np.sqrt(K) + 2e-4)


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR])
def test_fp16_accumulation_error_follows_the_model(rounding):
    # FP32-stored A, so every contribution is rounded by the rule (Section 4.2)
    m, n, d, s = 65536, 32, 256, 4
    A = workloads.gaussian(m, n, 31, np.float32)
    ref = apply_f64(A, d, s, 4)
    got = run(A, m, d, s, 4, rounding, epoch=1).astype(np.float64)
    seq = model.apply_per_contribution_model(A, d, s, 4, rounding, epoch=1).astype(np.float64)
    e_gpu = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    e_seq = np.linalg.norm(seq - ref) / np.linalg.norm(ref)
    assert e_gpu <= fp16_bound(m * s / d)
    assert 0.5 * e_seq <= e_gpu <= 2.0 * e_seq
    # the partial-sum scheme stays inside the 4e-3 budget on the same input
    lds = Sketch(m, d, s, 4, rounding).apply(torch.from_numpy(A).cuda(), epoch=1)
    torch.cuda.synchronize()
    e_lds = np.linalg.norm(lds.double().cpu().numpy() - ref) / np.linalg.norm(ref)
    assert e_lds <= 4e-3 and e_lds < e_gpu


def test_dither_accumulation_error_is_bounded():
    m, n, d, s = 65536, 32, 256, 4
    A = workloads.gaussian(m, n, 32, np.float32)
    ref = apply_f64(A, d, s, 6)
    got = run(A, m, d, s, 6, ACC_F16_DITHER, epoch=4).astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= fp16_bound(m * s / d)


def test_fp32_per_contribution_non_power_of_two_scale():
    # s = 8: each contribution is fl32(+-fl32(1/sqrt 8) x); FP32 sums in any order
    A = workloads.gaussian(20000, 16, 41, np.float32)
    got = run(A, 20000, 256, 8, 6, ACC_F32).astype(np.float64)
    ref = apply_f64(A, 256, 8, 6)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-6


@pytest.mark.parametrize("rounding", [ACC_F32, ACC_F16_RN])
def test_empty_row_range_clears_or_keeps(rounding):
    sk = Sketch(1000, 64, 4, 2, rounding)
    sk.set_schedule(**PC)
    dt = torch.float32 if rounding == ACC_F32 else torch.float16
    A = torch.zeros((0, 8), dtype=dt, device="cuda")
    SA = torch.full((64, 8), 3.0, dtype=dt, device="cuda")
    sk.apply(A, SA=SA, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(SA == 3.0)
    sk.apply(A, SA=SA)
    torch.cuda.synchronize()
    assert torch.all(SA == 0)
