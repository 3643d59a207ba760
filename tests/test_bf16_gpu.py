"""GPU parity of the BF16 output modes (BF16 as the 16-bit target format of
the paper's Section 4.2; the whole call is summed in FP32 and each entry is
rounded once).

Bars: the quantiser export is bit-exact to the oracle's BF16 rules; integer
inputs (every FP32 sum exact) are bit-exact to the model in every rule,
also when accumulating; Gaussian inputs stay within 4e-3 relative Frobenius
error of the FP64 oracle (one BF16 rounding, about 2^-9 / sqrt 3)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import model, quant
from oracle.sketch import apply_f64
from paper_2606_20195_amd import (ACC_BF16_DITHER, ACC_BF16_RN, ACC_BF16_SR, Batch, Sketch, SketchError,
                                  quantize)

pytestmark = pytest.mark.gpu

MODES = [ACC_BF16_RN, ACC_BF16_SR, ACC_BF16_DITHER]


def bits(t):
    return t.view(torch.int16).cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("mode", MODES)
def test_quantizer_is_bit_exact(mode):
    g = workloads.rng(90 + mode)
    x = (g.standard_normal(3000) * 10.0 ** g.integers(-40, 38, 3000)).astype(np.float32)
    x = np.concatenate([x[np.isfinite(x)], np.array([0, -0.0, 3.39e38, -1e-40, 2.0 ** -133], np.float32)])
    got = quantize(mode, torch.from_numpy(x).cuda(), seed=77, epoch=5, site0=1000).cpu().numpy().view(np.uint16)
    u = model.round_u24(77, 5, np.arange(1000, 1000 + len(x), dtype=np.uint64))
    ref = quant.bf16_bits(quant.quantize_bf16(mode, x, u))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("d,s,n", [(512, 4, 32), (4096, 1, 17), (300, 3, 40)])
def test_integer_inputs_are_bit_exact(mode, d, s, n):
    A = workloads.integers(20000, n, seed=91, lim=4).astype(np.float16)
    sk = Sketch(20000 + 77, d, s, 19, mode)
    SA = sk.apply(torch.from_numpy(A).cuda(), row_offset=77, epoch=3)
    torch.cuda.synchronize()
    assert SA.dtype == torch.bfloat16
    ref = model.apply_bf16_model(A, d, s, 19, mode, 3, row_offset=77)
    assert np.array_equal(bits(SA), quant.bf16_bits(ref))


def test_accumulate_adds_once_in_bf16():
    A = workloads.integers(8000, 24, seed=92, lim=3).astype(np.float32)
    SA0 = workloads.integers(256, 24, seed=93, lim=300).astype(np.float32) * np.float32(0.75)
    sk = Sketch(8000, 256, 4, 20, ACC_BF16_SR)
    SA = torch.from_numpy(SA0).to(torch.bfloat16).cuda()
    sa0 = SA.double().cpu().numpy()
    sk.apply(torch.from_numpy(A).cuda(), SA=SA, accumulate=True, epoch=8)
    torch.cuda.synchronize()
    ref = model.apply_bf16_model(A, 256, 4, 20, ACC_BF16_SR, 8, SA0=sa0)
    assert np.array_equal(bits(SA), quant.bf16_bits(ref))


@pytest.mark.parametrize("mode", MODES)
def test_gaussian_within_tolerance(mode):
    for d, s in ((1024, 4), (8192, 2)):                # 32-column tiles; 2-column tiles (4096 bucket rows)
        A = workloads.gaussian(50000, 32, 94, np.float16)
        SA = Sketch(50000, d, s, 21, mode).apply(torch.from_numpy(A).cuda(), epoch=1)
        torch.cuda.synchronize()
        ref = apply_f64(A, d, s, 21)
        err = np.linalg.norm(SA.double().cpu().numpy() - ref) / np.linalg.norm(ref)
        assert err <= 4e-3, (d, s, err)


def test_bf16_handles_are_refused_by_batches_and_solve():
    A = torch.zeros((1000, 8), dtype=torch.float16, device="cuda")
    sk = Sketch(1000, 64, 4, 1, ACC_BF16_RN)
    with pytest.raises(SketchError) as ei:
        sk.solve(A, torch.zeros(1000, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -2
    SA = torch.zeros((64, 8), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(SketchError) as ei:
        Batch([dict(A=A, SA=SA, d=64, s=4, seed=1, rounding=ACC_BF16_RN)])
    assert ei.value.code == -2


def test_empty_row_range_clears_or_keeps():
    sk = Sketch(1000, 64, 4, 2, ACC_BF16_SR)
    A = torch.zeros((0, 8), dtype=torch.float16, device="cuda")
    SA = torch.full((64, 8), 3.0, dtype=torch.bfloat16, device="cuda")
    sk.apply(A, SA=SA, accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(SA == 3.0)
    sk.apply(A, SA=SA)
    torch.cuda.synchronize()
    assert torch.all(SA == 0)
