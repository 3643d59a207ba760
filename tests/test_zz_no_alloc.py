"""sketch_apply_noalloc against sketch_apply (needs an MI355X).

The no-allocation entry point runs the same kernels with the library's static
device scratch in place of the handle's workspace.  Each case makes two calls
in a row on the same GPU, the second with a smaller input, and compares each
with sketch_apply on the same input: bit for bit where the result is
deterministic (integer input, whose FP32 sums are exact in any order).
"""
import numpy as np
import pytest
import torch

import workloads
from paper_2606_20195_amd import ACC_BF16_SR, ACC_F16_DITHER, ACC_F32, SketchError, Sketch

pytestmark = pytest.mark.gpu


def _pair(m, d, s, rounding, A, epoch=3, accumulate=False, sa0=None, sched=None):
    sk = Sketch(m, d, s, 17, rounding)
    if sched:
        sk.set_schedule(**sched)
    dev = torch.from_numpy(A).cuda()
    n = A.shape[1]
    ref = sk.empty_output(n) if sa0 is None else sa0.clone()
    got = torch.zeros_like(ref) if sa0 is None else sa0.clone()
    sk.apply(dev, SA=ref, epoch=epoch, accumulate=accumulate)
    sk.apply(dev, SA=got, epoch=epoch, accumulate=accumulate, noalloc=True)
    torch.cuda.synchronize()
    return got.cpu(), ref.cpu()


GLOBAL = dict(global_atomics=1)


@pytest.mark.parametrize("rounding,d,s,sched", [
    (ACC_F32, 4096, 1, GLOBAL),           # the global-atomic path: workspace of the whole call
    (ACC_F16_DITHER, 8192, 2, GLOBAL),    # the same with one FP16 rounding per entry
    (ACC_BF16_SR, 256, 4, None),          # BF16 output: FP32 sum of the call, then one rounding
    (ACC_F32, 16384, 4, dict(gather=1)),  # the bucket-sorted gather: sum and lists in the scratch
])
def test_noalloc_matches_apply_on_two_calls(rounding, d, s, sched):
    for rows, n in ((30000, 48), (9000, 20)):          # second call smaller
        A = workloads.integers(rows, n, seed=rows + n, lim=4).astype(np.float32)
        got, ref = _pair(rows, d, s, rounding, A, sched=sched)
        assert torch.equal(got.view(torch.int16) if got.dtype != torch.float32 else got,
                           ref.view(torch.int16) if ref.dtype != torch.float32 else ref)


def test_noalloc_accumulate_with_a_non_power_of_two_scale():
    # FP32 accumulation into SA with 1/sqrt(8): the sum goes through the scratch
    for rows, n in ((20000, 40), (5000, 8)):
        A = workloads.integers(rows, n, seed=rows, lim=4).astype(np.float32)
        sa0 = torch.full((256, n), 0.25, device="cuda")
        got, ref = _pair(rows, 256, 8, ACC_F32, A, accumulate=True, sa0=sa0)
        assert torch.equal(got, ref)


def test_noalloc_rejects_workspaces_beyond_the_scratch():
    sk = Sketch(1000, 1 << 18, 1, 0, ACC_F32)            # d x n = 2^18 * 32 floats > 2^22
    sk.set_schedule(global_atomics=1)
    A = torch.zeros((1000, 32), device="cuda")
    SA = torch.zeros((1 << 18, 32), device="cuda")
    with pytest.raises(SketchError, match="scratch"):
        sk.apply(A, SA=SA, noalloc=True)
    # a call that needs no workspace runs at any size
    sk2 = Sketch(1000, 1024, 4, 0, ACC_F32)
    SA2 = torch.zeros((1024, 32), device="cuda")
    sk2.apply(A, SA=SA2, noalloc=True)
    torch.cuda.synchronize()
    assert torch.count_nonzero(SA2).item() == 0
