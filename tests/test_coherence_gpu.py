"""The coherence sweep's properties at a size the oracle finishes quickly
(the paper's Section 5 coherence sweep; the full m = 2^21, n = 1024 sweep is
`bench.py --coherence`).

U(alpha) = orth((1 - alpha) Q_rand + alpha [I; 0]), stored in FP32.  Bars:
the FP32 sketch's distortion equals the FP64 oracle's (same S) to 1e-5; the
FP16 rounding rules move it by less than 5e-3 (the paper's observation that
the rounding rule does not matter); at full coherence CountSketch (s = 1)
loses the embedding (two coordinate rows share a bucket) while SparseStack
(s = 4) keeps a bounded distortion."""
import numpy as np
import pytest
import torch

import workloads
from oracle.sketch import apply_f64, coherence, distortion
from paper_2606_20195_amd import ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, Sketch

pytestmark = pytest.mark.gpu

M, N, D = 1 << 15, 64, 256


def basis(alpha):
    Q = np.linalg.qr(workloads.rng(81).standard_normal((M, N)))[0]
    X = (1.0 - alpha) * Q
    X[:N] += alpha * np.eye(N)
    return np.linalg.qr(X)[0].astype(np.float32)


@pytest.mark.parametrize("alpha", [0.0, 0.9, 1.0])
def test_distortion_against_the_oracle(alpha):
    U = basis(alpha)
    mu = coherence(U.astype(np.float64))
    if alpha == 1.0:
        assert abs(mu - M / N) < 1e-6
    if alpha == 0.0:
        assert mu < 10
    Ud = torch.from_numpy(U).cuda()
    etas = {}
    for s in (1, 4):
        eta64 = distortion(apply_f64(U, D, s, 3))
        for rounding in (ACC_F32, ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER):
            SA = Sketch(M, D, s, 3, rounding).apply(Ud, epoch=1)
            torch.cuda.synchronize()
            eta = distortion(SA.double().cpu().numpy())
            tol = 1e-5 if rounding == ACC_F32 else 5e-3
            assert abs(eta - eta64) <= tol, (s, rounding, eta, eta64)
        etas[s] = eta64
    if alpha == 1.0:
        assert etas[1] > 0.99 and etas[4] < 0.9
