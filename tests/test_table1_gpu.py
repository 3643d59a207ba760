"""The paper's Table 1 experiment at a reduced size, against the FP64 oracle
(needs an MI355X).

Section 5.3 solves the coherent adversarial least-squares problem
A = [I_n; tau G / sqrt(m - n)] (tau = 1e-3, noise 0.5 on the identity block
of b, rows permuted) by sketch-and-solve: x0 = argmin ||S A x - S b|| with an
FP32 QR of SA.  Here m = 2^17, n = 64, A stored in FP32, for CountSketch
(s = 1) and SparseStack (s = 4) with FP32 accumulation and every FP16 rule.
The GPU's kappa(SA) (FP64 SVD of the GPU's SA) and sketch-and-solve residual
||A x0 - b|| / ||b|| are compared with the oracle's FP64 sketch-and-solve with
the same S; the paper's qualitative findings are checked on the GPU values:
CountSketch's kappa(SA) and residual far above SparseStack's, and FP16
SparseStack as accurate as FP32 SparseStack.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle.sketch import apply_f64, condition_number
from paper_2606_20195_amd import ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, Sketch

pytestmark = pytest.mark.gpu

M, N, SEED = 1 << 17, 64, 31
METHODS = [("countsketch", 1, ACC_F32), ("countsketch_mxp", 1, ACC_F16_RN), ("sparsestack", 4, ACC_F32),
           ("sparsestack_detm", 4, ACC_F16_RN), ("sparsestack_dither", 4, ACC_F16_DITHER),
           ("sparsestack_stoch", 4, ACC_F16_SR)]


@pytest.fixture(scope="module")
def problem():
    A, b, _ = workloads.table1(M, N, 41, np.float32)
    return A, b, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda()


def oracle_sketch_and_solve(A, b, d, s):
    """FP64 sketch of [A | b] with the same S, then the FP64 least-squares
    solution of the sketched problem and its residual on the full problem."""
    SAb = apply_f64(np.column_stack([A.astype(np.float64), b]), d, s, SEED)
    SA, Sb = SAb[:, :-1], SAb[:, -1]
    x0 = np.linalg.lstsq(SA, Sb, rcond=None)[0]
    res = np.linalg.norm(A.astype(np.float64) @ x0 - b) / np.linalg.norm(b)
    return res, condition_number(SA)


@pytest.fixture(scope="module")
def results(problem):
    A, b, Ad, bd = problem
    out = {}
    for ratio in (2, 4):
        d = ratio * N
        for name, s, code in METHODS:
            sk = Sketch(M, d, s, SEED, code)
            SA = sk.apply(Ad).double().cpu().numpy()
            _, info = sk.solve(Ad, bd, raise_on_notconv=False)
            res64, kap64 = oracle_sketch_and_solve(A, b, d, s)
            out[(ratio, name)] = dict(kappa=condition_number(SA), kappa64=kap64,
                                      res=info["rel_residual_x0"], res64=res64,
                                      refined=info["rel_residual"], converged=info["converged"])
    return out


# Residual bars against the FP64 sketch-and-solve.  FP32: the GPU's x0 comes
# from an FP32 QR of SA, whose error grows with kappa(SA) (backward stable QR:
# |dx| / |x| about kappa * 2^-24), so the bar is 1e-3 relative plus
# 20 kappa 2^-24 absolute (CountSketch: kappa ~ 4e3).  FP16 rules: the stored
# FP16 sketch perturbs SA by about 2^-11 per entry; RN and SR within 10 %.
# Dither adds noise of up to one FP16 ulp per entry on purpose, which the
# paper's Table 1 shows as an 8-9 % higher residual than FP32 at every d/n;
# it is held within 25 %.
RES_REL = {ACC_F32: 1e-3, ACC_F16_RN: 0.1, ACC_F16_SR: 0.1, ACC_F16_DITHER: 0.25}


@pytest.mark.parametrize("ratio", [2, 4])
@pytest.mark.parametrize("name,s,code", METHODS)
def test_kappa_and_sketch_and_solve_residual_match_the_oracle(results, ratio, name, s, code):
    r = results[(ratio, name)]
    fp32 = code == ACC_F32
    assert abs(r["kappa"] - r["kappa64"]) <= (1e-4 if fp32 else 5e-3) * r["kappa64"], r
    extra = 20 * r["kappa64"] * 2.0 ** -24 if fp32 else 0.0
    assert abs(r["res"] - r["res64"]) <= RES_REL[code] * r["res64"] + extra, r
    assert r["converged"] == 1


@pytest.mark.parametrize("ratio", [2, 4])
def test_the_papers_orderings_hold(results, ratio):
    ss = results[(ratio, "sparsestack")]
    cs = results[(ratio, "countsketch")]
    assert cs["kappa"] > 20 * ss["kappa"]
    assert cs["res"] > 20 * ss["res"]
    for name, bar in (("sparsestack_detm", 1.1), ("sparsestack_stoch", 1.1), ("sparsestack_dither", 1.25)):
        assert results[(ratio, name)]["res"] <= bar * ss["res"], (name, results[(ratio, name)], ss)
    # refinement reaches the same optimum from every start
    best = min(results[(ratio, n)]["refined"] for n, _, _ in METHODS)
    for n, _, _ in METHODS:
        assert results[(ratio, n)]["refined"] <= best * (1 + 1e-6)
