"""Accuracy of the fixed-point unit partials on real-valued input (needs an MI355X).

The apply kernel sums each unit in fixed point with a per-column exponent
chosen from a sample of the unit's first rows, and keeps the few contributions
far above that exponent (outliers) in FP32 beside it.  With one unit per call
the result is one quantisation per entry, so the GPU must equal the oracle's
model of that computation bit for bit, on Gaussian input, on the coherent
input (100 * I rows over a 1e-3 tail) and on the paper's Table 1 construction
([I_n; tau G / sqrt(m - n)], rows permuted).  Over many units, the entries
that hold only tail contributions must keep their relative precision.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import model, native
from oracle.sketch import apply_f64, hash_rows
from paper_2606_20195_amd import ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, F16, F32, Sketch

pytestmark = pytest.mark.gpu


def _input(kind, rows, n, dtype):
    if kind == "gaussian":
        return workloads.gaussian(rows, n, 21, dtype)
    if kind == "coherent":
        return workloads.coherent(rows, n, 22, dtype)
    return workloads.table1(rows, n, 23, dtype)[0]


def _one_unit(A, d, s, mode, seed=9, r0=100, epoch=11, col_tile=0):
    rows, n = A.shape
    sk = Sketch(rows + r0, d, s, seed, mode)
    sk.set_schedule(chunk_rows=(rows + 63) // 64 * 64, col_tile=col_tile)
    plan = sk.plan(F16 if A.dtype == np.float16 else F32, rows, n)
    SA = sk.apply(torch.from_numpy(A).cuda(), row_offset=r0, epoch=epoch)
    torch.cuda.synchronize()
    return SA.cpu().numpy(), plan


@pytest.mark.parametrize("kind", ["gaussian", "coherent", "table1"])
@pytest.mark.parametrize("mode", [ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER])
@pytest.mark.parametrize("s,d", [(4, 256), (8, 512), (1, 64)])
def test_fp16_one_unit_matches_the_fixed_point_model(kind, mode, s, d):
    A = _input(kind, 8192, 40, np.float16)
    got, plan = _one_unit(A, d, s, mode)
    ref = model.apply_f16_model(A, d, s, 9, mode, 11, chunk_rows=8192, row_offset=100,
                                waves=plan["waves"], block_group=plan["block_group"], col_tile=plan["col_tile"])
    bad = np.flatnonzero(got.view(np.uint16) != ref.view(np.uint16))
    assert bad.size == 0, (bad[:8], got.ravel()[bad[:4]], ref.ravel()[bad[:4]])


@pytest.mark.parametrize("kind", ["gaussian", "coherent", "table1"])
@pytest.mark.parametrize("dt", [np.float32, np.float16])
@pytest.mark.parametrize("s,d", [(4, 256), (2, 128)])
def test_fp32_one_unit_matches_the_fixed_point_model(kind, dt, s, d):
    A = _input(kind, 6000, 33, dt)
    got, plan = _one_unit(A, d, s, ACC_F32)
    ref = model.apply_f32_one_unit_model(A, d, s, 9, row_offset=100, waves=plan["waves"],
                                         block_group=plan["block_group"], col_tile=plan["col_tile"])
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, (bad[:8], got.ravel()[bad[:4]], ref.ravel()[bad[:4]])


@pytest.mark.parametrize("col_tile", [8, 4, 2])
@pytest.mark.parametrize("kind", ["gaussian", "coherent", "table1"])
@pytest.mark.parametrize("mode", [ACC_F16_RN, ACC_F32])
def test_narrow_column_tiles_match_the_model(col_tile, kind, mode):
    """Narrow tiles (quad broadcasts of the row hash, more rows per wave
    instruction) on a 40-column input: the same one-unit bit-exact bar."""
    A = _input(kind, 4096, 40, np.float16)
    d, s = 512, 4
    got, plan = _one_unit(A, d, s, mode, col_tile=col_tile)
    assert plan["col_tile"] == col_tile
    kw = dict(waves=plan["waves"], block_group=plan["block_group"], col_tile=col_tile)
    if mode == ACC_F32:
        ref = model.apply_f32_one_unit_model(A, d, s, 9, row_offset=100, **kw)
        bad = np.flatnonzero(got != ref)
    else:
        ref = model.apply_f16_model(A, d, s, 9, mode, 11, chunk_rows=4096, row_offset=100, **kw)
        bad = np.flatnonzero(got.view(np.uint16) != ref.view(np.uint16))
    assert bad.size == 0, (bad[:8], got.ravel()[bad[:4]], ref.ravel()[bad[:4]])


def _tail_mask(A, d, s, seed, big):
    """Entries of SA that receive no contribution of magnitude >= big."""
    n = A.shape[1]
    rows_big, cols_big = np.nonzero(np.abs(A.astype(np.float64)) >= big)
    mask = np.ones((d, n), dtype=bool)
    if rows_big.size:
        b, _ = hash_rows(seed, rows_big.astype(np.uint64), d, s)
        for j in range(s):
            mask[b[:, j], cols_big] = False
    return mask


def _tail_err(got, ref, mask):
    got = np.asarray(got, dtype=np.float64)
    return float(np.linalg.norm((got - ref)[mask]) / np.linalg.norm(ref[mask]))


@pytest.mark.parametrize("kind", ["coherent", "table1"])
@pytest.mark.parametrize("mode,tol", [(ACC_F16_RN, 4e-3), (ACC_F16_SR, 4e-3), (ACC_F16_DITHER, 4e-3),
                                      (ACC_F32, 1e-5)])
def test_tail_entries_keep_their_precision_over_many_units(kind, mode, tol):
    m, n, d, s = 1 << 17, 64, 256, 4
    A = _input(kind, m, n, np.float16)
    sk = Sketch(m, d, s, 3, mode)
    SA = sk.apply(torch.from_numpy(A).cuda(), epoch=5)
    torch.cuda.synchronize()
    got = SA.float().cpu().numpy()
    ref = apply_f64(A, d, s, 3)
    mask = _tail_mask(A, d, s, 3, 0.5)
    assert mask.sum() > 0.9 * mask.size
    assert _tail_err(got, ref, mask) <= tol
    assert _tail_err(got, ref, ~mask) <= tol


@pytest.mark.parametrize("mode,tol", [(ACC_F16_RN, 4e-3), (ACC_F32, 1e-5)])
def test_full_size_coherent_tail_entries(mode, tol):
    A = workloads.apply_case("coherent", dtype=np.float16)
    m = A.shape[0]
    SA = Sketch(m, 1024, 4, 0, mode).apply(torch.from_numpy(A).cuda())
    torch.cuda.synchronize()
    got = SA.float().cpu().numpy()
    ref = native.sketch_f64(A, 1024, 4, 0)
    mask = _tail_mask(A[:64], 1024, 4, 0, 1.0)
    assert _tail_err(got, ref, mask) <= tol
