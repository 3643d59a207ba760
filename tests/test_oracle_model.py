"""Pins of the per-call model (units, scale, rounding stream) (CPU only)."""
import numpy as np

import workloads
from oracle import model, quant
from oracle.philox import philox_scalar
from oracle.sketch import TAG_ROUND, apply_f64, hash_rows


def test_f32_exact_int_matches_fp64_when_representable():
    A = workloads.integers(3000, 8, 1)
    for s in (1, 4, 8, 2):
        exact = model.apply_f32_exact_int(A, 64, s, 5)
        f64 = apply_f64(A, 64, s, 5)
        # two roundings away from the FP64 value: fl32(c_s) and the product
        assert np.allclose(exact, f64, rtol=2 ** -22, atol=1e-12)
        if s in (1, 4):          # c_s is a power of two: exactly the FP64 value rounded
            assert np.array_equal(exact, f64.astype(np.float32))


def test_round_stream_words():
    seed, epoch = 0x1122334455667788, 9
    q = np.array([0, 1, 2, 3, 4, 7, 2 ** 35 + 5], dtype=np.uint64)
    u = model.round_u24(seed, epoch, q)
    for qi, ui in zip(q, u):
        c = int(qi) >> 2
        w = philox_scalar((c & 0xFFFFFFFF, c >> 32, epoch, TAG_ROUND),
                          (seed & 0xFFFFFFFF, seed >> 32))[int(qi) & 3]
        assert int(ui) == (w & 0xFFFFFF)


def test_f16_model_one_unit_is_one_quantisation():
    A = workloads.integers(500, 6, 2)
    d, s = 32, 8
    P = apply_f64(A, d, s, 3, scale=1.0)
    v = (model.c_s32(s) * P.astype(np.float32)).astype(np.float32)
    site = np.arange(d * 6, dtype=np.uint64).reshape(d, 6)
    u = model.round_u24(3, 4, site)
    for mode, ref in [(1, quant.rn16(v)), (2, quant.sr16(v, u)), (3, quant.dither16(v, u))]:
        got = model.apply_f16_model(A, d, s, 3, mode, 4, chunk_rows=1000)
        assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_f16_model_units_accumulate_close_to_fp64():
    A = workloads.gaussian(20000, 8, 3)
    ref = apply_f64(A, 64, 4, 1)
    for mode in (1, 2, 3):
        got = model.apply_f16_model(A, 64, 4, 1, mode, 0, chunk_rows=2000).astype(np.float64)
        assert np.linalg.norm(got - ref) <= 4e-3 * np.linalg.norm(ref)


# ---- the fixed-point work item (per-column exponent, outlier list) ---------

def _item(X, W=16, waves=8, dual=False, seed=0):
    """One work item (one block) of rows X with a seeded random bucket map."""
    g = workloads.rng(seed)
    R = X.shape[0]
    bk = g.integers(0, W, size=(R, 1))
    sg = np.where(g.random((R, 1)) < 0.5, -1, 1)
    return model.work_item_partial(X, bk, sg, W, waves, dual), bk, sg


def _exact(X, bk, sg, W):
    P = np.zeros((W, X.shape[1]))
    np.add.at(P, bk[:, 0], sg[:, 0:1] * X)
    return P


def test_column_grid_is_set_by_the_sample_and_small_values_round_to_it():
    # column 0: sample values 3/8 -> E = binade(0.375) + 2 = 0, S = 19: a value
    # of 2^-21 lies below half the grid 2^-19 and vanishes; 5 * 2^-20 rounds
    # to 2 * 2^-19 (ties to even); column 1 is all 2^-10 -> E = -8, S = 27.
    R = 1024
    X = np.zeros((R, 2))
    X[:, 0] = 0.375
    X[700, 0] = 2.0 ** -21
    X[701, 0] = 5 * 2.0 ** -20
    X[:, 1] = 2.0 ** -10
    (P, h, n_out, redone), bk, sg = _item(X)
    assert h == 0 and n_out == 0 and not redone
    expect = _exact(X, bk, sg, 16)
    # the grid value of 5 * 2^-20 is 2.5 * 2^-19 -> 2 * 2^-19: it loses 2^-20
    loss = np.zeros_like(expect)
    loss[bk[700, 0], 0] += sg[700, 0] * 2.0 ** -21
    loss[bk[701, 0], 0] += sg[701, 0] * 2.0 ** -20
    assert np.array_equal(P.astype(np.float64), (expect - loss).astype(np.float32))


def test_outliers_bypass_the_field_and_are_added_in_fp32():
    # three large values in column 0 (fewer than the sample rank): outliers,
    # each one record per block; the rest keeps the fine grid
    R = 2048
    X = workloads.rng(4).standard_normal((R, 3)) * 1e-3
    X[[5, 300, 1500], 0] = [100.0, -250.0, 7.0]
    (P, h, n_out, redone), bk, sg = _item(X, W=64)
    assert n_out == 3 and not redone
    exact = _exact(X, bk, sg, 64)
    small = X.copy()
    small[[5, 300, 1500], 0] = 0.0
    ex_small = _exact(small, bk, sg, 64)
    # tail entries: within the fixed-point grid (2^(E-19) per contribution)
    big_rows = {bk[5, 0], bk[300, 0], bk[1500, 0]}
    mask = np.ones_like(exact, dtype=bool)
    for b in big_rows:
        mask[b, 0] = False
    err = np.abs(P.astype(np.float64) - exact)[mask]
    assert err.max() <= 64 * 2.0 ** -27                   # E = -8 -> grid 2^-27
    # entries holding an outlier: fl32(fl32(small part) + outlier) per row
    for i in (5, 300, 1500):
        b = bk[i, 0]
        expect = np.float32(np.float32(ex_small[b, 0]) + np.float32(sg[i, 0] * X[i, 0]))
        if sum(bk[j, 0] == b for j in (5, 300, 1500)) == 1:
            assert P[b, 0] == expect


def test_four_large_values_set_the_exponent_and_overflowing_lists_redo_at_the_maximum():
    R = 4096
    X = workloads.rng(5).standard_normal((R, 1)) * 1e-3
    # four sample lanes (rows 0, 1, 2, 3 are lanes k = 0..3 of wave 0) hold 10:
    # the 4th largest lane maximum is 10, so nothing is an outlier
    X[0:4, 0] = 10.0
    (P, h, n_out, redone), bk, sg = _item(X)
    assert n_out == 0 and not redone
    # 1100 values of 10 outside the sample: the list (1024 records) overflows,
    # the item is redone with E = binade(10) = 3 and keeps every value exact
    Y = workloads.rng(6).standard_normal((R, 1)) * 1e-3
    Y[2048:2048 + 1100, 0] = 10.0
    (P, h, n_out, redone), bk, sg = _item(Y)
    assert redone and n_out == 0
    assert np.allclose(P, _exact(Y, bk, sg, 16), rtol=0, atol=4096 * 2.0 ** -16)


def test_count_headroom_grows_when_a_bucket_row_takes_many_rows():
    R = 3000
    X = np.ones((R, 2))
    g = workloads.rng(7)
    bk = np.zeros((R, 1), dtype=np.int64)          # every row in bucket row 0
    sg = np.where(g.random((R, 1)) < 0.5, -1, 1)
    P, h, n_out, redone = model.work_item_partial(X, bk, sg, 4, 8, False)
    assert h == 2 and redone                       # K = 3000 needs K < 2^(10+h)
    assert P[0, 0] == sg.sum()


def test_dual_fields_carry_the_residual():
    R = 1024
    X = workloads.rng(8).standard_normal((R, 4)).astype(np.float32).astype(np.float64)
    (P, h, n_out, redone), bk, sg = _item(X, dual=True)
    exact = _exact(X, bk, sg, 16)
    # grid 2^(E - 40) with E <= 4 for N(0,1) samples: far below FP32 rounding
    assert np.max(np.abs(P - exact) / np.maximum(np.abs(exact), 1.0)) <= 2.0 ** -23
    (P1, _, _, _), _, _ = _item(X, dual=False)
    assert np.max(np.abs(P1 - exact)) > np.max(np.abs(P - exact))


def test_whole_call_model_on_integers_is_the_exact_one_unit_result():
    # integer sums are exact in every model: the whole-call model must agree
    # with the FP32 exact-integer result and with the fixed-point unit model
    # run with one unit spanning the call
    A = workloads.integers(4000, 10, 7, lim=5)
    d, s = 96, 3
    assert np.array_equal(model.apply_whole_call_model(A, d, s, 8, model.ACC_F32),
                          model.apply_f32_exact_int(A, d, s, 8))
    sa0 = np.full((d, 10), 0.5, dtype=np.float32)
    assert np.array_equal(model.apply_whole_call_model(A, d, s, 8, model.ACC_F32, SA0=sa0),
                          model.apply_f32_exact_int(A, d, s, 8, SA0=sa0))
    for mode in (model.ACC_F16_RN, model.ACC_F16_SR, model.ACC_F16_DITHER):
        got = model.apply_whole_call_model(A, d, s, 8, mode, epoch=3, row_offset=100)
        ref = model.apply_f16_model(A, d, s, 8, mode, 3, chunk_rows=4000, row_offset=100)
        assert np.array_equal(got.view(np.uint16), ref.view(np.uint16)), mode


def test_whole_call_model_brute_force_on_one_row():
    # one row: entry (b_j, c) holds fl32(c_s * sign_j * x_c), rounded to FP16
    # to nearest by numpy's own conversion; every other entry is zero
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 7)).astype(np.float32)
    d, s, r0 = 40, 4, 123
    b, sg = hash_rows(9, [r0], d, s)
    cs = np.float32(1.0 / np.sqrt(4.0))
    want32 = np.zeros((d, 7), dtype=np.float32)
    for j in range(s):
        want32[b[0, j]] = (cs * (np.float32(sg[0, j]) * x[0])).astype(np.float32)
    got32 = model.apply_whole_call_model(x, d, s, 9, model.ACC_F32, row_offset=r0)
    assert np.array_equal(got32, want32)
    got16 = model.apply_whole_call_model(x, d, s, 9, model.ACC_F16_RN, row_offset=r0)
    assert np.array_equal(got16.view(np.uint16), want32.astype(np.float16).view(np.uint16))


def test_whole_call_model_gaussian_is_the_fp32_rounding_of_fp64():
    A = workloads.gaussian(3000, 5, 11, np.float32)
    d, s = 64, 8
    got = model.apply_whole_call_model(A, d, s, 2, model.ACC_F32)
    f64 = apply_f64(A, d, s, 2)
    # fl32 of the unscaled sum, then fl32 of c_s times it: within 2^-23 relative
    assert np.allclose(got, f64, rtol=2 ** -22, atol=0)


def test_count_headroom_starts_from_the_average_bucket_count():
    # 16384 rows over 8 bucket rows: 2048 on average, so the item starts at
    # h = 2 (3 * 2048 / 2 + 64 < 2^12) and is not recomputed; 4096 rows over
    # 16 bucket rows (256: 448 < 2^10) start at h = 0, 2048 over 4 (512: 832)
    # too; the exact integer sums come out whatever h is
    g = workloads.rng(9)
    for R, W, h_want in ((16384, 8, 2), (4096, 16, 0), (2048, 4, 0), (6000, 4, 2)):
        X = g.integers(-3, 4, size=(R, 2)).astype(np.float64)
        bk = g.integers(0, W, size=(R, 1))
        sg = np.where(g.random((R, 1)) < 0.5, -1, 1)
        P, h, n_out, redone = model.work_item_partial(X, bk, sg, W, 8, False)
        assert h == h_want and not redone, (R, W, h)
        assert np.array_equal(P, _exact(X, bk, sg, W).astype(np.float32))
