"""Pins of the per-call model (units, scale, rounding stream) (CPU only)."""
import numpy as np

import workloads
from oracle import model, quant
from oracle.philox import philox_scalar
from oracle.sketch import TAG_ROUND, apply_f64


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
