"""Pins of the oracle's FP16 quantisers (CPU only).

RN is checked against numpy's float32 -> float16 cast; the directed roundings
by bracketing; SR by exhaustive counting of the noise values that round up
(the rule is unbiased to 2**-24); the FMA of the dither against libm fmaf;
the dither mean against the continuous-noise closed form.
"""
import ctypes
from fractions import Fraction

import numpy as np
import pytest

from oracle import quant


def _random_f32(count, seed):
    g = np.random.default_rng(seed)
    bits = g.integers(0, 2 ** 32, size=count, dtype=np.uint64).astype(np.uint32)
    x = bits.view(np.float32)
    # concentrate on the FP16 range too, including the subnormal and overflow zones
    y = (g.standard_normal(count) * np.exp2(g.integers(-30, 18, size=count))).astype(np.float32)
    return np.concatenate([x, y])


def _bits16(a):
    return np.asarray(a, dtype=np.float16).view(np.uint16)


def test_rn16_matches_numpy_cast():
    x = _random_f32(200_000, 1)
    ties = np.array([1 + 2 ** -11, 1 + 3 * 2 ** -11, 65520.0, 65519.99, 2 ** -25, 3 * 2 ** -25,
                     -2 ** -25, 2048 + 1, 2048 + 3, 0.0, -0.0, np.inf, -np.inf], dtype=np.float32)
    x = np.concatenate([x, ties])
    mine = quant.rn16(x)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(mine), nan)
    assert np.array_equal(_bits16(mine)[~nan], _bits16(ref)[~nan])


def test_rn16_from_f64_matches_numpy_cast_on_f16_sums():
    g = np.random.default_rng(2)
    a = (g.standard_normal(100_000) * np.exp2(g.integers(-20, 12, 100_000))).astype(np.float16)
    b = (g.standard_normal(100_000) * np.exp2(g.integers(-20, 12, 100_000))).astype(np.float16)
    s = a.astype(np.float64) + b.astype(np.float64)     # exact
    ref = s.astype(np.float16)                          # numpy rounds FP64 -> FP16 directly
    fin = np.isfinite(ref)
    assert np.array_equal(_bits16(quant.rn16(s))[fin], _bits16(ref)[fin])


def test_directed_rounding_brackets_with_adjacent_values():
    x = _random_f32(50_000, 3)
    x = x[np.isfinite(x) & (np.abs(x) <= 65504)]
    lo, hi = quant.rd16(x), quant.ru16(x)
    xd = x.astype(np.float64)
    assert np.all(lo.astype(np.float64) <= xd) and np.all(xd <= hi.astype(np.float64))
    exact = lo == hi
    assert np.array_equal(exact, xd == lo.astype(np.float64))
    step = np.nextafter(lo[~exact], np.float16(np.inf))
    assert np.array_equal(_bits16(step), _bits16(hi[~exact]))


def test_sr_up_count_is_exact_and_unbiased():
    g = np.random.default_rng(4)
    u = np.arange(2 ** 24, dtype=np.uint64)
    xs = [np.float32(1 / np.sqrt(8)), np.float32(-2.7182817), np.float32(3e-7)]
    for x in xs:
        r = quant.sr16(np.full(u.shape, x, dtype=np.float32), u).astype(np.float64)
        lo, hi = float(quant.rd16(x)), float(quant.ru16(x))
        up = int(np.count_nonzero(r == hi))
        assert Fraction(up, 2 ** 24) == quant.sr16_up_probability(x)
        # E[SR(x)] = x exactly: (x - lo)/(hi - lo) has at most 24 fractional bits here
        mean = Fraction(lo) + Fraction(up, 2 ** 24) * (Fraction(hi) - Fraction(lo))
        assert mean == Fraction(float(x))


def test_rules_keep_representable_values():
    x = np.array([0.0, 1.0, -0.5, 65504.0, 2 ** -24, 1 + 2 ** -10], dtype=np.float32)
    u = np.arange(x.size, dtype=np.uint64) * 1234567
    # RN and SR return FP16-representable inputs unchanged (dither may not: its
    # noise reaches one ULP, so it is left out here)
    assert np.array_equal(quant.rn16(x).astype(np.float32), x)
    for shift in range(0, 24, 5):
        assert np.array_equal(quant.sr16(x, u << np.uint64(shift)).astype(np.float32), x)


def test_fma32_matches_libm_fmaf():
    libm = ctypes.CDLL("libm.so.6")
    libm.fmaf.restype = ctypes.c_float
    libm.fmaf.argtypes = [ctypes.c_float] * 3
    g = np.random.default_rng(5)
    for _ in range(3000):
        a, b, c = (g.standard_normal(3) * np.exp2(g.integers(-30, 30, 3))).astype(np.float32)
        assert quant.fma32(a, b, c) == float(libm.fmaf(float(a), float(b), float(c)))
    for a, b, c in [(0.0, -1.0, -0.0), (-0.0, -0.0, -0.0), (0.5, -0.0, -0.0), (-0.5, -0.0, -0.0),
                    (0.0, 1.0, -0.0), (-2.0, 3.0, 6.0), (2.0, 3.0, -6.0), (0.0, 2.0, 0.0), (-0.0, 2.0, 0.0),
                    (1e-30, 1e-30, -0.0), (-1e-30, 1e-30, 0.0)]:   # exact zeros and underflow
        ref = float(libm.fmaf(a, b, c))
        got = quant.fma32(a, b, c)
        assert got == ref and np.signbit(got) == np.signbit(ref), (a, b, c, got, ref)
    for _ in range(1000):   # the dither's shape: t in [-1/2, 1/2), x * 2**-10, x
        x = np.float32(g.standard_normal())
        t = np.float32(int(g.integers(0, 2 ** 24)) * 2.0 ** -24 - 0.5)
        xf = np.float32(x * np.float32(2 ** -10))
        assert quant.fma32(t, xf, x) == float(libm.fmaf(float(t), float(xf), float(x)))


@pytest.mark.parametrize("x", [1 / np.sqrt(8), 0.3, 1.7, -0.77])
def test_dither_mean_matches_continuous_noise_closed_form(x):
    x = np.float32(x)
    lo = float(quant.rd16(x))
    ulp = float(quant.ru16(x)) - lo
    # noise xi ~ U[-w/2, w/2) with w = |x| 2**-10; RN picks the nearest FP16
    w = abs(float(x)) * 2.0 ** -10
    tau = (float(x) - lo) / ulp
    def prob_between(a, b):        # P(a <= tau + xi/ulp < b)
        a0, b0 = (a - tau) * ulp, (b - tau) * ulp
        a0, b0 = max(a0, -w / 2), min(b0, w / 2)
        return max(b0 - a0, 0.0) / w
    mean = sum((lo + k * ulp) * prob_between(k - 0.5, k + 0.5) for k in range(-2, 4))
    # the FP32 rounding inside the FMA moves each of the two rounding thresholds by
    # at most half an FP32 ulp, i.e. a probability of 2**-24 |x| / w = 2**-14
    assert abs(float(quant.dither16_mean(x)) - mean) < 2 * 2.0 ** -13 * ulp
    if abs(float(x) - 1 / np.sqrt(8)) < 1e-7:
        assert (float(quant.dither16_mean(x)) - float(x)) / ulp == pytest.approx(0.0641, abs=2e-3)


# ---- BF16 rules: pinned by torch's bfloat16 cast (round-to-nearest-even),
# bracketing of the directed roundings, an exhaustive count of the SR
# decision and the dither's bounds and mean.

def _bf16_samples():
    g = np.random.default_rng(17)
    x = g.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** g.integers(-40, 38, 20000).astype(np.float32)
    extra = np.array([0.0, -0.0, 1.00390625, 1.01171875, -1.01171875, 3.3895314e38, 3.4e38, -3.4e38, np.inf,
                      -np.inf, 1e-40, -1e-41, 2.0 ** -133, 3 * 2.0 ** -134], dtype=np.float32)
    return np.concatenate([x[np.isfinite(x)], extra])


def test_bf16_rn_matches_torch_cast():
    torch = pytest.importorskip("torch")
    x = _bf16_samples()
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(quant.bf16_bits(quant.rnb16(x)), ref)


def test_bf16_directed_roundings_bracket():
    torch = pytest.importorskip("torch")
    x = _bf16_samples()
    x = x[np.isfinite(x) & (np.abs(x) <= quant.BF16_MAX)]
    lo, hi = quant.rdb16(x), quant.rub16(x)
    xd = x.astype(np.float64)
    assert np.all(lo <= xd) and np.all(hi >= xd)
    exact = lo == hi
    assert np.all(lo[exact] == xd[exact])
    # adjacent: nothing representable strictly between them
    for v_lo, v_hi in zip(lo[~exact][:500], hi[~exact][:500]):
        b = torch.tensor([v_lo], dtype=torch.float64).to(torch.bfloat16).view(torch.int16).item() & 0xFFFF
        nxt = torch.tensor([b + (1 if v_lo >= 0 else -1)], dtype=torch.int32).to(torch.int16).view(torch.bfloat16)
        assert float(nxt.double().item()) == v_hi or (v_lo == 0 and v_hi > 0)


@pytest.mark.parametrize("x", [1.0 + 2.0 ** -9, -(3.0 + 2.0 ** -8 + 2.0 ** -12), 7.3e-39, 1.234567e20])
def test_bf16_sr_exhaustive_probability(x):
    x32 = np.float32(x)
    u = np.arange(1 << 24, dtype=np.uint64)
    out = quant.srb16(np.full(u.shape, x32), u)
    lo, hi = float(quant.rdb16(x32)), float(quant.rub16(x32))
    ups = int(np.count_nonzero(out == hi))
    assert np.all((out == hi) | (out == lo))
    p = (Fraction(float(x32)) - Fraction(lo)) / (Fraction(hi) - Fraction(lo))
    assert Fraction(ups, 1 << 24) == p                          # exact: p has at most 16 fraction bits


def test_bf16_sr_beyond_range_is_rn():
    x = np.array([3.39e38, -3.4e38, np.inf, -np.inf], dtype=np.float32)
    assert np.array_equal(quant.bf16_bits(quant.srb16(x, 123)), quant.bf16_bits(quant.rnb16(x)))


def test_bf16_dither_bounds_and_mean():
    g = np.random.default_rng(3)
    x = np.float32(1.0 + 3 * 2.0 ** -10)                         # 3/8 of a BF16 spacing above 1
    u = g.integers(0, 1 << 24, 4000).astype(np.uint64)
    out = quant.ditherb16(np.full(u.shape, x), u)
    assert set(np.unique(out)) <= {1.0, 1.0 + 2.0 ** -7}
    # noise = t * x * 2**-7, t uniform on [-1/2, 1/2): P(up) = P(t x 2**-7 > 1/8 spacing) = 1/2 - 1/8 / x
    p_up = 0.5 - 0.125 / float(x)
    assert abs(np.mean(out == 1.0 + 2.0 ** -7) - p_up) < 4 * np.sqrt(p_up * (1 - p_up) / len(u))
