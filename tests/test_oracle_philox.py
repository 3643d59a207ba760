"""Pins of the oracle's Philox4x32-10 (CPU only).

The oracle's generator is checked against rocRAND's philox4x32_10 engine, an
independent third-party implementation called through its public API
(seed -> key, subsequence -> counter words 2-3, offset/4 -> counter words 0-1),
and the three implementations written for this library (Python integers,
numpy, C) are checked against each other.
"""
import numpy as np

from oracle import native
from oracle.philox import philox, philox_scalar
from oracle.sketch import TAG_ROUND, TAG_SKETCH


def _rocrand(lib, ctr, key):
    seed = int(key[0]) | (int(key[1]) << 32)
    sub = int(ctr[2]) | (int(ctr[3]) << 32)
    off = 4 * (int(ctr[0]) | (int(ctr[1]) << 32))
    out = np.zeros(4, dtype=np.uint32)
    lib.rr_philox_next4(seed, sub, off, out.ctypes.data)
    return tuple(int(v) for v in out)


def _cases(count=300, seed=11):
    g = np.random.default_rng(seed)
    cases = []
    for k in range(count):
        ctr = [int(v) for v in g.integers(0, 2 ** 32, size=4)]
        ctr[1] >>= 2        # rocRAND's 64-bit offset is 4 * (ctr0 + 2**32 ctr1)
        if k % 3 == 0:
            ctr[3] = TAG_SKETCH
            ctr[2] = int(g.integers(0, 4))
        elif k % 3 == 1:
            ctr[3] = TAG_ROUND
        key = [int(v) for v in g.integers(0, 2 ** 32, size=2)]
        cases.append((tuple(ctr), tuple(key)))
    cases += [((0, 0, 0, 0), (0, 0)), ((2 ** 32 - 1, 2 ** 30 - 1, 2 ** 32 - 1, 2 ** 32 - 1), (2 ** 32 - 1,) * 2)]
    return cases


def test_philox_matches_rocrand(rocrand_ref):
    for ctr, key in _cases():
        assert philox_scalar(ctr, key) == _rocrand(rocrand_ref, ctr, key), (ctr, key)


def test_philox_three_implementations_agree():
    cases = _cases(500, seed=12)
    ctr = np.array([c for c, _ in cases], dtype=np.uint64)
    key = np.array([k for _, k in cases], dtype=np.uint64)
    vec = philox(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], key[:, 0], key[:, 1])
    for t, (c, k) in enumerate(cases):
        ref = philox_scalar(c, k)
        assert tuple(int(v[t]) for v in vec) == ref
        assert native.philox(c, k) == ref


def test_philox_output_bits_balanced():
    # 2**16 blocks: every output bit is set about half the time.
    i = np.arange(2 ** 16, dtype=np.uint64)
    words = np.stack(philox(i, 0, 0, TAG_SKETCH, 0x1234, 0x5678)).astype(np.uint64)
    bits = ((words[..., None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)).mean(axis=1)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / np.sqrt(2 ** 16))
