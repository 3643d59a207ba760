"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects invalid calls with the documented codes before any HIP
call is made (fake, never dereferenced pointers are used here)."""
import ctypes
import glob
import os
import re

import pytest

from paper_2606_20195_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(0x10000)      # never dereferenced: every call below fails validation first


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(sketch_\w+|sk_server_\w+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert {"sketch_create", "sketch_apply", "sketch_destroy"} <= names
    for n in names:
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTS) <= names


def test_version(lib):
    assert lib.sketch_version() == 101


def _create(lib, m=1000, d=64, s=4, rounding=0):
    h = ctypes.c_void_p()
    rc = lib.sketch_create(m, d, s, 0, rounding, ctypes.byref(h))
    return rc, h


def test_create_validation(lib):
    assert _create(lib, m=0)[0] == _lib.EINVAL
    assert _create(lib, d=0)[0] == _lib.EINVAL
    assert _create(lib, s=0)[0] == _lib.EINVAL
    assert _create(lib, s=17)[0] == _lib.EINVAL
    assert _create(lib, d=30, s=4)[0] == _lib.EINVAL          # d % s != 0
    assert b"multiple" in lib.sketch_last_error()
    assert _create(lib, rounding=7)[0] == _lib.EINVAL          # 4..6 are the BF16 rules
    assert lib.sketch_create(10, 8, 1, 0, 0, None) == _lib.EINVAL
    rc, h = _create(lib)
    assert rc == 0 and h.value
    assert lib.sketch_destroy(h) == 0
    assert lib.sketch_destroy(None) == 0


def test_apply_validation(lib):
    rc, h = _create(lib, m=1000, d=64, s=4, rounding=0)
    assert rc == 0
    ap = lambda **kw: lib.sketch_apply(   # noqa: E731
        kw.get("h", h), kw.get("A", FAKE), kw.get("dt", 0), kw.get("rows", 100), kw.get("n", 8),
        kw.get("lda", 8), kw.get("off", 0), kw.get("SA", FAKE), kw.get("ldsa", 8), kw.get("flags", 0),
        0, None)
    assert ap(h=None) == _lib.EINVAL
    assert ap(dt=7) == _lib.EINVAL
    assert ap(rows=-1) == _lib.EINVAL
    assert ap(n=0) == _lib.EINVAL
    assert ap(lda=7) == _lib.EINVAL
    assert ap(off=950) == _lib.EINVAL                        # past m
    assert ap(off=-1) == _lib.EINVAL
    assert ap(SA=None) == _lib.EINVAL
    assert ap(ldsa=4) == _lib.EINVAL
    assert ap(A=None) == _lib.EINVAL
    assert ap(flags=2) == _lib.EINVAL
    assert ap(A=ctypes.c_void_p(0x10001), dt=0) == _lib.EINVAL  # misaligned FP32 A
    lib.sketch_destroy(h)
    rc, h16 = _create(lib, m=1000, d=64, s=4, rounding=1)
    # FP16 SA needs 4-byte alignment and an even leading dimension
    assert lib.sketch_apply(h16, FAKE, 1, 10, 8, 8, 0, ctypes.c_void_p(0x10002), 8, 0, 0, None) == _lib.EUNSUPPORTED
    assert lib.sketch_apply(h16, FAKE, 1, 10, 8, 8, 0, FAKE, 9, 0, 0, None) == _lib.EUNSUPPORTED
    lib.sketch_destroy(h16)


def test_schedule_validation(lib):
    rc, h = _create(lib)
    S = _lib.Schedule
    assert lib.sketch_set_schedule(h, ctypes.byref(S(100, 0, 0, 1))) == _lib.EINVAL    # not a multiple of 64
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 3, 0, 1))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 32, 1))) == _lib.EINVAL
    bad = S(0, 0, 0, 1)
    bad.reserved[0] = 1
    assert lib.sketch_set_schedule(h, ctypes.byref(bad)) == _lib.EINVAL
    # column tiles: 32, 8, 4, 2 only, and only with the block groups that have kernels
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 16))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 8, 0, 1, 0, 8))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 2, 0, 1, 0, 2))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 4, 0, 1, 0, 8))) == 0
    # the global-atomic path: 0 or 1, not with the per-contribution scheme
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 0, 2))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 1, 0, 1))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 0, 1))) == 0
    # the bucket-sorted gather: 0 or 1, alone among the workspace paths
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 0, 0, 2))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 0, 1, 1))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 1, 0, 0, 1))) == _lib.EINVAL
    assert lib.sketch_set_schedule(h, ctypes.byref(S(0, 0, 0, 1, 0, 0, 0, 1))) == 0
    assert lib.sketch_set_schedule(h, ctypes.byref(S(4096, 4, 8, 0))) == 0
    assert lib.sketch_set_schedule(h, None) == 0
    lib.sketch_destroy(h)


def test_debug_exports_validation(lib):
    rc, h = _create(lib, m=100)
    assert lib.sketch_hash(h, 90, 20, FAKE, FAKE, None) == _lib.EINVAL
    assert lib.sketch_hash(h, 0, 5, None, FAKE, None) == _lib.EINVAL
    assert lib.sketch_hash(h, 0, 0, None, None, None) == 0              # empty range: nothing to do
    assert lib.sketch_quantize(0, FAKE, FAKE, 4, 0, 0, 0, None) == _lib.EINVAL   # FP32 is not a rounding rule
    assert lib.sketch_quantize(2, FAKE, FAKE, -1, 0, 0, 0, None) == _lib.EINVAL
    assert lib.sketch_quantize(2, None, FAKE, 3, 0, 0, 0, None) == _lib.EINVAL
    assert lib.sketch_quantize(2, None, None, 0, 0, 0, 0, None) == 0
    lib.sketch_destroy(h)


def test_solve_validation(lib):
    rc, h = _create(lib, m=1000, d=64, s=4, rounding=1)
    O = _lib.SolveOpts
    sv = lambda **kw: lib.sketch_solve(   # noqa: E731
        kw.get("h", h), kw.get("A", FAKE), kw.get("dt", 1), kw.get("n", 8), kw.get("lda", 8),
        kw.get("b", FAKE), kw.get("x", FAKE), kw.get("opts", None), None, None)
    assert sv(h=None) == _lib.EINVAL
    assert sv(dt=5) == _lib.EINVAL
    assert sv(n=0) == _lib.EINVAL
    assert sv(lda=4) == _lib.EINVAL
    assert sv(n=65, lda=65) == _lib.EINVAL                     # n > d
    assert sv(A=None) == _lib.EINVAL
    assert sv(b=None) == _lib.EINVAL
    assert sv(x=ctypes.c_void_p(0x10004)) == _lib.EINVAL       # x not 8-byte aligned
    assert sv(A=ctypes.c_void_p(0x10001)) == _lib.EINVAL       # A not element aligned
    bad = O()
    bad.reserved[1] = 3
    assert sv(opts=ctypes.byref(bad)) == _lib.EINVAL
    assert sv(opts=ctypes.byref(O(-1.0))) == _lib.EINVAL
    assert sv(opts=ctypes.byref(O(0.0, 0.0, -2))) == _lib.EINVAL
    lib.sketch_destroy(h)
    rc, hbig = _create(lib, m=100000, d=4096, s=4, rounding=0)
    assert lib.sketch_solve(hbig, FAKE, 0, 2000, 2000, FAKE, FAKE, None, None, None) == _lib.EUNSUPPORTED
    lib.sketch_destroy(hbig)


def test_qr_trinv_validation(lib):
    assert lib.sketch_qr_f32(None, 10, 4, 4, 4, FAKE, None) == _lib.EINVAL
    assert lib.sketch_qr_f32(FAKE, 10, 4, 3, 4, FAKE, None) == _lib.EINVAL   # ldm < cols
    assert lib.sketch_qr_f32(FAKE, 3, 4, 4, 4, FAKE, None) == _lib.EINVAL    # k > rows
    assert lib.sketch_qr_f32(FAKE, 10, 4, 4, 5, FAKE, None) == _lib.EINVAL   # k > cols
    assert lib.sketch_qr_f32(FAKE, 20000, 4, 4, 4, FAKE, None) == _lib.EUNSUPPORTED
    assert lib.sketch_qr_f32(FAKE, 10, 4, 4, 0, FAKE, None) == 0             # nothing to factor
    assert lib.sketch_trinv_f32(FAKE, 0, 4, FAKE, FAKE, 4, FAKE, None) == _lib.EINVAL
    assert lib.sketch_trinv_f32(FAKE, 2000, 2000, FAKE, FAKE, 2000, FAKE, None) == _lib.EINVAL
    assert lib.sketch_trinv_f32(FAKE, 8, 7, FAKE, FAKE, 8, FAKE, None) == _lib.EINVAL
    assert lib.sketch_trinv_f32(FAKE, 8, 8, FAKE, None, 8, FAKE, None) == _lib.EINVAL


def _problem(**kw):
    P = _lib.Problem
    base = dict(m=1000, n=8, d=32, s=4, rounding=1, seed=0, A=0x10000, lda=8, SA=0x20000, ldsa=8, a_dtype=1)
    base.update(kw)
    return P(base["m"], base["n"], base["d"], base["s"], base["rounding"], base["seed"], base["A"], base["lda"],
             base["SA"], base["ldsa"], base["a_dtype"], 0)


def test_batch_validation(lib):
    h = ctypes.c_void_p()
    arr = lambda *ps: (_lib.Problem * len(ps))(*ps)   # noqa: E731
    mk = lambda *ps: lib.sketch_batch_create(arr(*ps), len(ps), None, ctypes.byref(h))   # noqa: E731
    assert lib.sketch_batch_create(None, 0, None, ctypes.byref(h)) == _lib.EINVAL
    assert mk(_problem(m=0)) == _lib.EINVAL
    assert mk(_problem(d=30)) == _lib.EINVAL                                 # d % s
    assert mk(_problem(s=17)) == _lib.EINVAL
    assert mk(_problem(rounding=9)) == _lib.EINVAL
    assert mk(_problem(A=0)) == _lib.EINVAL
    assert mk(_problem(lda=4)) == _lib.EINVAL
    assert mk(_problem(ldsa=9)) == _lib.EUNSUPPORTED                         # FP16 SA needs even ldsa
    assert mk(_problem(), _problem(a_dtype=0)) == _lib.EINVAL                # mixed element types
    assert mk(_problem(), _problem(rounding=0)) == _lib.EINVAL               # mixed accumulation classes
    bad = _problem()
    bad.reserved[0] = 1
    assert mk(bad) == _lib.EINVAL
    S = _lib.Schedule
    assert lib.sketch_batch_create(arr(_problem()), 1, ctypes.byref(S(100, 0, 0, 0)), ctypes.byref(h)) == _lib.EINVAL
    assert lib.sketch_batch_destroy(None) == 0
    assert lib.sketch_batch_apply(None, None) == _lib.EINVAL
    assert lib.sketch_batch_graph(None, None) == _lib.EINVAL


def test_tuning_file_roundtrip(lib, tmp_path):
    lib.sketch_clear_tuning()
    good = tmp_path / "tune.json"
    good.write_text('{"version": 1, "entries": [\n'
                    ' {"key": "apply a=1 r=1 d=1024 s=4 n=64 rows=2^22", "chunk_rows": 4096, "block_group": 4,'
                    ' "waves": 8, "xcd_remap": 1, "ms": 0.2},\n'
                    ' {"key": "batch a=1 acc=f16 k=512 bytes=2^33 nmax=128", "chunk_rows": 8192, "block_group": 4,'
                    ' "waves": 16, "xcd_remap": 0, "ms": 1.5}]}\n')
    assert lib.sketch_load_tuning(str(good).encode()) == 2
    bad = tmp_path / "bad.json"
    bad.write_text('{"version": 1, "entries": [{"chunk_rows": 1}]}')       # entry without a key
    assert lib.sketch_load_tuning(str(bad).encode()) == _lib.EINVAL
    assert lib.sketch_load_tuning(str(tmp_path / "missing.json").encode()) == _lib.EINVAL
    assert lib.sketch_load_tuning(None) == _lib.EINVAL
    assert lib.sketch_clear_tuning() == 0


def test_per_contribution_schedule_validation():
    from paper_2606_20195_amd import ACC_F16_RN, SketchError, Sketch
    sk = Sketch(1000, 64, 4, 1, ACC_F16_RN)
    with pytest.raises(SketchError) as ei:
        sk.set_schedule(per_contribution=2)
    assert ei.value.code == -1
    sk.set_schedule(per_contribution=1)
    sk.clear_schedule()
