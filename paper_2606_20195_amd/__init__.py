"""Sparse oblivious subspace embeddings on MI355X (gfx950).

Python binding of libsketch.so (include/sketch.h).  PyTorch supplies device
memory and streams; the binding only marshals tensor pointers, shapes and
the current HIP stream into the C ABI.  All arithmetic happens in the
library's HIP kernels.

    sk = Sketch(m, d, s, seed, rounding=ACC_F16_RN)
    SA = sk.apply(A)                      # A: (rows, n) CUDA tensor
"""
from __future__ import annotations

import ctypes

from ._lib import (ACC_BF16_DITHER, ACC_BF16_RN, ACC_BF16_SR, ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32,
                   ACCUMULATE, BF16, ENOTCONV, F16, F32,
                   Problem, Request, Result, Schedule, ServerInfo, SketchError, SolveInfo, SolveOpts, check, load)

__all__ = ["Sketch", "SketchError", "Schedule", "Batch", "Server", "simulate_admission", "tune_batch", "load_tuning", "clear_tuning", "quantize",
           "qr_f32", "trinv_f32", "version", "sync", "stream_read", "ACC_F32",
           "ACC_F16_RN",
           "ACC_F16_SR", "ACC_F16_DITHER", "ACC_BF16_RN", "ACC_BF16_SR", "ACC_BF16_DITHER", "F32", "F16", "BF16",
           "ACCUMULATE"]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float16:
        return F16
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError("unsupported dtype %s" % t.dtype)


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _matrix(t, name):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D tensor with unit column stride" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    return t.stride(0)


def version():
    return load().sketch_version()


def stream_read(t, out, stream=None):
    """Read every byte of the contiguous device tensor t once (the read
    ceiling measurement, sketch_stream_read); out: an int32 device tensor of
    256 elements that receives the XOR folds."""
    check(load().sketch_stream_read(ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size(),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)), "sketch_stream_read")


def sync(stream=None):
    """Wait for the library's work on `stream` and raise on an asynchronous
    HIP failure of that work (sketch_sync)."""
    check(load().sketch_sync(None, _stream(stream)), "sketch_sync")


class Sketch:
    """S (d x m) = SparseStack with s nonzeros per column (s = 1: CountSketch)."""

    def __init__(self, m, d, s, seed=0, rounding=ACC_F32):
        self._lib = load()
        h = ctypes.c_void_p()
        check(self._lib.sketch_create(int(m), int(d), int(s), int(seed) & (2 ** 64 - 1), int(rounding),
                                      ctypes.byref(h)), "sketch_create")
        self._h = h
        self.m, self.d, self.s, self.seed, self.rounding = int(m), int(d), int(s), int(seed), int(rounding)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sketch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def out_dtype(self):
        torch = _torch()
        if self.rounding == ACC_F32:
            return torch.float32
        return torch.bfloat16 if self.rounding >= ACC_BF16_RN else torch.float16

    def empty_output(self, n, device=None):
        torch = _torch()
        return torch.empty((self.d, n), dtype=self.out_dtype, device=device or "cuda")

    def apply(self, A, SA=None, row_offset=0, accumulate=False, epoch=0, stream=None, noalloc=False):
        """SA = S[:, row_offset:row_offset+rows] @ A (or +=, with accumulate).
        noalloc: call sketch_apply_noalloc (no device allocation; SA must be
        given, the library's static scratch takes any workspace)."""
        if noalloc and SA is None:
            raise ValueError("noalloc needs SA")
        lda = _matrix(A, "A")
        rows, n = A.shape
        if SA is None:
            SA = self.empty_output(n, A.device)
        ldsa = _matrix(SA, "SA")
        if SA.dtype != self.out_dtype or tuple(SA.shape) != (self.d, n):
            raise ValueError("SA must be a (%d, %d) %s tensor" % (self.d, n, self.out_dtype))
        fn = self._lib.sketch_apply_noalloc if noalloc else self._lib.sketch_apply
        check(fn(self._h, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), rows, n, lda,
                 int(row_offset), ctypes.c_void_p(SA.data_ptr()), ldsa,
                 ACCUMULATE if accumulate else 0, int(epoch) & 0xFFFFFFFF,
                 _stream(stream)), "sketch_apply_noalloc" if noalloc else "sketch_apply")
        return SA

    def solve(self, A, b, x=None, tol=0.0, inner_tol=0.0, max_refine=0, max_inner=0, epoch=0, stream=None,
              raise_on_notconv=True):
        """x = argmin ||A x - b|| (FP64) for A (m x n, this sketch's m) on the device.

        b: FP64 device vector of m values.  Returns (x, info dict).  Zero
        options take the library defaults (tol 1e-10, inner_tol 1e-6,
        max_refine 10, max_inner 100).
        """
        torch = _torch()
        lda = _matrix(A, "A")
        m, n = A.shape
        if m != self.m:
            raise ValueError("A has %d rows, the sketch has m = %d" % (m, self.m))
        if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m or not b.is_cuda:
            raise ValueError("b must be a contiguous FP64 device vector of %d values" % m)
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=A.device)
        if x.dtype != torch.float64 or not x.is_contiguous() or x.numel() != n:
            raise ValueError("x must be a contiguous FP64 vector of %d values" % n)
        opts = SolveOpts(float(tol), float(inner_tol), int(max_refine), int(max_inner), int(epoch) & 0xFFFFFFFF)
        info = SolveInfo()
        rc = self._lib.sketch_solve(self._h, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), n, lda,
                                    ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                    ctypes.byref(opts), ctypes.byref(info), _stream(stream))
        if rc != ENOTCONV or raise_on_notconv:
            check(rc, "sketch_solve")
        return x, info.as_dict()

    def tune(self, A, SA=None, cache_path=None, stream=None):
        """Time candidate schedules for sketch_apply on A (SA is overwritten);
        the winner is used by later calls with the same signature."""
        lda = _matrix(A, "A")
        rows, n = A.shape
        if SA is None:
            SA = self.empty_output(n, A.device)
        sch = Schedule()
        check(self._lib.sketch_tune_apply(self._h, ctypes.c_void_p(A.data_ptr()), _dtype_code(A), rows, n, lda,
                                          ctypes.c_void_p(SA.data_ptr()), _matrix(SA, "SA"),
                                          cache_path.encode() if cache_path else None, ctypes.byref(sch),
                                          _stream(stream)), "sketch_tune_apply")
        return sch.as_dict()

    def set_schedule(self, chunk_rows=0, block_group=0, waves=0, xcd_remap=1, per_contribution=0, col_tile=0,
                     global_atomics=0, gather=0):
        """per_contribution=1: one global atomic per contribution (the paper's
        kernel scheme, a slow reference); the other fields are then ignored.
        global_atomics=1 / gather=1: the d x n FP32 workspace paths (FP32
        atomics, or rows listed by bucket and summed in FP64)."""
        sch = Schedule(chunk_rows, block_group, waves, xcd_remap, per_contribution, col_tile, global_atomics, gather)
        check(self._lib.sketch_set_schedule(self._h, ctypes.byref(sch)), "sketch_set_schedule")

    def clear_schedule(self):
        check(self._lib.sketch_set_schedule(self._h, None), "sketch_set_schedule")

    def plan(self, a_dtype, rows, n):
        sch = Schedule()
        check(self._lib.sketch_plan(self._h, int(a_dtype), int(rows), int(n), ctypes.byref(sch)), "sketch_plan")
        return sch.as_dict()

    def hash(self, row_begin, count, stream=None):
        """Device (buckets int32 [count, s], signs int8 [count, s])."""
        torch = _torch()
        b = torch.empty((count, self.s), dtype=torch.int32, device="cuda")
        g = torch.empty((count, self.s), dtype=torch.int8, device="cuda")
        check(self._lib.sketch_hash(self._h, int(row_begin), int(count), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(g.data_ptr()), _stream(stream)), "sketch_hash")
        return b, g


def _problems(specs):
    """specs: dicts with m (optional: A.shape[0]), d, s, seed, rounding, A, SA, epoch."""
    arr = (Problem * len(specs))()
    for i, sp in enumerate(specs):
        A, SA = sp["A"], sp["SA"]
        m, n = A.shape
        arr[i] = Problem(m, n, int(sp["d"]), int(sp["s"]), int(sp.get("rounding", ACC_F16_RN)),
                         int(sp.get("seed", 0)) & (2 ** 64 - 1), A.data_ptr(), _matrix(A, "A"), SA.data_ptr(),
                         _matrix(SA, "SA"), _dtype_code(A), int(sp.get("epoch", 0)) & 0xFFFFFFFF)
    return arr


class Batch:
    """Many independent sketches run by one persistent launch (optionally a
    replayed HIP graph).  The tensors in `specs` must outlive the batch."""

    def __init__(self, specs, chunk_rows=0, block_group=0, waves=0):
        self._lib = load()
        self._specs = list(specs)
        arr = _problems(self._specs)
        sch = Schedule(chunk_rows, block_group, waves, 0)
        use = ctypes.byref(sch) if (chunk_rows or block_group or waves) else None
        h = ctypes.c_void_p()
        check(self._lib.sketch_batch_create(arr, len(arr), use, ctypes.byref(h)), "sketch_batch_create")
        self._h = h

    def apply(self, stream=None):
        check(self._lib.sketch_batch_apply(self._h, _stream(stream)), "sketch_batch_apply")

    def graph(self, stream=None):
        check(self._lib.sketch_batch_graph(self._h, _stream(stream)), "sketch_batch_graph")

    def schedule(self):
        sch = Schedule()
        check(self._lib.sketch_batch_schedule(self._h, ctypes.byref(sch)), "sketch_batch_schedule")
        return sch.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sketch_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_batch(specs, cache_path=None):
    arr = _problems(specs)
    sch = Schedule()
    check(load().sketch_tune_batch(arr, len(arr), cache_path.encode() if cache_path else None, ctypes.byref(sch)),
          "sketch_tune_batch")
    return sch.as_dict()


def load_tuning(path):
    rc = load().sketch_load_tuning(str(path).encode())
    if rc < 0:
        check(rc, "sketch_load_tuning")
    return rc


def clear_tuning():
    check(load().sketch_clear_tuning(), "sketch_clear_tuning")


class Server:
    """Continuous-batching least-squares server (sk_server_* in the C ABI)."""

    def __init__(self, budget_bytes, slots=4):
        self._lib = load()
        h = ctypes.c_void_p()
        check(self._lib.sk_server_create(int(budget_bytes), int(slots), ctypes.byref(h)), "sk_server_create")
        self._h = h
        self._keep = {}

    @staticmethod
    def request(m, n, d, s=4, seed=0, rounding=ACC_F16_RN, A=None, b=None, x=None, a_dtype=None, gen=0,
                gen_seed=0, tol=0.0, inner_tol=0.0, max_refine=0, max_inner=0, epoch=0):
        """A Request; A/b are device tensors (gen = 0) or None (generated)."""
        torch = _torch()
        if a_dtype is None:
            a_dtype = _dtype_code(A) if A is not None else F16
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device="cuda")
        r = Request(int(m), int(n), int(d), int(s), int(rounding), int(seed) & (2 ** 64 - 1), int(a_dtype),
                    int(gen), A.data_ptr() if A is not None else None, _matrix(A, "A") if A is not None else 0,
                    b.data_ptr() if b is not None else None, x.data_ptr(), int(gen_seed) & (2 ** 64 - 1),
                    SolveOpts(float(tol), float(inner_tol), int(max_refine), int(max_inner),
                              int(epoch) & 0xFFFFFFFF))
        return r, (A, b, x)

    def submit(self, req, keep=()):
        t = ctypes.c_uint64()
        check(self._lib.sk_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "sk_server_submit")
        self._keep[t.value] = keep           # tensors stay alive until the result is collected
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32()
        res = Result()
        check(self._lib.sk_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(res)),
              "sk_server_poll")
        if not done.value:
            return None
        self._keep.pop(int(ticket), None)
        return res.as_dict()

    def wait(self, ticket):
        res = Result()
        check(self._lib.sk_server_wait(self._h, int(ticket), ctypes.byref(res)), "sk_server_wait")
        self._keep.pop(int(ticket), None)
        return res.as_dict()

    def stats(self):
        info = ServerInfo()
        check(self._lib.sk_server_stats(self._h, ctypes.byref(info)), "sk_server_stats")
        return info.as_dict()

    def clock(self):
        return self._lib.sk_server_clock(self._h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sk_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(req):
    n = ctypes.c_size_t()
    check(load().sk_server_footprint(ctypes.byref(req), ctypes.byref(n)), "sk_server_footprint")
    return n.value


def simulate_admission(budget, slots, arrive, footprints, service):
    """Host-only replay of the server's admission policy: (admit, done) times."""
    import numpy as np
    k = len(arrive)
    arrive = np.ascontiguousarray(arrive, dtype=np.float64)
    fp = np.ascontiguousarray(footprints, dtype=np.uint64)
    sv = np.ascontiguousarray(service, dtype=np.float64)
    admit = np.zeros(k)
    done = np.zeros(k)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)   # noqa: E731
    check(load().sk_server_simulate(int(budget), int(slots), k, ptr(arrive), ptr(fp), ptr(sv), ptr(admit),
                                    ptr(done)), "sk_server_simulate")
    return admit, done


def qr_f32(M, k, stream=None):
    """In-place FP32 Householder QR of the first k columns of M (device FP32,
    unit column stride); returns tau (k floats)."""
    torch = _torch()
    ldm = _matrix(M, "M")
    if M.dtype != torch.float32:
        raise ValueError("M must be FP32")
    tau = torch.empty(max(int(k), 1), dtype=torch.float32, device=M.device)
    check(load().sketch_qr_f32(ctypes.c_void_p(M.data_ptr()), M.shape[0], M.shape[1], ldm, int(k),
                               ctypes.c_void_p(tau.data_ptr()), _stream(stream)), "sketch_qr_f32")
    return tau[:k]


def trinv_f32(R, stream=None):
    """(P, P^T, bad) with P = R^-1 for the upper triangle of a square FP32 device matrix R."""
    torch = _torch()
    ldr = _matrix(R, "R")
    n = R.shape[0]
    if R.dtype != torch.float32 or R.shape[1] < n:
        raise ValueError("R must be FP32 with at least n columns")
    P = torch.empty((n, n), dtype=torch.float32, device=R.device)
    PT = torch.empty((n, n), dtype=torch.float32, device=R.device)
    bad = torch.zeros(1, dtype=torch.int32, device=R.device)
    check(load().sketch_trinv_f32(ctypes.c_void_p(R.data_ptr()), n, ldr, ctypes.c_void_p(P.data_ptr()),
                                  ctypes.c_void_p(PT.data_ptr()), n, ctypes.c_void_p(bad.data_ptr()),
                                  _stream(stream)), "sketch_trinv_f32")
    return P, PT, bad


def quantize(mode, x, seed=0, epoch=0, site0=0, stream=None):
    """16-bit patterns (int16 tensor) of x (FP32 device tensor) under rule
    `mode`: FP16 for ACC_F16_*, BF16 for ACC_BF16_*."""
    torch = _torch()
    if x.dtype != torch.float32 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x must be a contiguous FP32 device tensor")
    out = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    check(load().sketch_quantize(int(mode), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 x.numel(), int(seed) & (2 ** 64 - 1), int(epoch) & 0xFFFFFFFF, int(site0),
                                 _stream(stream)), "sketch_quantize")
    return out
