"""ctypes loading of libsketch.so and the raw C-ABI signatures.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsketch.so.  Importing this module fails loudly when the library
has not been built (``python -m paper_2606_20195_amd.build``); there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsketch.so")

# return codes (include/sketch.h)
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENOTCONV, EADMIT, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
F32, F16, BF16 = 0, 1, 2
ACC_F32, ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER = 0, 1, 2, 3
ACC_BF16_RN, ACC_BF16_SR, ACC_BF16_DITHER = 4, 5, 6
ACCUMULATE = 1

EXPORTS = ("sketch_create", "sketch_destroy", "sketch_apply", "sketch_set_schedule", "sketch_plan",
           "sketch_hash", "sketch_quantize", "sketch_solve", "sketch_qr_f32", "sketch_trinv_f32",
           "sketch_batch_create", "sketch_batch_apply", "sketch_batch_graph", "sketch_batch_schedule",
           "sketch_batch_destroy", "sketch_apply_batched", "sketch_tune_batch", "sketch_tune_apply",
           "sketch_load_tuning", "sketch_clear_tuning", "sk_server_create", "sk_server_footprint",
           "sk_server_submit", "sk_server_poll", "sk_server_wait", "sk_server_stats", "sk_server_clock",
           "sk_server_destroy", "sk_server_simulate", "sketch_last_error", "sketch_version", "sketch_sync",
           "sketch_apply_noalloc", "sketch_stream_read")


class Schedule(ctypes.Structure):
    _fields_ = [("chunk_rows", ctypes.c_int32), ("block_group", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("per_contribution", ctypes.c_int32), ("col_tile", ctypes.c_int32),
                ("global_atomics", ctypes.c_int32), ("gather", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]

    def as_dict(self):
        return dict(chunk_rows=self.chunk_rows, block_group=self.block_group, waves=self.waves,
                    xcd_remap=self.xcd_remap, per_contribution=self.per_contribution, col_tile=self.col_tile,
                    global_atomics=self.global_atomics, gather=self.gather)


class Problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("s", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("seed", ctypes.c_uint64), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("SA", ctypes.c_void_p), ("ldsa", ctypes.c_int64),
                ("a_dtype", ctypes.c_int32), ("round_epoch", ctypes.c_uint32), ("reserved", ctypes.c_int32 * 4)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("round_epoch", ctypes.c_uint32), ("reserved", ctypes.c_int32 * 3)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("inner_iters", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("crit", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("rel_residual_x0", ctypes.c_double), ("ms_sketch", ctypes.c_double),
                ("ms_factor", ctypes.c_double), ("ms_refine", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("reserved", ctypes.c_double * 4)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class Request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("s", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("seed", ctypes.c_uint64), ("a_dtype", ctypes.c_int32),
                ("gen", ctypes.c_int32), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("gen_seed", ctypes.c_uint64), ("opts", SolveOpts),
                ("reserved", ctypes.c_int32 * 4)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("ms_ingest", ctypes.c_double),
                ("info", SolveInfo)]

    def as_dict(self):
        d = dict(status=self.status, t_submit=self.t_submit, t_admit=self.t_admit, t_done=self.t_done,
                 ms_ingest=self.ms_ingest)
        d.update(self.info.as_dict())
        return d


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64), ("bytes_high_water", ctypes.c_int64),
                ("budget", ctypes.c_int64), ("slots", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class SketchError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsketch.so is not built; run python -m paper_2606_20195_amd.build "
                          "(expected at %s)" % LIB_PATH)
    # The library binds to the HIP runtime already in the process.  PyTorch
    # ships its own copy of that runtime; loading torch first makes both use
    # the same one (loaded the other way round, torch would find no device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "sketch_create": ([i64, i64, i32, u64, i32, ctypes.POINTER(P)], ctypes.c_int),
        "sketch_destroy": ([P], ctypes.c_int),
        "sketch_apply": ([P, P, i32, i64, i64, i64, i64, P, i64, u32, u32, P], ctypes.c_int),
        "sketch_apply_noalloc": ([P, P, i32, i64, i64, i64, i64, P, i64, u32, u32, P], ctypes.c_int),
        "sketch_set_schedule": ([P, ctypes.POINTER(Schedule)], ctypes.c_int),
        "sketch_plan": ([P, i32, i64, i64, ctypes.POINTER(Schedule)], ctypes.c_int),
        "sketch_hash": ([P, i64, i64, P, P, P], ctypes.c_int),
        "sketch_quantize": ([i32, P, P, i64, u64, u32, u64, P], ctypes.c_int),
        "sketch_solve": ([P, P, i32, i64, i64, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), P],
                         ctypes.c_int),
        "sketch_qr_f32": ([P, i64, i64, i64, i64, P, P], ctypes.c_int),
        "sketch_trinv_f32": ([P, i64, i64, P, P, i64, P, P], ctypes.c_int),
        "sketch_batch_create": ([ctypes.POINTER(Problem), i32, ctypes.POINTER(Schedule), ctypes.POINTER(P)],
                                ctypes.c_int),
        "sketch_batch_apply": ([P, P], ctypes.c_int),
        "sketch_batch_graph": ([P, P], ctypes.c_int),
        "sketch_batch_schedule": ([P, ctypes.POINTER(Schedule)], ctypes.c_int),
        "sketch_batch_destroy": ([P], ctypes.c_int),
        "sketch_apply_batched": ([ctypes.POINTER(Problem), i32, ctypes.POINTER(Schedule), P], ctypes.c_int),
        "sketch_tune_batch": ([ctypes.POINTER(Problem), i32, ctypes.c_char_p, ctypes.POINTER(Schedule)],
                              ctypes.c_int),
        "sketch_tune_apply": ([P, P, i32, i64, i64, i64, P, i64, ctypes.c_char_p, ctypes.POINTER(Schedule), P],
                              ctypes.c_int),
        "sketch_load_tuning": ([ctypes.c_char_p], ctypes.c_int),
        "sketch_clear_tuning": ([], ctypes.c_int),
        "sk_server_create": ([ctypes.c_size_t, i32, ctypes.POINTER(P)], ctypes.c_int),
        "sk_server_footprint": ([ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "sk_server_submit": ([P, ctypes.POINTER(Request), ctypes.POINTER(u64)], ctypes.c_int),
        "sk_server_poll": ([P, u64, ctypes.POINTER(i32), ctypes.POINTER(Result)], ctypes.c_int),
        "sk_server_wait": ([P, u64, ctypes.POINTER(Result)], ctypes.c_int),
        "sk_server_stats": ([P, ctypes.POINTER(ServerInfo)], ctypes.c_int),
        "sk_server_clock": ([P], ctypes.c_double),
        "sk_server_destroy": ([P], ctypes.c_int),
        "sk_server_simulate": ([ctypes.c_size_t, i32, i32, P, P, P, P, P], ctypes.c_int),
        "sketch_last_error": ([], ctypes.c_char_p),
        "sketch_version": ([], ctypes.c_int),
        "sketch_sync": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
        "sketch_stream_read": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(rc, where):
    if rc != OK:
        msg = load().sketch_last_error().decode(errors="replace")
        raise SketchError(rc, where, msg)
    return rc
