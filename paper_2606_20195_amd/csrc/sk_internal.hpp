// Host-side internals shared by the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <string>

#include "../../include/sketch.h"

namespace sk { struct SolveWs; }

struct sk_sketch {
    int64_t m = 0, d = 0;
    int32_t s = 0;
    uint64_t seed = 0;
    int32_t rounding = 0;
    bool forced = false;
    sk_schedule sched{};
    // FP32 workspace for SK_ACCUMULATE when 1/sqrt(s) is not a power of two
    float *ws = nullptr;
    size_t ws_floats = 0;
    bool ws_borrowed = false;   // ws lies in memory owned elsewhere (a solve job's block)
    // device workspace of sketch_solve (allocated on first use)
    sk::SolveWs *sw = nullptr;
};

namespace sk {

int set_error(int code, const char *fmt, ...);

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    size_t lds_max = 0;
};
int device_info(DeviceInfo *out);

// Resolved launch plan of one apply call.
struct Plan {
    int32_t bg = 0;          // blocks per workgroup
    int32_t bgroups = 0;     // s / bg
    int32_t nt = 32;         // columns per tile: 32, 8, 4 or 2
    int32_t col_tiles = 0;   // ceil(n / nt)
    int32_t waves = 0;
    int32_t chunk_rows = 0;
    int64_t units = 0;
    int32_t xcd_remap = 0;
    size_t lds_bytes = 0;
    bool direct = false;     // one global atomic per contribution
    bool global = false;     // d/s too large for LDS partials: FP32 workspace of the whole call
    bool gather = false;     // the workspace filled by the bucket-sorted gather (implies global)
};

// LDS bytes of one work item: bg blocks of W bucket rows of nt columns.
size_t apply_lds_bytes(int32_t bg, int64_t W, bool dual, int32_t nt);
// Whether kernels exist for this (column tile, block group).
bool apply_tile_ok(int32_t nt, int32_t bg);
int make_plan(const sk_sketch *h, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda, const DeviceInfo &dev,
              Plan *out);
// Most waves per workgroup of the single-call kernels (by element type and
// blocks per workgroup) and of the persistent batched kernel.
int apply_max_waves(int32_t a_dtype, int32_t bg);
int batch_max_waves();

struct ApplyArgs {
    const void *A;
    int64_t lda, rows, row_offset;
    void *SA;
    int64_t ldsa;
    int32_t n, d, s;
    uint32_t W;
    uint32_t k0, k1;
    int32_t chunk_rows, col_tiles, bgroups;
    int32_t nt;          // columns per tile (the batched kernel dispatches on it)
    int32_t mode;        // 0: FP32 atomics, 1 RN, 2 SR, 3 dither
    float scale;         // multiplier of each flushed partial
    uint32_t epoch;
    int32_t xcd_remap;
    int32_t aligned;     // vector loads allowed
};

// One problem of a batched apply.
struct BatchDesc {
    ApplyArgs a;
    int64_t item0;       // first flat work item of this problem
    float post_scale;    // FP32 mode with a non-power-of-two 1/sqrt(s): c_s, else 0
    int32_t pad;
};

hipError_t launch_apply(int a_dtype, const Plan &plan, const ApplyArgs &args, hipStream_t st);
// Per element type (sk_apply_f32.hip, sk_apply_f16.hip, sk_apply_bf16.hip).
hipError_t launch_apply_f32(const Plan &plan, const ApplyArgs &a, hipStream_t st);
hipError_t launch_apply_f16(const Plan &plan, const ApplyArgs &a, hipStream_t st);
hipError_t launch_apply_bf16(const Plan &plan, const ApplyArgs &a, hipStream_t st);
hipError_t batched_f32(int bg, bool vec, bool dual, const BatchDesc *descs, int32_t count, int64_t total_items,
                       uint32_t *counter, int grid, int waves, size_t lds_bytes, hipStream_t st);
hipError_t batched_f16(int bg, bool vec, bool dual, const BatchDesc *descs, int32_t count, int64_t total_items,
                       uint32_t *counter, int grid, int waves, size_t lds_bytes, hipStream_t st);
hipError_t batched_bf16(int bg, bool vec, bool dual, const BatchDesc *descs, int32_t count, int64_t total_items,
                        uint32_t *counter, int grid, int waves, size_t lds_bytes, hipStream_t st);
// One global atomic per contribution (args.mode: 0 FP32 SA, 1..3 FP16 SA).
hipError_t launch_contrib(int a_dtype, const ApplyArgs &args, hipStream_t st);
// Bucket-sorted gather (sk_gather.hip): 32-bit words of its counters, offsets
// and lists beyond the d x n sum; whether a call's shape fits its 32-bit lists
// and its grid.
size_t gather_aux_words(int64_t d, int64_t rows, int32_t s);
bool gather_fits(int64_t d, int64_t n, int64_t rows, int32_t s);
// ws (d x n FP32, ld n) = the unscaled sum of the call; aux holds
// gather_aux_words(d, rows, s) words.
hipError_t launch_gather(int a_dtype, const ApplyArgs &args, float *ws, uint32_t *aux, hipStream_t st);
// FP32 words of the workspace a plan needs: d x n for the workspace paths,
// plus the gather's lists (offset 256-byte aligned), else 0.
size_t plan_ws_floats(const Plan &pl, int64_t d, int64_t n, int64_t rows, int32_t s);

// SA (BF16, ld ldsa) = (or += with one BF16 RN add) the BF16 rounding of fl32(scale * ws).
hipError_t launch_finish_bf16(const float *ws, int64_t d, int32_t n, uint16_t *SA, int64_t ldsa, int32_t mode,
                              float scale, uint64_t site0, uint32_t epoch, uint32_t k0, uint32_t k1, bool accumulate,
                              hipStream_t st);
// SA (FP16, ld ldsa) += rounding of fl32(scale * ws) per entry, sites site0 + b*n + c.
hipError_t launch_finish16(const float *ws, int64_t d, int32_t n, uint16_t *SA, int64_t ldsa, int32_t mode,
                           float scale, uint64_t site0, uint32_t epoch, uint32_t k0, uint32_t k1, hipStream_t st);
// Clear all SAs, one persistent apply over all problems, FP32 epilogue scale if needed.
hipError_t launch_batched(int a_dtype, int bg, bool vec, bool dual, const BatchDesc *descs, int32_t count,
                          int64_t total_items, uint32_t *counter, int grid, int waves, size_t lds_bytes,
                          bool post_scale, int64_t max_dn, hipStream_t st);
hipError_t launch_fill(void *p, int elem_bytes, int64_t rows, int64_t cols, int64_t ld, hipStream_t st);
hipError_t launch_stream_read(const void *p, int64_t bytes, uint32_t *out, hipStream_t st);
hipError_t launch_scale(float *SA, int64_t d, int64_t n, int64_t ldsa, const float *ws, float c,
                        int accumulate, hipStream_t st);
hipError_t launch_hash(uint64_t seed, int64_t d, int32_t s, int64_t row_begin, int64_t count,
                       int32_t *buckets, int8_t *signs, hipStream_t st);
void solve_release(sk_sketch *h);

// A least-squares solve as resumable asynchronous phases (sk_solve.hip).
struct SolveJob;
SolveJob *job_new();
void job_delete(SolveJob *j);
// Validate and plan; *footprint = device bytes needed at the job's base.
int job_prepare(SolveJob *j, const sk_sketch &S, const void *A, int32_t a_dtype, int64_t n, int64_t lda,
                const double *b, double *x, const sk_solve_opts *opts, size_t *footprint);
// Bind to device memory and a stream; enqueue the first phases.
int job_start(SolveJob *j, void *device_base, hipStream_t st);
// 1 while in flight, SK_OK / SK_ENOTCONV when finished, other codes on failure.
int job_step(SolveJob *j, bool block);
void job_info(const SolveJob *j, sk_solve_info *info);

// Tuning table (filled by the autotuners, read by the planners).
std::string apply_key(const sk_sketch *h, int32_t a_dtype, int64_t rows, int64_t n);
bool tuning_lookup(const std::string &key, sk_schedule *out);
// Raise the batched kernel's dynamic-LDS limit without launching.
hipError_t prepare_batched(int a_dtype, int bg, bool vec, bool dual, size_t lds_bytes);

hipError_t launch_quantize(int mode, const float *x, uint16_t *out, int64_t count, uint64_t seed,
                           uint32_t epoch, uint64_t site0, hipStream_t st);

}  // namespace sk
