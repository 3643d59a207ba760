// C ABI of libsketch.so: argument checks, planning and launches.
// The argument checks run before any HIP call so that invalid calls fail the
// same way with or without a GPU.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "sk_internal.hpp"

#define SK_LIB_VERSION 1
#define SK_HASH_VERSION 1

namespace sk {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

static int hip_fail(hipError_t e, const char* what)
{
    return set_error(SK_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int device_info(DeviceInfo* out)
{
    static std::mutex mu;
    static DeviceInfo cache[64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return set_error(SK_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (cache[dev].device != dev) {
        int cus = 0, lds = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CU count)");
        e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(LDS size)");
        cache[dev].device = dev;
        cache[dev].cus = cus > 0 ? cus : 1;
        cache[dev].lds_max = (size_t)lds;
    }
    *out = cache[dev];
    return SK_OK;
}

static int elem_size(int32_t dt)
{
    return dt == SK_F32 ? 4 : (dt == SK_F16 || dt == SK_BF16) ? 2 : 0;
}


int make_plan(const sk_sketch* h, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda, const DeviceInfo& dev,
              Plan* out)
{
    if (!h->forced) {
        // a tuned schedule for this signature, if one is known and valid here
        sk_sketch tuned = *h;
        if (tuning_lookup(apply_key(h, a_dtype, rows, n), &tuned.sched)) {
            tuned.forced = true;
            Plan pl;
            if (make_plan(&tuned, a_dtype, rows, n, lda, dev, &pl) == SK_OK) {
                *out = pl;
                return SK_OK;
            }
            set_error(SK_OK, "");
        }
    }
    const int64_t W = h->d / h->s;
    const sk_schedule* f = h->forced ? &h->sched : nullptr;
    if (f && f->per_contribution) {
        Plan pl;
        pl.direct = true;
        *out = pl;
        return SK_OK;
    }
    if (f && f->global_atomics) {
        Plan g;
        g.global = true;
        *out = g;
        return SK_OK;
    }
    if (f && f->gather) {
        if (!gather_fits(h->d, n, rows, h->s))
            return set_error(SK_EUNSUPPORTED, "the gather's 32-bit lists do not hold %lld rows x s = %d",
                             (long long)rows, h->s);
        Plan g;
        g.global = true;
        g.gather = true;
        *out = g;
        return SK_OK;
    }
    const int64_t row_bytes = n * (int64_t)elem_size(a_dtype);
    const bool gather_ok = gather_fits(h->d, n, rows, h->s);
    // FP32 partials (two fields per element) for FP32 and BF16 output
    const bool dual = h->rounding == SK_ACC_F32 || h->rounding >= SK_ACC_BF16_RN;
    Plan pl;
    // Column tile and blocks per workgroup: the widest tile with the most
    // blocks that fits in LDS (8-column tiles first when n <= 16, where a
    // 32-column tile would leave half its lanes idle), then narrower tiles
    // for larger d/s.
    const int32_t want_nt = (f && f->col_tile) ? f->col_tile : 0;
    const int32_t want_bg = (f && f->block_group) ? f->block_group : 0;
    if (want_bg && h->s % want_bg) return set_error(SK_EINVAL, "block_group %d does not divide s = %d", want_bg, h->s);
    const int32_t order_wide[] = {32, 8, 4, 2}, order_narrow[] = {8, 32, 4, 2};
    const int32_t* order = (n <= 16) ? order_narrow : order_wide;
    for (int i = 0; i < 4 && !pl.bg; ++i) {
        const int32_t nt = order[i];
        if (want_nt && nt != want_nt) continue;
        for (int bg : {8, 4, 2, 1}) {
            if (want_bg && bg != want_bg) continue;
            if (h->s % bg || !apply_tile_ok(nt, bg)) continue;
            if (apply_lds_bytes(bg, W, dual, nt) <= dev.lds_max) {
                pl.bg = bg;
                pl.nt = nt;
                break;
            }
        }
    }
    if (!pl.bg) {
        if (want_nt || want_bg)
            return set_error(SK_EUNSUPPORTED, "no kernel for col_tile %d, block_group %d fits %lld bucket rows in LDS",
                             want_nt, want_bg, (long long)W);
        // No block fits in LDS: the whole call goes to the FP32 workspace,
        // by the bucket-sorted gather for rows of 64 bytes or more, else by
        // FP32 atomics (narrow rows make the gather's list traffic and its
        // 4-byte reads cost more than one atomic per contribution).
        Plan g;
        g.global = true;
        g.gather = !f && gather_ok && row_bytes >= 64;
        *out = g;
        return SK_OK;
    }
    // With rows of 256 bytes or more, reading each row s times by bucket
    // costs less than a tile narrower than the width calls for (d/s too large
    // for it in LDS), which hashes every row once per column tile, and than
    // one-block FP32 partials (two fields per element, s passes over A).
    // Table 1 sizes, 2^21 x 1024 FP32: d/n = 8 and 16 with 8- and 2-column
    // tiles 19 and 37 ms, gather 6.3 and 6.5 ms; FP32 mode at d/n = 2 with
    // one-block 32-column tiles 7.6 ms, gather 6.4 ms.  FP16 partials with
    // one block keep the tiles (d/n = 4: 3.9 against 6.2 ms): a unit's s
    // passes run together and share its rows through the caches.
    if (!f && gather_ok && row_bytes >= 256 &&
        (pl.nt < ((n <= 16) ? 8 : 32) || (dual && pl.bg == 1 && h->s > 1))) {
        Plan g;
        g.global = true;
        g.gather = true;
        *out = g;
        return SK_OK;
    }
    pl.lds_bytes = apply_lds_bytes(pl.bg, W, dual, pl.nt);
    pl.bgroups = h->s / pl.bg;
    pl.col_tiles = (int32_t)((n + pl.nt - 1) / pl.nt);
    const int maxw = apply_max_waves(a_dtype, pl.bg);
    // the most waves the element type allows (16 for 16-bit A, 8 for FP32 A)
    // measured fastest for 32-column tiles: more waves keep more LDS atomics
    // in flight.  Narrow matrices (n <= 16, 8-column tiles) take 8: their
    // items are short, and two workgroups a CU overlap one's clearing,
    // sample and flush with the other's stream (n = 16: 0.044 against
    // 0.072 ms at 2^21 rows)
    const int autow = (pl.nt == 8 && n <= 16) ? std::min(maxw, 8) : maxw;
    pl.waves = (f && f->waves) ? f->waves : autow;
    // odd n or lda take the scalar-load kernels, built for at most 8 waves
    if (((n | lda) & 1) && pl.waves > 8) pl.waves = 8;
    if (pl.waves > maxw) return set_error(SK_EINVAL, "waves = %d exceeds %d for this element type", pl.waves, maxw);
    const int64_t per_unit = (int64_t)pl.col_tiles * pl.bgroups;
    const int esz = elem_size(a_dtype);
    // A unit is addressed through one buffer resource: keep it below 2 GiB.
    const int64_t max_chunk = ((((int64_t)1 << 31) - 1) / (lda * esz)) / 64 * 64;
    if (max_chunk < 64) return set_error(SK_EUNSUPPORTED, "64 rows of lda = %lld exceed 2 GiB", (long long)lda);
    if (f && f->chunk_rows) {
        pl.chunk_rows = f->chunk_rows;
        if (pl.chunk_rows > max_chunk)
            return set_error(SK_EUNSUPPORTED, "chunk_rows = %d spans more than 2 GiB", pl.chunk_rows);
    } else {
        // One round of work items fills the GPU: a CU holds as many workgroups
        // as fit both its LDS and its wave slots (maxw waves at the kernels'
        // register budget).  More, smaller units only add fixed per-item
        // work (clearing, the exponent sample, decoding and the flush): with
        // 16-wave workgroups, 2048-row units at n = 32 measured 1.7x slower
        // than units four to eight times larger.
        const int64_t wg_lds = std::max<int64_t>(1, (int64_t)(dev.lds_max / pl.lds_bytes));
        const int64_t wg_per_cu = std::max<int64_t>(1, std::min<int64_t>(wg_lds, maxw / pl.waves));
        const int64_t target = std::max<int64_t>(1, (int64_t)dev.cus * wg_per_cu / per_unit);
        int64_t chunk = (rows + target - 1) / target;
        chunk = (chunk + 63) / 64 * 64;
        chunk = std::max<int64_t>(chunk, 2048);
        chunk = std::min<int64_t>(chunk, max_chunk);
        pl.chunk_rows = (int32_t)chunk;
    }
    pl.units = rows > 0 ? (rows + pl.chunk_rows - 1) / pl.chunk_rows : 0;
    if (pl.units * per_unit > 0x7FFFFFFF) return set_error(SK_EUNSUPPORTED, "grid too large");
    const int want_remap = f ? f->xcd_remap : 1;
    pl.xcd_remap = (want_remap && per_unit > 1 && pl.units % 8 == 0) ? 1 : 0;
    *out = pl;
    return SK_OK;
}

static int check_schedule(const sk_schedule* s)
{
    if (s->chunk_rows < 0 || s->chunk_rows % 64)
        return set_error(SK_EINVAL, "chunk_rows must be a non-negative multiple of 64");
    if (s->block_group && s->block_group != 1 && s->block_group != 2 && s->block_group != 4 && s->block_group != 8)
        return set_error(SK_EINVAL, "block_group must be 0, 1, 2, 4 or 8");
    if (s->waves && s->waves != 4 && s->waves != 8 && s->waves != 16)
        return set_error(SK_EINVAL, "waves must be 0, 4, 8 or 16");
    if (s->xcd_remap != 0 && s->xcd_remap != 1) return set_error(SK_EINVAL, "xcd_remap must be 0 or 1");
    if (s->per_contribution != 0 && s->per_contribution != 1)
        return set_error(SK_EINVAL, "per_contribution must be 0 or 1");
    if (s->col_tile && s->col_tile != 32 && s->col_tile != 8 && s->col_tile != 4 && s->col_tile != 2)
        return set_error(SK_EINVAL, "col_tile must be 0, 32, 8, 4 or 2");
    if (s->col_tile && s->block_group && !apply_tile_ok(s->col_tile, s->block_group))
        return set_error(SK_EINVAL, "no kernel for col_tile %d with block_group %d", s->col_tile, s->block_group);
    if (s->global_atomics != 0 && s->global_atomics != 1) return set_error(SK_EINVAL, "global_atomics must be 0 or 1");
    if (s->global_atomics && s->per_contribution)
        return set_error(SK_EINVAL, "global_atomics and per_contribution exclude each other");
    if (s->gather != 0 && s->gather != 1) return set_error(SK_EINVAL, "gather must be 0 or 1");
    if (s->gather && (s->global_atomics || s->per_contribution))
        return set_error(SK_EINVAL, "gather excludes global_atomics and per_contribution");
    if (s->reserved[0]) return set_error(SK_EINVAL, "reserved schedule fields must be zero");
    return SK_OK;
}

// Workspace of sketch_apply_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code uses the device address from
// hipGetSymbolAddress, taken once per device with that device current (the
// array's name is only a host-side stand-in).  Every call on a GPU shares its
// copy, so calls that overlap on one GPU race.
constexpr size_t kNoallocFloats = (size_t)1 << 22;    // 16 MiB: d * n <= 4194304
static __device__ __align__(256) float scratch[kNoallocFloats];

static int scratch_address(float** out)
{
    static std::mutex mu;
    static float* addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return set_error(SK_EUNSUPPORTED, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        addr[dev] = (float*)p;
    }
    *out = addr[dev];
    return SK_OK;
}

static float value_scale32(int32_t s) { return (float)(1.0 / std::sqrt((double)s)); }
static bool scale_is_pow2(int32_t s) { return s == 1 || s == 4 || s == 16; }

}  // namespace sk

using namespace sk;

extern "C" {

int sketch_version(void) { return SK_LIB_VERSION * 100 + SK_HASH_VERSION; }

const char* sketch_last_error(void) { return g_err; }

int sketch_stream_read(const void* p, int64_t bytes, uint32_t* out, void* stream)
{
    if (!p || !out) return set_error(SK_EINVAL, "NULL argument");
    if (bytes < 16 || bytes % 16 || ((uintptr_t)p & 15u))
        return set_error(SK_EINVAL, "bytes must be a positive multiple of 16 and p 16-byte aligned");
    (void)hipGetLastError();
    const hipError_t e = launch_stream_read(p, bytes, out, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_fail(e, "stream read kernel");
}

int sketch_sync(sk_handle, void* stream)
{
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "asynchronous failure on the stream");
    return SK_OK;
}

int sketch_create(int64_t m, int64_t d, int32_t s, uint64_t seed, int32_t rounding, sk_handle* out)
{
    if (!out) return set_error(SK_EINVAL, "out is NULL");
    *out = nullptr;
    if (m < 1) return set_error(SK_EINVAL, "m = %lld must be >= 1", (long long)m);
    if (s < 1 || s > 16) return set_error(SK_EINVAL, "s = %d must be in 1..16", s);
    if (d < 1 || d % s) return set_error(SK_EINVAL, "d = %lld must be >= 1 and a multiple of s = %d", (long long)d, s);
    if (d / s > (1LL << 24)) return set_error(SK_EUNSUPPORTED, "d/s = %lld too large", (long long)(d / s));
    if (rounding < SK_ACC_F32 || rounding > SK_ACC_BF16_DITHER)
        return set_error(SK_EINVAL, "unknown rounding code %d", rounding);
    sk_sketch* h = new (std::nothrow) sk_sketch;
    if (!h) return set_error(SK_ENOMEM, "out of host memory");
    h->m = m;
    h->d = d;
    h->s = s;
    h->seed = seed;
    h->rounding = rounding;
    *out = h;
    return SK_OK;
}

int sketch_destroy(sk_handle h)
{
    if (!h) return SK_OK;
    if (h->ws && !h->ws_borrowed) (void)hipFree(h->ws);
    solve_release(h);
    delete h;
    return SK_OK;
}

int sketch_set_schedule(sk_handle h, const sk_schedule* sched)
{
    if (!h) return set_error(SK_EINVAL, "handle is NULL");
    if (!sched) {
        h->forced = false;
        return SK_OK;
    }
    int rc = check_schedule(sched);
    if (rc) return rc;
    h->sched = *sched;
    h->forced = true;
    return SK_OK;
}

int sketch_plan(sk_handle h, int32_t a_dtype, int64_t rows, int64_t n, sk_schedule* out)
{
    if (!h || !out) return set_error(SK_EINVAL, "NULL argument");
    if (!elem_size(a_dtype)) return set_error(SK_EINVAL, "unknown element type %d", a_dtype);
    if (rows < 0 || n < 1) return set_error(SK_EINVAL, "bad shape");
    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc) return rc;
    Plan pl;
    rc = make_plan(h, a_dtype, rows, n, n, dev, &pl);
    if (rc) return rc;
    std::memset(out, 0, sizeof(*out));
    out->chunk_rows = pl.chunk_rows;
    out->block_group = pl.bg;
    out->waves = pl.waves;
    out->xcd_remap = pl.xcd_remap;
    out->per_contribution = pl.direct ? 1 : 0;
    out->col_tile = pl.bg ? pl.nt : 0;
    out->global_atomics = (pl.global && !pl.gather) ? 1 : 0;
    out->gather = pl.gather ? 1 : 0;
    return SK_OK;
}

// sketch_apply with the d x n FP32 workspace (large d/s, BF16 output, FP32
// accumulation with a non-power-of-two scale) either held by the handle
// (ext_ws == nullptr: allocated on first need) or given by the caller.
static int apply_impl(sk_handle h, const void* A, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda,
                      int64_t row_offset, void* SA, int64_t ldsa, uint32_t flags, uint32_t round_epoch,
                      void* stream, float* ext_ws, size_t ext_floats)
{
    if (!h) return set_error(SK_EINVAL, "handle is NULL");
    const int esz = elem_size(a_dtype);
    if (!esz) return set_error(SK_EINVAL, "unknown element type %d", a_dtype);
    if (rows < 0 || n < 1 || n > (1LL << 30)) return set_error(SK_EINVAL, "bad shape rows=%lld n=%lld",
                                                               (long long)rows, (long long)n);
    if (lda < n) return set_error(SK_EINVAL, "lda = %lld < n = %lld", (long long)lda, (long long)n);
    if (row_offset < 0 || row_offset + rows > h->m)
        return set_error(SK_EINVAL, "rows [%lld, %lld) outside the sketch's m = %lld", (long long)row_offset,
                         (long long)(row_offset + rows), (long long)h->m);
    if (!SA) return set_error(SK_EINVAL, "SA is NULL");
    if (ldsa < n) return set_error(SK_EINVAL, "ldsa = %lld < n = %lld", (long long)ldsa, (long long)n);
    if (rows > 0 && !A) return set_error(SK_EINVAL, "A is NULL");
    if (flags & ~SK_ACCUMULATE) return set_error(SK_EINVAL, "unknown flags 0x%x", flags);
    const bool bf16 = h->rounding >= SK_ACC_BF16_RN;
    const bool f16 = h->rounding != SK_ACC_F32 && !bf16;
    if (f16 && (((uintptr_t)SA & 3u) || (ldsa & 1)))
        return set_error(SK_EUNSUPPORTED, "FP16 SA needs a 4-byte aligned base and an even ldsa");
    if (bf16 && ((uintptr_t)SA & 1u)) return set_error(SK_EINVAL, "BF16 SA is not 2-byte aligned");
    if (!f16 && !bf16 && ((uintptr_t)SA & 3u)) return set_error(SK_EINVAL, "FP32 SA is not 4-byte aligned");
    if (rows > 0 && ((uintptr_t)A % (uintptr_t)esz)) return set_error(SK_EINVAL, "A is not element aligned");
    const bool accumulate = (flags & SK_ACCUMULATE) != 0;

    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc) return rc;
    Plan pl;
    if (rows > 0) {
        rc = make_plan(h, a_dtype, rows, n, lda, dev, &pl);
        if (rc) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    (void)hipGetLastError();            // launch checks below report this call's errors only

    ApplyArgs a{};
    a.A = A;
    a.lda = lda;
    a.rows = rows;
    a.row_offset = row_offset;
    a.n = (int32_t)n;
    a.d = (int32_t)h->d;
    a.s = h->s;
    a.W = (uint32_t)(h->d / h->s);
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    a.chunk_rows = pl.chunk_rows;
    a.col_tiles = pl.col_tiles;
    a.bgroups = pl.bgroups;
    a.nt = pl.nt;
    a.epoch = round_epoch;
    a.xcd_remap = pl.xcd_remap;
    const uintptr_t vec_align = esz == 4 ? 8u : 4u;
    a.aligned = (n % 2 == 0) && (lda % 2 == 0) && ((uintptr_t)A % vec_align == 0);
    // a base address off the vector alignment also takes the scalar-load kernels
    if (!a.aligned && pl.waves > 8) pl.waves = 8;
    const float cs = value_scale32(h->s);

    // The bucket-sorted gather's lists may not fit a caller's scratch: then
    // the planner's choice falls back to FP32 atomics into the d x n sum.
    const size_t sum_floats = (size_t)h->d * (size_t)n;
    if (pl.gather && ext_ws && plan_ws_floats(pl, h->d, n, rows, h->s) > ext_floats) {
        if (h->forced && h->sched.gather)
            return set_error(SK_EINVAL, "the gather's workspace of %zu floats exceeds the %zu-float scratch",
                             plan_ws_floats(pl, h->d, n, rows, h->s), ext_floats);
        pl.gather = false;
    }
    const size_t ws_need = pl.gather ? plan_ws_floats(pl, h->d, n, rows, h->s) : sum_floats;

    // d x n FP32 workspace held by the handle (allocated on first need)
    float* ws = nullptr;
    auto ensure_ws = [&](size_t need) -> int {
        if (ext_ws) {
            if (need > ext_floats)
                return set_error(SK_EINVAL, "the d x n workspace of %zu floats exceeds the %zu-float scratch", need,
                                 ext_floats);
            ws = ext_ws;
            return SK_OK;
        }
        if (h->ws_floats < need) {
            if (h->ws_borrowed)
                return set_error(SK_EINVAL, "borrowed workspace of %zu floats is smaller than %zu", h->ws_floats,
                                 need);
            if (h->ws) (void)hipFree(h->ws);
            h->ws = nullptr;
            h->ws_floats = 0;
            if ((e = hipMalloc((void**)&h->ws, need * sizeof(float))) != hipSuccess)
                return set_error(SK_ENOMEM, "workspace of %zu floats: %s", need, hipGetErrorString(e));
            h->ws_floats = need;
        }
        ws = h->ws;
        return SK_OK;
    };
    // ws = the unscaled FP32 sum of the call: by the gather, else cleared and
    // filled by FP32 atomics (global) or the LDS partials' FP32 flush
    auto sum_into_ws = [&]() -> hipError_t {
        a.SA = ws;
        a.ldsa = n;
        a.mode = 0;
        a.scale = 1.0f;
        if (pl.gather)   // counters, offsets and lists follow the sum
            return launch_gather(a_dtype, a, ws, (uint32_t*)(ws + (sum_floats + 63) / 64 * 64), st);
        hipError_t e2 = launch_fill(ws, 4, h->d, n, n, st);
        if (e2 != hipSuccess) return e2;
        return pl.global ? launch_contrib(a_dtype, a, st) : launch_apply(a_dtype, pl, a, st);
    };
    if (bf16) {
        // FP32 sum of the whole call in the workspace, one BF16 rounding per entry
        if (rows == 0) {
            if (!accumulate && (e = launch_fill(SA, 2, h->d, n, ldsa, st)) != hipSuccess) return hip_fail(e, "fill SA");
            return SK_OK;
        }
        if ((rc = ensure_ws(ws_need))) return rc;
        if ((e = sum_into_ws()) != hipSuccess) return hip_fail(e, "apply kernel");
        e = launch_finish_bf16(ws, h->d, (int32_t)n, (uint16_t*)SA, ldsa, h->rounding, cs,
                               (uint64_t)row_offset * (uint64_t)h->d * (uint64_t)n, round_epoch, a.k0, a.k1,
                               accumulate, st);
        return e == hipSuccess ? SK_OK : hip_fail(e, "finish kernel");
    }
    if (pl.global) {
        // d/s bucket rows beyond LDS: the whole call is one unit, summed
        // unscaled in an FP32 workspace (FP64 sums of the bucket-sorted
        // gather, or FP32 atomics), then finished once.
        if (rows == 0) {
            if (!accumulate && (e = launch_fill(SA, f16 ? 2 : 4, h->d, n, ldsa, st)) != hipSuccess)
                return hip_fail(e, "fill SA");
            return SK_OK;
        }
        if ((rc = ensure_ws(ws_need))) return rc;
        if ((e = sum_into_ws()) != hipSuccess) return hip_fail(e, pl.gather ? "gather kernels" : "workspace kernel");
        if (f16) {
            if (!accumulate && (e = launch_fill(SA, 2, h->d, n, ldsa, st)) != hipSuccess)
                return hip_fail(e, "fill SA");
            e = launch_finish16(ws, h->d, (int32_t)n, (uint16_t*)SA, ldsa, h->rounding, cs,
                                (uint64_t)row_offset * (uint64_t)h->d * (uint64_t)n, round_epoch, a.k0, a.k1, st);
            if (e != hipSuccess) return hip_fail(e, "finish kernel");
        } else if ((e = launch_scale((float*)SA, h->d, n, ldsa, ws, cs, accumulate ? 1 : 0, st)) != hipSuccess) {
            return hip_fail(e, "scale kernel");
        }
        return SK_OK;
    }
    if (pl.direct) {
        // one global atomic per contribution (the paper's kernel scheme)
        if (!accumulate) {
            if ((e = launch_fill(SA, f16 ? 2 : 4, h->d, n, ldsa, st)) != hipSuccess) return hip_fail(e, "fill SA");
        }
        if (rows == 0) return SK_OK;
        a.SA = SA;
        a.ldsa = ldsa;
        a.mode = f16 ? h->rounding : 0;
        a.scale = cs;
        if ((e = launch_contrib(a_dtype, a, st)) != hipSuccess) return hip_fail(e, "per-contribution kernel");
        return SK_OK;
    }
    if (f16) {
        if (!accumulate) {
            if ((e = launch_fill(SA, 2, h->d, n, ldsa, st)) != hipSuccess) return hip_fail(e, "fill SA");
        }
        if (rows == 0) return SK_OK;
        a.SA = SA;
        a.ldsa = ldsa;
        a.mode = h->rounding;
        a.scale = cs;
        if ((e = launch_apply(a_dtype, pl, a, st)) != hipSuccess) return hip_fail(e, "apply kernel");
        return SK_OK;
    }
    a.mode = 0;
    if (scale_is_pow2(h->s) || !accumulate) {
        // FP32 partials go straight into SA; a non-power-of-two scale is applied
        // once to the finished sum so the result has a single final rounding.
        if (!accumulate) {
            if ((e = launch_fill(SA, 4, h->d, n, ldsa, st)) != hipSuccess) return hip_fail(e, "fill SA");
        }
        if (rows == 0) return SK_OK;
        a.SA = SA;
        a.ldsa = ldsa;
        a.scale = scale_is_pow2(h->s) ? cs : 1.0f;
        if ((e = launch_apply(a_dtype, pl, a, st)) != hipSuccess) return hip_fail(e, "apply kernel");
        if (!scale_is_pow2(h->s)) {
            if ((e = launch_scale((float*)SA, h->d, n, ldsa, nullptr, cs, 0, st)) != hipSuccess)
                return hip_fail(e, "scale kernel");
        }
        return SK_OK;
    }
    // Accumulating with a non-power-of-two scale: sum into a workspace, then
    // SA += fl32(c_s * sum).
    if (rows == 0) return SK_OK;
    if ((rc = ensure_ws((size_t)h->d * (size_t)n))) return rc;
    if ((e = launch_fill(ws, 4, h->d, n, n, st)) != hipSuccess) return hip_fail(e, "fill workspace");
    a.SA = ws;
    a.ldsa = n;
    a.scale = 1.0f;
    if ((e = launch_apply(a_dtype, pl, a, st)) != hipSuccess) return hip_fail(e, "apply kernel");
    if ((e = launch_scale((float*)SA, h->d, n, ldsa, ws, cs, 1, st)) != hipSuccess)
        return hip_fail(e, "scale kernel");
    return SK_OK;
}

int sketch_apply(sk_handle h, const void* A, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda,
                 int64_t row_offset, void* SA, int64_t ldsa, uint32_t flags, uint32_t round_epoch, void* stream)
{
    return apply_impl(h, A, a_dtype, rows, n, lda, row_offset, SA, ldsa, flags, round_epoch, stream, nullptr, 0);
}

int sketch_apply_noalloc(sk_handle h, const void* A, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda,
                         int64_t row_offset, void* SA, int64_t ldsa, uint32_t flags, uint32_t round_epoch,
                         void* stream)
{
    float* ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc) return rc;
    return apply_impl(h, A, a_dtype, rows, n, lda, row_offset, SA, ldsa, flags, round_epoch, stream, ws,
                      kNoallocFloats);
}

int sketch_hash(sk_handle h, int64_t row_begin, int64_t count, int32_t* buckets, int8_t* signs, void* stream)
{
    if (!h) return set_error(SK_EINVAL, "handle is NULL");
    if (row_begin < 0 || count < 0 || row_begin + count > h->m)
        return set_error(SK_EINVAL, "rows [%lld, %lld) outside m = %lld", (long long)row_begin,
                         (long long)(row_begin + count), (long long)h->m);
    if (count > 0 && (!buckets || !signs)) return set_error(SK_EINVAL, "NULL output");
    if (count == 0) return SK_OK;
    hipError_t e = launch_hash(h->seed, h->d, h->s, row_begin, count, buckets, signs, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_fail(e, "hash kernel");
}

int sketch_quantize(int32_t mode, const float* x, uint16_t* out, int64_t count, uint64_t seed, uint32_t epoch,
                    uint64_t site0, void* stream)
{
    if (mode < SK_ACC_F16_RN || mode > SK_ACC_BF16_DITHER)
        return set_error(SK_EINVAL, "mode %d is not a 16-bit rounding mode", mode);
    if (count < 0) return set_error(SK_EINVAL, "count < 0");
    if (count > 0 && (!x || !out)) return set_error(SK_EINVAL, "NULL array");
    if (count == 0) return SK_OK;
    hipError_t e = launch_quantize(mode, x, out, count, seed, epoch, site0, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_fail(e, "quantize kernel");
}

}  // extern "C"
