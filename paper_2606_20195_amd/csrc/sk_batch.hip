// Batches of independent sketches (one persistent launch, optional HIP graph)
// and the schedule autotuner with its process-wide tuning table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sk_internal.hpp"

namespace sk {

namespace {

int hip_err(hipError_t e, const char* what) { return set_error(SK_EHIP, "%s: %s", what, hipGetErrorString(e)); }

int esize(int32_t dt) { return dt == SK_F32 ? 4 : (dt == SK_F16 || dt == SK_BF16) ? 2 : 0; }

bool pow2_scale(int32_t s) { return s == 1 || s == 4 || s == 16; }

// ---------------------------------------------------------------- tuning table

struct TuneEntry {
    sk_schedule sched;
    double ms;
};

std::mutex g_tune_mu;
std::map<std::string, TuneEntry>& table()
{
    static std::map<std::string, TuneEntry> t;
    return t;
}

std::string batch_key(int32_t a_dtype, bool dual, int32_t count, double bytes, int64_t nmax)
{
    char buf[160];
    snprintf(buf, sizeof(buf), "batch a=%d acc=%s k=%d bytes=2^%d nmax=%lld", a_dtype, dual ? "f32" : "f16", count,
             (int)std::lround(std::log2(std::max(bytes, 1.0))), (long long)nmax);
    return buf;
}

// Minimal reader for the files this library writes:
// {"version": 1, "entries": [{"key": "...", "chunk_rows": N, ...}, ...]}
struct JsonCursor {
    const std::string& s;
    size_t i = 0;
    void ws()
    {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c)
    {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    bool str(std::string& out)
    {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        ++i;
        out.clear();
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\' && i + 1 < s.size()) ++i;
            out.push_back(s[i++]);
        }
        if (i >= s.size()) return false;
        ++i;
        return true;
    }
    bool num(double& out)
    {
        ws();
        const char* b = s.c_str() + i;
        char* e = nullptr;
        out = std::strtod(b, &e);
        if (e == b) return false;
        i += (size_t)(e - b);
        return true;
    }
};

int parse_tuning(const std::string& text, std::vector<std::pair<std::string, TuneEntry>>& out)
{
    JsonCursor c{text};
    if (!c.eat('{')) return -1;
    bool have_entries = false;
    while (true) {
        std::string k;
        if (!c.str(k) || !c.eat(':')) return -1;
        if (k == "entries") {
            have_entries = true;
            if (!c.eat('[')) return -1;
            if (!c.eat(']')) {
                do {
                    if (!c.eat('{')) return -1;
                    std::string key;
                    TuneEntry te{};
                    bool has_key = false;
                    do {
                        std::string f;
                        if (!c.str(f) || !c.eat(':')) return -1;
                        if (f == "key") {
                            if (!c.str(key)) return -1;
                            has_key = true;
                        } else {
                            double v;
                            if (!c.num(v)) return -1;
                            if (f == "chunk_rows") te.sched.chunk_rows = (int32_t)v;
                            else if (f == "block_group") te.sched.block_group = (int32_t)v;
                            else if (f == "waves") te.sched.waves = (int32_t)v;
                            else if (f == "xcd_remap") te.sched.xcd_remap = (int32_t)v;
                            else if (f == "col_tile") te.sched.col_tile = (int32_t)v;
                            else if (f == "global_atomics") te.sched.global_atomics = (int32_t)v;
                            else if (f == "gather") te.sched.gather = (int32_t)v;
                            else if (f == "ms") te.ms = v;
                        }
                    } while (c.eat(','));
                    if (!c.eat('}') || !has_key) return -1;
                    out.emplace_back(key, te);
                } while (c.eat(','));
                if (!c.eat(']')) return -1;
            }
        } else {
            double v;
            if (!c.num(v)) return -1;
        }
        if (c.eat(',')) continue;
        if (c.eat('}')) break;
        return -1;
    }
    return have_entries ? (int)out.size() : -1;
}

int read_file(const char* path, std::string& text)
{
    FILE* f = fopen(path, "rb");
    if (!f) return -1;
    char buf[4096];
    size_t k;
    text.clear();
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    fclose(f);
    return 0;
}

// Merge the file's entries with the table and write the table back.
int save_tuning(const char* path)
{
    if (!path) return SK_OK;
    std::string text;
    std::vector<std::pair<std::string, TuneEntry>> old;
    if (read_file(path, text) == 0) (void)parse_tuning(text, old);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& kv : old)
        if (!table().count(kv.first)) table()[kv.first] = kv.second;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return set_error(SK_EINVAL, "cannot write %s", tmp.c_str());
    fprintf(f, "{\"version\": 1, \"entries\": [");
    bool first = true;
    for (auto& kv : table()) {
        const sk_schedule& s = kv.second.sched;
        fprintf(f, "%s\n  {\"key\": \"%s\", \"chunk_rows\": %d, \"block_group\": %d, \"waves\": %d, \"xcd_remap\": %d, "
                   "\"col_tile\": %d, \"global_atomics\": %d, \"gather\": %d, \"ms\": %.6f}",
                first ? "" : ",", kv.first.c_str(), s.chunk_rows, s.block_group, s.waves, s.xcd_remap, s.col_tile,
                s.global_atomics, s.gather, kv.second.ms);
        first = false;
    }
    fprintf(f, "\n]}\n");
    fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) return set_error(SK_EINVAL, "cannot replace %s", path);
    return SK_OK;
}

void store_tuning(const std::string& key, const sk_schedule& s, double ms)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    table()[key] = TuneEntry{s, ms};
}

}  // namespace

std::string apply_key(const sk_sketch* h, int32_t a_dtype, int64_t rows, int64_t n)
{
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << lg) < rows) ++lg;
    char buf[160];
    snprintf(buf, sizeof(buf), "apply a=%d r=%d d=%lld s=%d n=%lld rows=2^%d", a_dtype, h->rounding,
             (long long)h->d, h->s, (long long)n, lg);
    return buf;
}

bool tuning_lookup(const std::string& key, sk_schedule* out)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = table().find(key);
    if (it == table().end()) return false;
    *out = it->second.sched;
    return true;
}

}  // namespace sk

// ---------------------------------------------------------------- batches

struct sk_batch {
    int device = -1;
    int32_t count = 0;
    int32_t a_dtype = 0;
    bool dual = false;
    bool vec = false;
    bool post_scale = false;
    int bg = 0;
    int waves = 0;
    int grid = 0;
    size_t lds_bytes = 0;
    int64_t total_items = 0;
    int64_t max_dn = 0;
    sk_schedule sched{};
    void* dmem = nullptr;                // descriptors + counter
    sk::BatchDesc* descs = nullptr;
    uint32_t* counter = nullptr;
    hipStream_t cap = nullptr;           // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace sk {
namespace {

int check_problem(const sk_problem& p, int idx)
{
    if (p.m < 1 || p.n < 1 || p.n > (1LL << 30)) return set_error(SK_EINVAL, "problem %d: bad shape", idx);
    if (p.s < 1 || p.s > 16) return set_error(SK_EINVAL, "problem %d: s = %d must be in 1..16", idx, p.s);
    if (p.d < 1 || p.d % p.s) return set_error(SK_EINVAL, "problem %d: d must be a positive multiple of s", idx);
    if (p.d / p.s > (1LL << 24)) return set_error(SK_EUNSUPPORTED, "problem %d: d/s too large", idx);
    if (p.rounding < SK_ACC_F32 || p.rounding > SK_ACC_BF16_DITHER)
        return set_error(SK_EINVAL, "problem %d: unknown rounding %d", idx, p.rounding);
    if (p.rounding >= SK_ACC_BF16_RN)
        return set_error(SK_EUNSUPPORTED, "problem %d: BF16 output is not supported in batches", idx);
    const int esz = esize(p.a_dtype);
    if (!esz) return set_error(SK_EINVAL, "problem %d: unknown element type %d", idx, p.a_dtype);
    if (!p.A || !p.SA) return set_error(SK_EINVAL, "problem %d: NULL A or SA", idx);
    if (p.lda < p.n || p.ldsa < p.n) return set_error(SK_EINVAL, "problem %d: leading dimension < n", idx);
    if ((uintptr_t)p.A % (uintptr_t)esz) return set_error(SK_EINVAL, "problem %d: A not element aligned", idx);
    for (int i = 0; i < 4; ++i)
        if (p.reserved[i]) return set_error(SK_EINVAL, "problem %d: reserved fields must be zero", idx);
    if (p.rounding != SK_ACC_F32) {
        if (((uintptr_t)p.SA & 3u) || (p.ldsa & 1))
            return set_error(SK_EUNSUPPORTED, "problem %d: FP16 SA needs a 4-byte aligned base and even ldsa", idx);
    } else if ((uintptr_t)p.SA & 3u) {
        return set_error(SK_EINVAL, "problem %d: FP32 SA not 4-byte aligned", idx);
    }
    return SK_OK;
}

int batch_plan(const sk_problem* probs, int32_t count, const sk_schedule* sched, sk_batch* b)
{
    if (!probs || count < 1) return set_error(SK_EINVAL, "empty batch");
    if (count > 65535) return set_error(SK_EUNSUPPORTED, "at most 65535 problems per batch");
    if (sched) {
        if (sched->chunk_rows < 0 || sched->chunk_rows % 64)
            return set_error(SK_EINVAL, "chunk_rows must be a non-negative multiple of 64");
        if (sched->block_group && sched->block_group != 1 && sched->block_group != 2 && sched->block_group != 4 &&
            sched->block_group != 8)
            return set_error(SK_EINVAL, "block_group must be 0, 1, 2, 4 or 8");
        if (sched->waves && sched->waves != 4 && sched->waves != 8 && sched->waves != 16)
            return set_error(SK_EINVAL, "waves must be 0, 4, 8 or 16");
        if (sched->per_contribution)
            return set_error(SK_EUNSUPPORTED, "per-contribution schedules apply to single sketches only");
        if (sched->col_tile && sched->col_tile != 32 && sched->col_tile != 8)
            return set_error(SK_EINVAL, "batches take col_tile 0 (per problem), 32 or 8");
        if (sched->global_atomics || sched->gather)
            return set_error(SK_EUNSUPPORTED, "global-atomic and gather schedules apply to single sketches only");
        if (sched->reserved[0]) return set_error(SK_EINVAL, "reserved schedule fields must be zero");
    }
    int rc;
    for (int32_t i = 0; i < count; ++i)
        if ((rc = check_problem(probs[i], i))) return rc;
    const int32_t a_dtype = probs[0].a_dtype;
    const bool dual = probs[0].rounding == SK_ACC_F32;
    int64_t maxW = 0, nmax = 0;
    double bytes = 0;
    for (int32_t i = 0; i < count; ++i) {
        if (probs[i].a_dtype != a_dtype) return set_error(SK_EINVAL, "problem %d: element types differ in a batch", i);
        if ((probs[i].rounding == SK_ACC_F32) != dual)
            return set_error(SK_EINVAL, "problem %d: FP32 and FP16 accumulation in one batch", i);
        maxW = std::max<int64_t>(maxW, probs[i].d / probs[i].s);
        nmax = std::max<int64_t>(nmax, probs[i].n);
        bytes += (double)probs[i].m * (double)probs[i].n * esize(a_dtype);
    }
    DeviceInfo dev;
    if ((rc = device_info(&dev))) return rc;
    sk_schedule use{};
    if (sched) use = *sched;
    else (void)tuning_lookup(batch_key(a_dtype, dual, count, bytes, nmax), &use);

    // Column tile per problem: the schedule's, else 8 columns for n <= 16
    // (a 32-column tile would idle half its lanes or more) and 32 otherwise;
    // 8-column tiles run with at most 4 blocks per workgroup.
    auto tile_of = [&](const sk_problem& p, int bgc) {
        int32_t nt = use.col_tile ? use.col_tile : (p.n <= 16 ? 8 : 32);
        if (!apply_tile_ok(nt, bgc)) nt = 32;
        return nt;
    };
    auto lds_for = [&](int bgc) {
        size_t mx = 0;
        for (int32_t i = 0; i < count; ++i)
            mx = std::max(mx, apply_lds_bytes(bgc, probs[i].d / probs[i].s, dual, tile_of(probs[i], bgc)));
        return mx;
    };
    int bg = use.block_group;
    if (bg) {
        for (int32_t i = 0; i < count; ++i)
            if (probs[i].s % bg) return set_error(SK_EINVAL, "block_group %d does not divide s of problem %d", bg, i);
        if (lds_for(bg) > dev.lds_max) return set_error(SK_EUNSUPPORTED, "block_group too large");
    } else {
        for (int cand : {8, 4, 2, 1}) {
            bool ok = lds_for(cand) <= dev.lds_max;
            for (int32_t i = 0; ok && i < count; ++i) ok = probs[i].s % cand == 0;
            if (ok) {
                bg = cand;
                break;
            }
        }
        if (!bg) return set_error(SK_EUNSUPPORTED, "d/s = %lld does not fit in LDS", (long long)maxW);
    }
    const int maxw = batch_max_waves();
    int waves = use.waves ? use.waves : 8;
    if (waves > maxw) return set_error(SK_EINVAL, "waves = %d exceeds %d for this element type", waves, maxw);
    // 16384-row units unless tuned: longer items amortise each item's fixed
    // work (clearing, the exponent sample, decoding, the flush); on the
    // 512-sketch benchmark batch 16384 rows measured 1.15x faster than 4096
    const int32_t chunk = use.chunk_rows ? use.chunk_rows : 16384;
    const int esz = esize(a_dtype);

    std::vector<BatchDesc> descs((size_t)count);
    std::vector<int64_t> items((size_t)count);
    bool vec = true, post = false;
    int64_t max_dn = 0;
    for (int32_t i = 0; i < count; ++i) {
        const sk_problem& p = probs[i];
        const uintptr_t va = esz == 4 ? 8u : 4u;
        const bool aligned = (p.n % 2 == 0) && (p.lda % 2 == 0) && ((uintptr_t)p.A % va == 0);
        vec = vec && aligned;
        const int64_t max_chunk = ((((int64_t)1 << 31) - 1) / (p.lda * esz)) / 64 * 64;
        if (max_chunk < 64) return set_error(SK_EUNSUPPORTED, "problem %d: 64 rows exceed 2 GiB", i);
        ApplyArgs a{};
        a.A = p.A;
        a.lda = p.lda;
        a.rows = p.m;
        a.row_offset = 0;
        a.SA = p.SA;
        a.ldsa = p.ldsa;
        a.n = (int32_t)p.n;
        a.d = (int32_t)p.d;
        a.s = p.s;
        a.W = (uint32_t)(p.d / p.s);
        a.k0 = (uint32_t)p.seed;
        a.k1 = (uint32_t)(p.seed >> 32);
        a.chunk_rows = (int32_t)std::min<int64_t>(chunk, max_chunk);
        a.nt = tile_of(p, bg);
        a.col_tiles = (int32_t)((p.n + a.nt - 1) / a.nt);
        a.bgroups = p.s / bg;
        a.mode = dual ? 0 : p.rounding;
        a.epoch = p.round_epoch;
        a.xcd_remap = 0;
        const float cs = (float)(1.0 / std::sqrt((double)p.s));
        a.scale = (dual && !pow2_scale(p.s)) ? 1.0f : cs;
        descs[i].a = a;
        descs[i].post_scale = (dual && !pow2_scale(p.s)) ? cs : 0.0f;
        post = post || descs[i].post_scale != 0.0f;
        const int64_t units = (p.m + a.chunk_rows - 1) / a.chunk_rows;
        items[i] = units * a.col_tiles * a.bgroups;
        max_dn = std::max<int64_t>(max_dn, p.d * p.n);
    }
    // largest problems first
    std::vector<int32_t> order((size_t)count);
    for (int32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return (double)probs[x].m * probs[x].n > (double)probs[y].m * probs[y].n;
    });
    std::vector<BatchDesc> sorted((size_t)count);
    int64_t total = 0;
    for (int32_t k = 0; k < count; ++k) {
        sorted[k] = descs[order[k]];
        sorted[k].item0 = total;
        total += items[order[k]];
    }
    for (int32_t k = 0; k < count; ++k) {
        sorted[k].a.aligned = vec ? 1 : 0;
    }
    if (total >= 0x7FFFFFFF) return set_error(SK_EUNSUPPORTED, "batch has too many work items");
    const size_t lds = lds_for(bg);
    const int64_t by_lds = std::max<int64_t>(1, (int64_t)(dev.lds_max / lds));
    const int64_t by_waves = std::max<int64_t>(1, 32 / waves);
    const int64_t grid = std::min<int64_t>(total, (int64_t)dev.cus * std::min(by_lds, by_waves));

    b->device = dev.device;
    b->count = count;
    b->a_dtype = a_dtype;
    b->dual = dual;
    b->vec = vec;
    b->post_scale = post;
    b->bg = bg;
    b->waves = waves;
    b->grid = (int)std::max<int64_t>(grid, 1);
    b->lds_bytes = lds;
    b->total_items = total;
    b->max_dn = max_dn;
    b->sched.chunk_rows = chunk;
    b->sched.block_group = bg;
    b->sched.waves = waves;
    b->sched.xcd_remap = 0;
    b->sched.col_tile = use.col_tile;

    const size_t dbytes = (size_t)count * sizeof(BatchDesc);
    const size_t cnt_off = (dbytes + 255) / 256 * 256;
    hipError_t e = hipMalloc(&b->dmem, cnt_off + 256);
    if (e != hipSuccess) {
        b->dmem = nullptr;
        return set_error(SK_ENOMEM, "batch descriptors: %s", hipGetErrorString(e));
    }
    b->descs = (BatchDesc*)b->dmem;
    b->counter = (uint32_t*)((char*)b->dmem + cnt_off);
    if ((e = hipMemcpy(b->descs, sorted.data(), dbytes, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_err(e, "uploading batch descriptors");
    return SK_OK;
}

void batch_free(sk_batch* b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

hipError_t batch_launch(sk_batch* b, hipStream_t st)
{
    (void)hipGetLastError();            // launch checks report this call's errors only
    return launch_batched(b->a_dtype, b->bg, b->vec, b->dual, b->descs, b->count, b->total_items, b->counter,
                          b->grid, b->waves, b->lds_bytes, b->post_scale, b->max_dn, st);
}

int check_device(const sk_batch* b)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice");
    if (dev != b->device) return set_error(SK_EINVAL, "batch was planned on device %d, current is %d", b->device, dev);
    return SK_OK;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

int sketch_batch_create(const sk_problem* probs, int32_t count, const sk_schedule* sched, sk_batch_handle* out)
{
    if (!out) return set_error(SK_EINVAL, "out is NULL");
    *out = nullptr;
    sk_batch* b = new (std::nothrow) sk_batch;
    if (!b) return set_error(SK_ENOMEM, "out of host memory");
    int rc = batch_plan(probs, count, sched, b);
    if (rc) {
        batch_free(b);
        return rc;
    }
    *out = b;
    return SK_OK;
}

int sketch_batch_apply(sk_batch_handle b, void* stream)
{
    if (!b) return set_error(SK_EINVAL, "batch is NULL");
    int rc = check_device(b);
    if (rc) return rc;
    hipError_t e = batch_launch(b, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_err(e, "batched apply");
}

int sketch_batch_graph(sk_batch_handle b, void* stream)
{
    if (!b) return set_error(SK_EINVAL, "batch is NULL");
    int rc = check_device(b);
    if (rc) return rc;
    hipError_t e;
    if (!b->exec) {
        // kernel attributes are set outside the capture
        if ((e = prepare_batched(b->a_dtype, b->bg, b->vec, b->dual, b->lds_bytes)) != hipSuccess)
            return hip_err(e, "preparing the batched kernel");
        if (!b->cap && (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
            b->cap = nullptr;
            return hip_err(e, "hipStreamCreate");
        }
        if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_err(e, "hipStreamBeginCapture");
        hipError_t le = batch_launch(b, b->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_err(le, "capturing the batched apply");
        }
        if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
            b->exec = nullptr;
            return hip_err(e, "hipGraphInstantiate");
        }
    }
    e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_err(e, "hipGraphLaunch");
}

int sketch_batch_schedule(sk_batch_handle b, sk_schedule* out)
{
    if (!b || !out) return set_error(SK_EINVAL, "NULL argument");
    *out = b->sched;
    return SK_OK;
}

int sketch_batch_destroy(sk_batch_handle b)
{
    batch_free(b);
    return SK_OK;
}

int sketch_apply_batched(const sk_problem* probs, int32_t count, const sk_schedule* sched, void* stream)
{
    sk_batch_handle b = nullptr;
    int rc = sketch_batch_create(probs, count, sched, &b);
    if (rc) return rc;
    rc = sketch_batch_apply(b, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    batch_free(b);
    if (rc) return rc;
    return e == hipSuccess ? SK_OK : hip_err(e, "hipStreamSynchronize");
}

int sketch_tune_batch(const sk_problem* probs, int32_t count, const char* cache_path, sk_schedule* out)
{
    if (!probs || count < 1) return set_error(SK_EINVAL, "empty batch");
    for (int32_t i = 0; i < count; ++i) {
        int rc = check_problem(probs[i], i);
        if (rc) return rc;
    }
    const int32_t a_dtype = probs[0].a_dtype;
    const bool dual = probs[0].rounding == SK_ACC_F32;
    const int maxw = batch_max_waves();
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return hip_err(e, "hipStreamCreate");
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipStreamDestroy(st);
        return hip_err(e, "hipEventCreate");
    }
    sk_schedule best{};
    double best_ms = 1e30;
    int rc = SK_OK;
    double bytes = 0;
    int64_t nmax = 0;
    for (int32_t i = 0; i < count; ++i) {
        bytes += (double)probs[i].m * (double)probs[i].n * esize(a_dtype);
        nmax = std::max<int64_t>(nmax, probs[i].n);
    }
    for (int32_t cand = 0; cand < 24; ++cand) {
        const int32_t tiles[] = {0, 32}, chunks[] = {2048, 4096, 8192, 16384}, wavesv[] = {4, 8, 16};
        const int32_t col_tile = tiles[cand / 12], chunk = chunks[(cand / 3) % 4], waves = wavesv[cand % 3];
        {
            if (waves > maxw) continue;
            sk_schedule s{};
            s.chunk_rows = chunk;
            s.waves = waves;
            s.col_tile = col_tile;
            sk_batch* b = new (std::nothrow) sk_batch;
            if (!b) {
                rc = set_error(SK_ENOMEM, "out of host memory");
                break;
            }
            rc = batch_plan(probs, count, &s, b);
            if (rc) {
                batch_free(b);
                if (rc == SK_EUNSUPPORTED) {
                    rc = SK_OK;
                    continue;
                }
                break;
            }
            e = batch_launch(b, st);                      // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = batch_launch(b, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            const sk_schedule used = b->sched;
            batch_free(b);
            if (e != hipSuccess) {
                rc = hip_err(e, "timing a candidate schedule");
                break;
            }
            if (ms / 3.0 < best_ms) {
                best_ms = ms / 3.0;
                best = used;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (rc) return rc;
    if (best_ms >= 1e30) return set_error(SK_EUNSUPPORTED, "no candidate schedule fits this batch");
    store_tuning(batch_key(a_dtype, dual, count, bytes, nmax), best, best_ms);
    if (out) *out = best;
    return save_tuning(cache_path);
}

int sketch_tune_apply(sk_handle h, const void* A, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda, void* SA,
                      int64_t ldsa, const char* cache_path, sk_schedule* out, void* stream)
{
    if (!h) return set_error(SK_EINVAL, "handle is NULL");
    if (rows < 1) return set_error(SK_EINVAL, "tuning needs rows >= 1");
    const int maxw = apply_max_waves(a_dtype, 1);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_err(e, "hipEventCreate");
    sk_sketch tmp = *h;                  // same S; forced schedules only here
    tmp.ws = nullptr;
    tmp.ws_floats = 0;
    tmp.sw = nullptr;
    sk_schedule best{};
    double best_ms = 1e30;
    int rc = SK_OK;
    // column tile x blocks per workgroup x rows per unit x waves, and the two
    // workspace paths: FP32 atomics per contribution, and the bucket-sorted
    // gather (LDS partials against atomics against reading A s times)
    static const int32_t kTiles[6] = {32, 8, 4, 2, 0, -1};   // 0: global atomics, -1: gather
    for (int32_t ti = 0; ti < 6; ++ti) {
        const int32_t nt = kTiles[ti];
      for (int32_t bg : {1, 2, 4, 8}) {
        if (h->s % bg) continue;
        if (nt > 0 ? !apply_tile_ok(nt, bg) : bg != 1) continue;
        for (int32_t chunk : {0, 2048, 4096, 8192, 16384, 32768}) {
            if (nt <= 0 && chunk) continue;
            for (int32_t waves : {4, 8, 16}) {
                if (waves > maxw || (nt <= 0 && waves != 4)) continue;
                if (nt > 0 && waves > apply_max_waves(a_dtype, bg)) continue;
                sk_schedule s{};
                s.block_group = nt > 0 ? bg : 0;
                s.chunk_rows = chunk;
                s.waves = nt > 0 ? waves : 0;
                s.xcd_remap = 1;
                s.col_tile = nt > 0 ? nt : 0;
                s.global_atomics = nt == 0 ? 1 : 0;
                s.gather = nt < 0 ? 1 : 0;
                tmp.sched = s;
                tmp.forced = true;
                rc = sketch_apply(&tmp, A, a_dtype, rows, n, lda, 0, SA, ldsa, 0, 0, stream);
                if (rc == SK_EUNSUPPORTED) {
                    rc = SK_OK;
                    continue;
                }
                if (rc) break;
                e = hipEventRecord(e0, st);
                for (int r = 0; r < 3 && e == hipSuccess && rc == SK_OK; ++r)
                    rc = sketch_apply(&tmp, A, a_dtype, rows, n, lda, 0, SA, ldsa, 0, 0, stream);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_err(e, "timing a candidate schedule");
                    break;
                }
                if (ms / 3.0 < best_ms) {
                    best_ms = ms / 3.0;
                    best = s;
                }
            }
            if (rc) break;
        }
        if (rc) break;
      }
      if (rc) break;
    }
    if (tmp.ws) (void)hipFree(tmp.ws);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (best_ms >= 1e30) return set_error(SK_EUNSUPPORTED, "no candidate schedule fits");
    store_tuning(apply_key(h, a_dtype, rows, n), best, best_ms);
    if (out) *out = best;
    return save_tuning(cache_path);
}

int sketch_load_tuning(const char* path)
{
    if (!path) return set_error(SK_EINVAL, "path is NULL");
    std::string text;
    if (read_file(path, text) != 0) return set_error(SK_EINVAL, "cannot read %s", path);
    std::vector<std::pair<std::string, TuneEntry>> entries;
    const int k = parse_tuning(text, entries);
    if (k < 0) return set_error(SK_EINVAL, "%s is not a tuning file", path);
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (auto& kv : entries) table()[kv.first] = kv.second;
    return k;
}

int sketch_clear_tuning(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    table().clear();
    return SK_OK;
}

}  // extern "C"
