// Continuous-batching least-squares server: requests are admitted in
// arrival order as slots (streams) and device memory free up, and all
// admitted solves advance together, each on its own stream, driven by one
// scheduler thread that polls their events and enqueues their next phases.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sk_device.hpp"
#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kTagGenA = 0x47454E41u;   // generator streams of the synthetic requests
constexpr uint32_t kTagGenX = 0x47454E58u;
constexpr uint32_t kTagGenN = 0x47454E4Eu;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int hip_err(hipError_t e, const char* what) { return set_error(SK_EHIP, "%s: %s", what, hipGetErrorString(e)); }

// ------------------------------------------------------------ memory pool

// First-fit allocator over byte offsets of one device allocation.
class Pool {
public:
    void init(size_t cap)
    {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(bytes ? bytes : 1);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t capacity() const { return cap_; }

private:
    size_t cap_ = 0;
    std::map<size_t, size_t> free_;
};

// Admission: the head of the FIFO queue goes in when a slot is free and the
// pool fits its footprint.  Shared by the server and the simulator.
struct Admission {
    Pool pool;
    int free_slots = 0;
    bool try_admit(size_t footprint, size_t* off)
    {
        if (free_slots <= 0) return false;
        if (!pool.alloc(footprint, off)) return false;
        --free_slots;
        return true;
    }
    void release(size_t off, size_t footprint)
    {
        pool.release(off, footprint);
        ++free_slots;
    }
};

// ------------------------------------------------------------ synthetic requests

__device__ __forceinline__ float2 normal2(uint64_t idx, uint32_t tag, uint32_t k0, uint32_t k1)
{
    const uint4 w = philox10(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), tag, 0u), k0, k1);
    const float u1 = ((float)w.x + 0.5f) * 2.3283064365386963e-10f;   // (0, 1)
    const float u2 = (float)w.y * 2.3283064365386963e-10f;
    const float r = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincosf(6.283185307179586f * u2, &sn, &cs);
    return make_float2(r * cs, r * sn);
}

template <typename T> __device__ __forceinline__ T from_float(float v);
template <> __device__ __forceinline__ float from_float<float>(float v) { return v; }
template <> __device__ __forceinline__ __half from_float<__half>(float v) { return __float2half_rn(v); }
template <> __device__ __forceinline__ __hip_bfloat16 from_float<__hip_bfloat16>(float v) { return __float2bfloat16(v); }

template <typename T> __device__ __forceinline__ double to_double(T v);
template <> __device__ __forceinline__ double to_double<float>(float v) { return v; }
template <> __device__ __forceinline__ double to_double<__half>(__half v) { return (double)__half2float(v); }
template <> __device__ __forceinline__ double to_double<__hip_bfloat16>(__hip_bfloat16 v)
{
    return (double)__bfloat162float(v);
}

// A[i][c] = N(0,1) (kind 1) or 1e-3 N(0,1) with rows < n replaced by 100 I (kind 2).
template <typename T>
__global__ void gen_matrix_kernel(int kind, uint32_t k0, uint32_t k1, int64_t m, int64_t n, int64_t lda, T* A)
{
    const int64_t total = m * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, c = e - i * n;
        float v;
        if (kind == 2 && i < n) {
            v = i == c ? 100.0f : 0.0f;
        } else {
            v = normal2((uint64_t)e, kTagGenA, k0, k1).x;
            if (kind == 2) v *= 1e-3f;
        }
        A[i * lda + c] = from_float<T>(v);
    }
}

__global__ void gen_xstar_kernel(uint32_t k0, uint32_t k1, int64_t n, double* xs)
{
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x)
        xs[c] = (double)normal2((uint64_t)c, kTagGenX, k0, k1).x;
}

// b = A x* (FP64, from the stored A) + 1e-6 N(0,1): one wave per row.
template <typename T>
__global__ void gen_rhs_kernel(uint32_t k0, uint32_t k1, int64_t m, int64_t n, int64_t lda, const T* A,
                               const double* xs, double* b)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < m; i += nwave) {
        double s = 0.0;
        for (int64_t c = lane; c < n; c += 64) s = fma(to_double<T>(A[i * lda + c]), xs[c], s);
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) b[i] = s + 1e-6 * (double)normal2((uint64_t)i, kTagGenN, k0, k1).x;
    }
}

int esize(int32_t dt) { return dt == SK_F32 ? 4 : (dt == SK_F16 || dt == SK_BF16) ? 2 : 0; }

// Layout of a generated request ahead of its solve workspace.
struct GenLayout {
    int64_t lda = 0;
    size_t oA = 0, ob = 0, ox = 0, bytes = 0;
};

GenLayout gen_layout(const sk_request& r)
{
    GenLayout g;
    const int esz = esize(r.a_dtype);
    g.lda = (r.n + (16 / esz) - 1) / (16 / esz) * (16 / esz);     // 16-byte rows
    g.oA = 0;
    g.ob = align_up((size_t)r.m * g.lda * esz);
    g.ox = g.ob + align_up((size_t)r.m * 8);
    g.bytes = g.ox + align_up((size_t)r.n * 8);
    return g;
}

int check_request(const sk_request& r)
{
    if (r.m < 1) return set_error(SK_EINVAL, "m = %lld must be >= 1", (long long)r.m);
    if (r.s < 1 || r.s > 16) return set_error(SK_EINVAL, "s = %d must be in 1..16", r.s);
    if (r.d < 1 || r.d % r.s) return set_error(SK_EINVAL, "d must be a positive multiple of s");
    if (r.d / r.s > (1LL << 24)) return set_error(SK_EUNSUPPORTED, "d/s too large");
    if (r.rounding < SK_ACC_F32 || r.rounding > SK_ACC_BF16_DITHER)
        return set_error(SK_EINVAL, "unknown rounding %d", r.rounding);
    if (r.gen < 0 || r.gen > 2) return set_error(SK_EINVAL, "gen must be 0, 1 or 2");
    if (!esize(r.a_dtype)) return set_error(SK_EINVAL, "unknown element type %d", r.a_dtype);
    for (int i = 0; i < 4; ++i)
        if (r.reserved[i]) return set_error(SK_EINVAL, "reserved request fields must be zero");
    return SK_OK;
}

sk_sketch sketch_of(const sk_request& r)
{
    sk_sketch S;
    S.m = r.m;
    S.d = r.d;
    S.s = r.s;
    S.seed = r.seed;
    S.rounding = r.rounding;
    return S;
}

// Validate a request and compute its footprint (generated data + workspace).
int footprint_of(const sk_request& r, size_t* bytes, SolveJob* scratch)
{
    int rc = check_request(r);
    if (rc) return rc;
    const void* A = r.A;
    const double* b = r.b;
    int64_t lda = r.lda;
    size_t gen_bytes = 0;
    if (r.gen) {
        const GenLayout g = gen_layout(r);
        A = (const void*)(uintptr_t)kAlign;   // placeholders with the pool's alignment
        b = (const double*)(uintptr_t)kAlign;
        lda = g.lda;
        gen_bytes = g.bytes;
    }
    size_t ws = 0;
    if ((rc = job_prepare(scratch, sketch_of(r), A, r.a_dtype, r.n, lda, b, r.x, &r.opts, &ws))) return rc;
    *bytes = gen_bytes + align_up(ws);
    return SK_OK;
}

struct ReqState {
    sk_request r{};
    uint64_t ticket = 0;
    double t_submit = 0, t_admit = -1, t_done = -1;
    size_t footprint = 0, off = 0;
    int status = 0;
    double ms_ingest = 0;
    sk_solve_info info{};
    bool done = false;
};

struct Slot {
    hipStream_t st = nullptr;
    SolveJob* job = nullptr;
    hipEvent_t g0 = nullptr, g1 = nullptr;
    ReqState* req = nullptr;
    bool gen_timed = false;
};

}  // namespace
}  // namespace sk

struct sk_server {
    int device = -1;
    size_t budget = 0;
    char* pool_base = nullptr;
    sk::Admission adm;
    std::vector<sk::Slot> slots;
    std::deque<sk::ReqState*> queue;
    std::unordered_map<uint64_t, sk::ReqState*> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stopping = false;
    uint64_t next_ticket = 1;
    int64_t submitted = 0, completed = 0;
    size_t in_use = 0, high_water = 0;
    std::chrono::steady_clock::time_point t0;
    sk::SolveJob* scratch = nullptr;       // footprint computation (under mu)
    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace sk {
namespace {

// Enqueue a newly admitted request on its slot: generation, then the solve.
int start_request(sk_server* srv, Slot& sl, ReqState* q)
{
    const sk_request& r = q->r;
    char* base = srv->pool_base + q->off;
    const void* A = r.A;
    const double* b = r.b;
    int64_t lda = r.lda;
    size_t gen_bytes = 0;
    hipError_t e;
    sl.gen_timed = false;
    (void)hipGetLastError();            // launch checks report this request's errors only
    if (r.gen) {
        const GenLayout g = gen_layout(r);
        gen_bytes = g.bytes;
        lda = g.lda;
        A = base + g.oA;
        b = (const double*)(base + g.ob);
        double* xs = (double*)(base + g.ox);
        const uint32_t k0 = (uint32_t)r.gen_seed, k1 = (uint32_t)(r.gen_seed >> 32);
        if ((e = hipEventRecord(sl.g0, sl.st)) != hipSuccess) return hip_err(e, "hipEventRecord");
        const int64_t total = r.m * r.n;
        const unsigned grid = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (total + 255) / 256));
        if (r.a_dtype == SK_F32)
            hipLaunchKernelGGL(gen_matrix_kernel<float>, dim3(grid), dim3(256), 0, sl.st, r.gen, k0, k1, r.m, r.n, lda,
                               (float*)(base + g.oA));
        else if (r.a_dtype == SK_F16)
            hipLaunchKernelGGL(gen_matrix_kernel<__half>, dim3(grid), dim3(256), 0, sl.st, r.gen, k0, k1, r.m, r.n,
                               lda, (__half*)(base + g.oA));
        else
            hipLaunchKernelGGL(gen_matrix_kernel<__hip_bfloat16>, dim3(grid), dim3(256), 0, sl.st, r.gen, k0, k1, r.m,
                               r.n, lda, (__hip_bfloat16*)(base + g.oA));
        hipLaunchKernelGGL(gen_xstar_kernel, dim3(1), dim3(256), 0, sl.st, k0, k1, r.n, xs);
        const unsigned rg = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (r.m + 3) / 4));
        if (r.a_dtype == SK_F32)
            hipLaunchKernelGGL(gen_rhs_kernel<float>, dim3(rg), dim3(256), 0, sl.st, k0, k1, r.m, r.n, lda,
                               (const float*)A, (const double*)xs, (double*)b);
        else if (r.a_dtype == SK_F16)
            hipLaunchKernelGGL(gen_rhs_kernel<__half>, dim3(rg), dim3(256), 0, sl.st, k0, k1, r.m, r.n, lda,
                               (const __half*)A, (const double*)xs, (double*)b);
        else
            hipLaunchKernelGGL(gen_rhs_kernel<__hip_bfloat16>, dim3(rg), dim3(256), 0, sl.st, k0, k1, r.m, r.n, lda,
                               (const __hip_bfloat16*)A, (const double*)xs, (double*)b);
        if ((e = hipGetLastError()) != hipSuccess) return hip_err(e, "generator kernels");
        if ((e = hipEventRecord(sl.g1, sl.st)) != hipSuccess) return hip_err(e, "hipEventRecord");
        sl.gen_timed = true;
    }
    size_t ws = 0;
    int rc = job_prepare(sl.job, sketch_of(r), A, r.a_dtype, r.n, lda, b, r.x, &r.opts, &ws);
    if (rc) return rc;
    return job_start(sl.job, base + gen_bytes, sl.st);
}

void finish_request(sk_server* srv, Slot& sl, int rc)
{
    ReqState* q = sl.req;
    // Kernels still queued on the slot's stream (a failed phase's, or LSQR
    // launches after convergence, which exit at once) may touch the request's
    // block: drain the stream before the block goes back to the allocator.
    (void)hipStreamSynchronize(sl.st);
    (void)hipGetLastError();
    q->status = rc;
    job_info(sl.job, &q->info);
    if (sl.gen_timed) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, sl.g0, sl.g1) == hipSuccess) q->ms_ingest = ms;
        (void)hipGetLastError();
    }
    std::lock_guard<std::mutex> lock(srv->mu);
    q->t_done = srv->now();
    q->done = true;
    srv->adm.release(q->off, q->footprint);
    srv->in_use -= align_up(q->footprint);
    ++srv->completed;
    sl.req = nullptr;
    srv->cv_done.notify_all();
}

void worker_loop(sk_server* srv)
{
    (void)hipSetDevice(srv->device);
    std::vector<Slot*> started;
    for (;;) {
        started.clear();
        {
            std::unique_lock<std::mutex> lock(srv->mu);
            for (;;) {
                bool busy = false;
                for (Slot& sl : srv->slots) busy = busy || sl.req != nullptr;
                // admit from the head while a slot and memory are free
                while (!srv->queue.empty()) {
                    Slot* fs = nullptr;
                    for (Slot& sl : srv->slots)
                        if (!sl.req) {
                            fs = &sl;
                            break;
                        }
                    if (!fs) break;
                    ReqState* q = srv->queue.front();
                    size_t off = 0;
                    if (!srv->adm.try_admit(q->footprint, &off)) break;
                    srv->queue.pop_front();
                    q->off = off;
                    q->t_admit = srv->now();
                    srv->in_use += align_up(q->footprint);
                    srv->high_water = std::max(srv->high_water, srv->in_use);
                    fs->req = q;
                    started.push_back(fs);
                    busy = true;
                }
                if (busy) break;
                if (srv->stopping) return;
                srv->cv_work.wait(lock);
            }
        }
        for (Slot* sl : started) {
            const int rc = start_request(srv, *sl, sl->req);
            if (rc) finish_request(srv, *sl, rc);
        }
        bool progressed = !started.empty();
        for (Slot& sl : srv->slots) {
            if (!sl.req) continue;
            const int rc = job_step(sl.job, false);
            if (rc != 1) {
                finish_request(srv, sl, rc);
                progressed = true;
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

void server_free(sk_server* srv)
{
    if (!srv) return;
    for (Slot& sl : srv->slots) {
        if (sl.st) (void)hipStreamDestroy(sl.st);
        if (sl.g0) (void)hipEventDestroy(sl.g0);
        if (sl.g1) (void)hipEventDestroy(sl.g1);
        job_delete(sl.job);
    }
    for (auto& kv : srv->reqs) delete kv.second;
    job_delete(srv->scratch);
    if (srv->pool_base) (void)hipFree(srv->pool_base);
    delete srv;
}

}  // namespace
}  // namespace sk

using namespace sk;

extern "C" {

int sk_server_create(size_t budget_bytes, int32_t max_slots, sk_server_handle* out)
{
    if (!out) return set_error(SK_EINVAL, "out is NULL");
    *out = nullptr;
    if (budget_bytes < kAlign) return set_error(SK_EINVAL, "budget of %zu bytes is too small", budget_bytes);
    if (max_slots < 1 || max_slots > 64) return set_error(SK_EINVAL, "max_slots must be in 1..64");
    sk_server* srv = new (std::nothrow) sk_server;
    if (!srv) return set_error(SK_ENOMEM, "out of host memory");
    hipError_t e = hipGetDevice(&srv->device);
    if (e != hipSuccess) {
        server_free(srv);
        return hip_err(e, "hipGetDevice");
    }
    srv->budget = budget_bytes / kAlign * kAlign;
    if ((e = hipMalloc((void**)&srv->pool_base, srv->budget)) != hipSuccess) {
        srv->pool_base = nullptr;
        server_free(srv);
        return set_error(SK_ENOMEM, "server pool of %zu bytes: %s", srv->budget, hipGetErrorString(e));
    }
    srv->adm.pool.init(srv->budget);
    srv->adm.free_slots = max_slots;
    srv->slots.resize((size_t)max_slots);
    srv->scratch = job_new();
    for (Slot& sl : srv->slots) {
        sl.job = job_new();
        if (!sl.job || !srv->scratch) {
            server_free(srv);
            return set_error(SK_ENOMEM, "out of host memory");
        }
        if ((e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreate(&sl.g0)) != hipSuccess || (e = hipEventCreate(&sl.g1)) != hipSuccess) {
            server_free(srv);
            return hip_err(e, "creating a server slot");
        }
    }
    srv->t0 = std::chrono::steady_clock::now();
    try {
        srv->worker = std::thread(worker_loop, srv);
    } catch (...) {
        server_free(srv);
        return set_error(SK_ENOMEM, "cannot start the scheduler thread");
    }
    *out = srv;
    return SK_OK;
}

int sk_server_footprint(const sk_request* req, size_t* bytes)
{
    if (!req || !bytes) return set_error(SK_EINVAL, "NULL argument");
    SolveJob* j = job_new();
    if (!j) return set_error(SK_ENOMEM, "out of host memory");
    const int rc = footprint_of(*req, bytes, j);
    job_delete(j);
    return rc;
}

int sk_server_submit(sk_server_handle srv, const sk_request* req, uint64_t* ticket)
{
    if (!srv || !req || !ticket) return set_error(SK_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lock(srv->mu);
    if (srv->stopping) return set_error(SK_EBUSY, "server is shutting down");
    size_t fp = 0;
    int rc = footprint_of(*req, &fp, srv->scratch);
    if (rc) return rc;
    if (align_up(fp) > srv->budget)
        return set_error(SK_EADMIT, "request needs %zu bytes, the server's budget is %zu", fp, srv->budget);
    ReqState* q = new (std::nothrow) ReqState;
    if (!q) return set_error(SK_ENOMEM, "out of host memory");
    q->r = *req;
    q->ticket = srv->next_ticket++;
    q->footprint = fp;
    q->t_submit = srv->now();
    srv->reqs[q->ticket] = q;
    srv->queue.push_back(q);
    ++srv->submitted;
    *ticket = q->ticket;
    srv->cv_work.notify_all();
    return SK_OK;
}

static void fill_result(const ReqState* q, sk_result* out)
{
    std::memset(out, 0, sizeof(*out));
    out->status = q->status;
    out->t_submit = q->t_submit;
    out->t_admit = q->t_admit;
    out->t_done = q->t_done;
    out->ms_ingest = q->ms_ingest;
    out->info = q->info;
}

int sk_server_poll(sk_server_handle srv, uint64_t ticket, int32_t* done, sk_result* out)
{
    if (!srv || !done) return set_error(SK_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_error(SK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    *done = it->second->done ? 1 : 0;
    if (it->second->done) {
        if (out) fill_result(it->second, out);
        delete it->second;
        srv->reqs.erase(it);
    }
    return SK_OK;
}

int sk_server_wait(sk_server_handle srv, uint64_t ticket, sk_result* out)
{
    if (!srv) return set_error(SK_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lock(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return set_error(SK_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ReqState* q = it->second;
    srv->cv_done.wait(lock, [&] { return q->done; });
    if (out) fill_result(q, out);
    srv->reqs.erase(ticket);
    delete q;
    return SK_OK;
}

int sk_server_stats(sk_server_handle srv, sk_server_info* out)
{
    if (!srv || !out) return set_error(SK_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(srv->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->queued = (int64_t)srv->queue.size();
    int64_t inflight = 0;
    for (const Slot& sl : srv->slots) inflight += sl.req ? 1 : 0;
    out->in_flight = inflight;
    out->bytes_in_use = (int64_t)srv->in_use;
    out->bytes_high_water = (int64_t)srv->high_water;
    out->budget = (int64_t)srv->budget;
    out->slots = (int32_t)srv->slots.size();
    return SK_OK;
}

double sk_server_clock(sk_server_handle srv) { return srv ? srv->now() : 0.0; }

int sk_server_destroy(sk_server_handle srv)
{
    if (!srv) return SK_OK;
    {
        std::lock_guard<std::mutex> lock(srv->mu);
        srv->stopping = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    server_free(srv);
    return SK_OK;
}

int sk_server_simulate(size_t budget_bytes, int32_t max_slots, int32_t count, const double* arrive,
                       const uint64_t* footprint, const double* service, double* admit, double* done)
{
    if (count < 0 || max_slots < 1) return set_error(SK_EINVAL, "bad count or slots");
    if (count > 0 && (!arrive || !footprint || !service || !admit || !done)) return set_error(SK_EINVAL, "NULL array");
    const size_t budget = budget_bytes / kAlign * kAlign;
    for (int32_t k = 0; k < count; ++k) {
        if (k > 0 && arrive[k] < arrive[k - 1]) return set_error(SK_EINVAL, "arrivals must be non-decreasing");
        if (!(service[k] >= 0)) return set_error(SK_EINVAL, "negative service time");
        if (align_up(footprint[k] ? footprint[k] : 1) > budget)
            return set_error(SK_EADMIT, "request %d needs %llu bytes > budget", k, (unsigned long long)footprint[k]);
    }
    Admission adm;
    adm.pool.init(budget);
    adm.free_slots = max_slots;
    using Ev = std::pair<double, int32_t>;            // (completion time, request)
    std::priority_queue<Ev, std::vector<Ev>, std::greater<Ev>> running;
    std::deque<int32_t> queue;
    std::vector<size_t> offs((size_t)count);
    int32_t next = 0;
    double t = 0.0;
    while (next < count || !queue.empty() || !running.empty()) {
        // next event: an arrival or a completion
        double tn = 1e300;
        if (next < count) tn = arrive[next];
        if (!running.empty()) tn = std::min(tn, running.top().first);
        t = std::max(t, tn);
        while (!running.empty() && running.top().first <= t) {
            const int32_t k = running.top().second;
            running.pop();
            adm.release(offs[k], footprint[k]);
        }
        while (next < count && arrive[next] <= t) queue.push_back(next++);
        while (!queue.empty()) {
            const int32_t k = queue.front();
            size_t off = 0;
            if (!adm.try_admit(footprint[k], &off)) break;
            queue.pop_front();
            offs[k] = off;
            admit[k] = t;
            done[k] = t + service[k];
            running.emplace(done[k], k);
        }
    }
    return SK_OK;
}

}  // extern "C"
