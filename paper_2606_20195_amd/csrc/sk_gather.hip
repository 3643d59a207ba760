// Bucket-sorted gather path of sketch_apply, for sketches whose d/s bucket
// rows leave only narrow column tiles (or none) in LDS.
//
// SA = S A with S a SparseStack operator (paper Section 2.2): row i of A is
// added, with sign sigma_j(i), into bucket row b_j(i) of every block j
// (Section 4.1).  Read by bucket, row b of SA is the signed sum of the rows
// of A hashed to it.  This path forms that sum directly, with no atomics on
// the values:
//
//   count   one thread per row hashes it and counts its s buckets (global
//           32-bit atomics on d counters);
//   scan    one workgroup turns the counts into list offsets and resets each
//           counter to its list's start;
//   fill    the rows are hashed again and each (row, block) appends
//           row | sign << 31 to its bucket's list;
//   sum     one wave per (bucket row, 64-lane column chunk) walks its list,
//           loading 16 bytes of each listed row per lane, and accumulates in
//           FP64; the FP32 rounding of the sum goes to the d x n workspace.
//
// A is read s times (each row once per block), against once for the LDS
// tiles; in exchange every row is hashed twice instead of once per column
// tile, and nothing is added atomically.  The order of a list depends on the
// atomics that fill it, so the FP64 sums may round differently from call to
// call; their FP32 roundings agree except when an FP64 sum lies within its
// own rounding error of an FP32 rounding boundary.  Exact sums (integer A
// with sums below 2^53) give identical results every call.
#include "sk_device.hpp"
#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr int kGatherThreads = 256;    // count / fill: one row per thread
constexpr int kScanThreads = 1024;
constexpr int kSumWaves = 4;           // waves per workgroup of the sum kernel
constexpr int kSumUnroll = 8;          // listed rows in flight per wave

__global__ __launch_bounds__(kGatherThreads) void gather_count_kernel(ApplyArgs p, uint32_t* cnt)
{
    const int64_t stride = (int64_t)gridDim.x * kGatherThreads;
    for (int64_t r = (int64_t)blockIdx.x * kGatherThreads + threadIdx.x; r < p.rows; r += stride) {
        const uint64_t gr = (uint64_t)(p.row_offset + r);
        uint4 w4 = make_uint4(0u, 0u, 0u, 0u);
        for (int j = 0; j < p.s; ++j) {
            if ((j & 3) == 0) w4 = row_words(gr, (uint32_t)j >> 2, p.k0, p.k1);
            const uint32_t w = word_of(w4, (uint32_t)j & 3u);
            const uint32_t b = (uint32_t)j * p.W + bucket_in_block(w, p.W);
            __hip_atomic_fetch_add(&cnt[b], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// off[b] = sum of cnt[b'] for b' < b (off[d] = the total), then cnt[b] = off[b]:
// the counters become the fill kernel's cursors.  One workgroup; each thread
// scans a contiguous segment of the d counters.
__global__ __launch_bounds__(kScanThreads) void gather_scan_kernel(uint32_t* cnt, uint32_t* off, int64_t d)
{
    __shared__ uint32_t part[kScanThreads];
    const int64_t seg = (d + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = min((int64_t)threadIdx.x * seg, d), b1 = min(b0 + seg, d);
    uint32_t sum = 0;
    for (int64_t b = b0; b < b1; ++b) sum += cnt[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    // Hillis-Steele inclusive scan of the segment sums
    for (int o = 1; o < kScanThreads; o <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int64_t b = b0; b < b1; ++b) {
        const uint32_t c = cnt[b];
        off[b] = run;
        cnt[b] = run;
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) off[d] = part[kScanThreads - 1];
}

// The four blocks of one hash call take their list slots with four atomics
// in flight before the entries are stored.
__global__ __launch_bounds__(kGatherThreads) void gather_fill_kernel(ApplyArgs p, uint32_t* cur, uint32_t* list)
{
    const int64_t stride = (int64_t)gridDim.x * kGatherThreads;
    for (int64_t r = (int64_t)blockIdx.x * kGatherThreads + threadIdx.x; r < p.rows; r += stride) {
        const uint64_t gr = (uint64_t)(p.row_offset + r);
        for (int j0 = 0; j0 < p.s; j0 += 4) {
            const uint4 w4 = row_words(gr, (uint32_t)j0 >> 2, p.k0, p.k1);
            const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
            uint32_t at[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + u < p.s) {
                    const uint32_t b = (uint32_t)(j0 + u) * p.W + bucket_in_block(w[u], p.W);
                    at[u] = __hip_atomic_fetch_add(&cur[b], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j0 + u < p.s) list[at[u]] = (uint32_t)r | ((w[u] & 1u) << 31);
        }
    }
}

// Elements per 16-byte lane load.
template <typename AT> struct Lanes { static constexpr int V = 16 / (int)sizeof(AT); };

template <typename AT> __device__ __forceinline__ float elem_to_f32(AT v);
template <> __device__ __forceinline__ float elem_to_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ float elem_to_f32<__half>(__half v) { return __half2float(v); }
template <> __device__ __forceinline__ float elem_to_f32<__hip_bfloat16>(__hip_bfloat16 v)
{
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, v) << 16);
}

// The lane's V elements of one row as FP32: one 16-byte load when the whole
// group lies inside the row and the rows are 16-byte aligned, else one load
// per element that exists (the rest read as zero).
template <typename AT>
__device__ __forceinline__ void load_group(const AT* row, int c, int n, bool vec, float (&x)[Lanes<AT>::V])
{
    constexpr int V = Lanes<AT>::V;
    if (vec && c + V <= n) {
        const uint4 raw = *(const uint4*)(row + c);
        const AT* e = (const AT*)&raw;
#pragma unroll
        for (int k = 0; k < V; ++k) x[k] = elem_to_f32<AT>(e[k]);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) x[k] = (c + k < n) ? elem_to_f32<AT>(row[c + k]) : 0.0f;
    }
}

// ws[b][c] = fl32(sum over the list of bucket row b of sign * A[r][c]), ld n.
// Work item = (bucket row, chunk of 64 V columns), one wave each, chunks of
// one bucket row in consecutive waves (they read the same list and adjacent
// bytes of the same rows).
template <typename AT>
__global__ __launch_bounds__(kSumWaves * 64) void gather_sum_kernel(ApplyArgs p, const uint32_t* off,
                                                                    const uint32_t* list, float* ws, int32_t chunks,
                                                                    int64_t items, int32_t vec)
{
    constexpr int V = Lanes<AT>::V;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int64_t item = (int64_t)blockIdx.x * kSumWaves + wave;
    if (item >= items) return;
    const int64_t b = item / chunks;
    const int c = (int)(item - b * chunks) * 64 * V + lane * V;
    const uint32_t e0 = off[b], e1 = off[b + 1];
    const AT* A = (const AT*)p.A;
    double acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0;
    for (uint32_t e = e0; e < e1; e += kSumUnroll) {
        float x[kSumUnroll][V];
        uint32_t sg[kSumUnroll];
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) {
            // entries past the list's end load nothing and add zero
            const bool live = e + (uint32_t)u < e1;
            const uint32_t ent = live ? list[e + (uint32_t)u] : 0u;
            sg[u] = live ? (ent & 0x80000000u) : 0u;
            if (live) {
                load_group<AT>(A + (int64_t)(ent & 0x7FFFFFFFu) * p.lda, c, p.n, vec != 0, x[u]);
            } else {
#pragma unroll
                for (int k = 0; k < V; ++k) x[u][k] = 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u)
#pragma unroll
            for (int k = 0; k < V; ++k) acc[k] += (double)__uint_as_float(__float_as_uint(x[u][k]) ^ sg[u]);
    }
    float* dst = ws + b * (int64_t)p.n;
#pragma unroll
    for (int k = 0; k < V; ++k)
        if (c + k < p.n) dst[c + k] = (float)acc[k];
}

template <typename AT>
hipError_t sum_typed(const ApplyArgs& a, const uint32_t* off, const uint32_t* list, float* ws, hipStream_t st)
{
    constexpr int V = Lanes<AT>::V;
    const int32_t chunks = (int32_t)((a.n + 64 * V - 1) / (64 * V));
    const int64_t items = (int64_t)a.d * chunks;
    const int64_t grid = (items + kSumWaves - 1) / kSumWaves;
    const int32_t vec = ((a.lda * (int64_t)sizeof(AT)) % 16 == 0 && (uintptr_t)a.A % 16 == 0) ? 1 : 0;
    hipLaunchKernelGGL(gather_sum_kernel<AT>, dim3((unsigned)grid), dim3(kSumWaves * 64), 0, st, a, off, list, ws,
                       chunks, items, vec);
    return hipGetLastError();
}

}  // namespace

size_t gather_aux_words(int64_t d, int64_t rows, int32_t s)
{
    // counters (d), offsets (d + 1), the lists (rows * s), each 256-byte aligned
    auto al = [](int64_t w) { return (size_t)((w + 63) / 64 * 64); };
    return al(d) + al(d + 1) + al(rows * (int64_t)s);
}

bool gather_fits(int64_t d, int64_t n, int64_t rows, int32_t s)
{
    // list entries hold a row index below 2^31; offsets are 32-bit (and a
    // list walk, 8 entries at a time, must not wrap them); the sum
    // kernel's grid (4 work items per workgroup, 64 columns or more per item)
    // stays below 2^31 workgroups
    const int64_t chunks = (n + 255) / 256;
    return rows < ((int64_t)1 << 31) && rows * (int64_t)s < ((int64_t)1 << 31) &&
           d * chunks < ((int64_t)1 << 32);
}

size_t plan_ws_floats(const Plan& pl, int64_t d, int64_t n, int64_t rows, int32_t s)
{
    if (!pl.global) return 0;
    const size_t sum = (size_t)d * (size_t)n;
    return pl.gather ? (sum + 63) / 64 * 64 + gather_aux_words(d, rows, s) : sum;
}

hipError_t launch_gather(int a_dtype, const ApplyArgs& a, float* ws, uint32_t* aux, hipStream_t st)
{
    if (a.rows <= 0) return hipSuccess;
    if (!gather_fits(a.d, a.n, a.rows, a.s)) return hipErrorInvalidValue;
    auto al = [](int64_t w) { return (size_t)((w + 63) / 64 * 64); };
    uint32_t* cnt = aux;
    uint32_t* off = cnt + al(a.d);
    uint32_t* list = off + al((int64_t)a.d + 1);
    hipError_t e = launch_fill(cnt, 4, 1, a.d, a.d, st);
    if (e != hipSuccess) return e;
    const int64_t blocks = (a.rows + kGatherThreads - 1) / kGatherThreads;
    const unsigned grid = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(gather_count_kernel, dim3(grid), dim3(kGatherThreads), 0, st, a, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(gather_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, cnt, off, (int64_t)a.d);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(gather_fill_kernel, dim3(grid), dim3(kGatherThreads), 0, st, a, cnt, list);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    switch (a_dtype) {
    case SK_F32: return sum_typed<float>(a, off, list, ws, st);
    case SK_F16: return sum_typed<__half>(a, off, list, ws, st);
    case SK_BF16: return sum_typed<__hip_bfloat16>(a, off, list, ws, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sk
