// sketch_apply: the generic kernels (clear, scale, hash, quantise, batch
// set-up) and the dispatch to the per-element-type kernels of
// sk_apply_item.hpp.
#include "sk_apply_item.hpp"

namespace sk {
namespace {

// Clears every problem's SA (and resets the work counter) before a batched apply.
__global__ void batch_fill_kernel(const BatchDesc* descs, int32_t count, uint32_t* counter)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter = 0u;
    const int pi = (int)blockIdx.y;
    if (pi >= count) return;
    const ApplyArgs& a = descs[pi].a;
    const int64_t total = (int64_t)a.d * a.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / a.n, c = e - r * a.n;
        if (a.mode == 0) ((float*)a.SA)[r * a.ldsa + c] = 0.0f;
        else ((uint16_t*)a.SA)[r * a.ldsa + c] = 0;
    }
}

// FP32 problems whose 1/sqrt(s) is not a power of two: SA = fl32(c_s * SA).
__global__ void batch_scale_kernel(const BatchDesc* descs, int32_t count)
{
    const int pi = (int)blockIdx.y;
    if (pi >= count) return;
    const BatchDesc& bd = descs[pi];
    if (bd.post_scale == 0.0f) return;
    const ApplyArgs& a = bd.a;
    const int64_t total = (int64_t)a.d * a.n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / a.n, c = e - r * a.n;
        float* dst = (float*)a.SA + r * a.ldsa + c;
        *dst = bd.post_scale * *dst;
    }
}

__global__ void fill_kernel(void* p, int elem_bytes, int64_t rows, int64_t cols, int64_t ld)
{
    const int64_t total = rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / cols, c = e % cols;
        if (elem_bytes == 4) ((float*)p)[r * ld + c] = 0.0f;
        else ((uint16_t*)p)[r * ld + c] = 0;
    }
}

// SA = (accumulate ? SA : 0) + fl32(c * ws), ws a d x n FP32 array (ld n).
// Without a workspace (ws == SA) the scale is applied in place.
__global__ void scale_kernel(float* SA, int64_t d, int64_t n, int64_t ldsa, const float* ws, float c,
                             int accumulate)
{
    const int64_t total = d * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / n, col = e % n;
        float* dst = SA + r * ldsa + col;
        if (ws == nullptr) {
            *dst = c * *dst;
        } else {
            const float v = c * ws[r * n + col];
            *dst = accumulate ? *dst + v : v;
        }
    }
}

__global__ void hash_kernel(uint32_t k0, uint32_t k1, uint32_t W, int32_t s, int64_t row_begin,
                            int64_t count, int32_t* buckets, int8_t* signs)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t i = (uint64_t)(row_begin + t);
        uint4 w4 = make_uint4(0, 0, 0, 0);
        for (int32_t j = 0; j < s; ++j) {
            if ((j & 3) == 0) w4 = row_words(i, (uint32_t)j >> 2, k0, k1);
            const uint32_t w = word_of(w4, (uint32_t)j & 3u);
            buckets[t * s + j] = (int32_t)((uint32_t)j * W + bucket_in_block(w, W));
            signs[t * s + j] = (w & 1u) ? (int8_t)-1 : (int8_t)1;
        }
    }
}

__global__ void quantize_kernel(int mode, const float* x, uint16_t* out, int64_t count, uint32_t k0,
                                uint32_t k1, uint32_t epoch, uint64_t site0)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (int64_t)gridDim.x * blockDim.x) {
        const bool noisy = mode == 2 || mode == 3 || mode == 5 || mode == 6;
        const uint32_t u = noisy ? round_bits(site0 + (uint64_t)t, epoch, k0, k1) : 0u;
        out[t] = mode >= 4 ? quantize_bf16(mode, x[t], u) : quantize(mode, x[t], u);
    }
}

// Streaming read of `bytes` bytes (a multiple of 16): every 16-byte word is
// loaded once with a non-temporal load and folded by XOR; each wave XORs its
// fold into one of 256 output words (workgroup id mod 256), so no word takes
// more than a few dozen atomics.  The read ceiling against which the apply
// kernel's bandwidth is judged.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_read_kernel(const u32x4* p, int64_t words, uint32_t* out)
{
    u32x4 acc = {0u, 0u, 0u, 0u};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < words; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i), b = __builtin_nontemporal_load(p + i + stride);
        const u32x4 c = __builtin_nontemporal_load(p + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(p + i + 3 * stride);
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < words; i += stride) acc ^= __builtin_nontemporal_load(p + i);
    uint32_t v = acc.x ^ acc.y ^ acc.z ^ acc.w;
    for (int o = 32; o > 0; o >>= 1) v ^= (uint32_t)__shfl_xor((int)v, o);
    if ((threadIdx.x & 63) == 0) atomicXor(out + (blockIdx.x & 255u), v);
}

unsigned grid_for(int64_t work, int threads)
{
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

}  // namespace

int apply_max_waves(int32_t a_dtype, int32_t bg)
{
    if (bg >= 8) return 8;
    return (a_dtype == SK_F32 ? kMaxThreads<float> : kMaxThreads<__half>) / 64;
}

int batch_max_waves() { return kBatchThreads / 64; }

bool apply_tile_ok(int32_t nt, int32_t bg)
{
    switch (nt) {
    case 32: return bg == 1 || bg == 2 || bg == 4 || bg == 8;
    case 8: return bg == 1 || bg == 2 || bg == 4;
    case 4: return bg == 1 || bg == 2;
    case 2: return bg == 1;
    default: return false;
    }
}

size_t apply_lds_bytes(int32_t bg, int64_t W, bool dual, int32_t nt)
{
    if (!apply_tile_ok(nt, bg)) return (size_t)-1;
    // fixed-point array(s) + per-bucket-row counters + control words + the
    // outlier list (which holds the exponent sample before the pass)
    const size_t extra = (2 * (size_t)bg * (size_t)W + kCtlWords + kAuxWords) * 4;
    const size_t narr = dual ? 2 : 1;
    size_t words;
    if (nt != kNT) words = (size_t)bg * (size_t)W * (size_t)nt;
    else if (bg == 1) words = (size_t)W * kNT;
    else words = (size_t)(bg / 2) * ((size_t)W * 64u + 64u);
    return narr * words * 4 + extra;
}

hipError_t launch_apply(int a_dtype, const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    switch (a_dtype) {
    case SK_F32: return launch_apply_f32(plan, a, st);
    case SK_F16: return launch_apply_f16(plan, a, st);
    case SK_BF16: return launch_apply_bf16(plan, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t prepare_batched(int a_dtype, int bg, bool vec, bool dual, size_t lds_bytes)
{
    switch (a_dtype) {
    case SK_F32: return batched_f32(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
    case SK_F16: return batched_f16(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
    case SK_BF16: return batched_bf16(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batched(int a_dtype, int bg, bool vec, bool dual, const BatchDesc* descs, int32_t count,
                          int64_t total_items, uint32_t* counter, int grid, int waves, size_t lds_bytes,
                          bool post_scale, int64_t max_dn, hipStream_t st)
{
    const unsigned fx = grid_for(max_dn, 256) < 64u ? grid_for(max_dn, 256) : 64u;
    hipLaunchKernelGGL(batch_fill_kernel, dim3(fx, (unsigned)count), dim3(256), 0, st, descs, count, counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (a_dtype) {
    case SK_F32: e = batched_f32(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    case SK_F16: e = batched_f16(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    case SK_BF16: e = batched_bf16(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || !post_scale) return e;
    hipLaunchKernelGGL(batch_scale_kernel, dim3(fx, (unsigned)count), dim3(256), 0, st, descs, count);
    return hipGetLastError();
}

hipError_t launch_stream_read(const void* p, int64_t bytes, uint32_t* out, hipStream_t st)
{
    hipLaunchKernelGGL(stream_read_kernel, dim3(8192), dim3(256), 0, st, (const u32x4*)p, bytes / 16, out);
    return hipGetLastError();
}

hipError_t launch_fill(void* p, int elem_bytes, int64_t rows, int64_t cols, int64_t ld, hipStream_t st)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(rows * cols, 256)), dim3(256), 0, st, p, elem_bytes, rows,
                       cols, ld);
    return hipGetLastError();
}

hipError_t launch_scale(float* SA, int64_t d, int64_t n, int64_t ldsa, const float* ws, float c, int accumulate,
                        hipStream_t st)
{
    hipLaunchKernelGGL(scale_kernel, dim3(grid_for(d * n, 256)), dim3(256), 0, st, SA, d, n, ldsa, ws, c,
                       accumulate);
    return hipGetLastError();
}

hipError_t launch_hash(uint64_t seed, int64_t d, int32_t s, int64_t row_begin, int64_t count, int32_t* buckets,
                       int8_t* signs, hipStream_t st)
{
    hipLaunchKernelGGL(hash_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, (uint32_t)seed,
                       (uint32_t)(seed >> 32), (uint32_t)(d / s), s, row_begin, count, buckets, signs);
    return hipGetLastError();
}

hipError_t launch_quantize(int mode, const float* x, uint16_t* out, int64_t count, uint64_t seed, uint32_t epoch,
                           uint64_t site0, hipStream_t st)
{
    hipLaunchKernelGGL(quantize_kernel, dim3(grid_for(count, 256)), dim3(256), 0, st, mode, x, out, count,
                       (uint32_t)seed, (uint32_t)(seed >> 32), epoch, site0);
    return hipGetLastError();
}

}  // namespace sk
