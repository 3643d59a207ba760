// One global atomic per contribution: the kernel scheme of the paper's
// Section 4, kept as a reference for accuracy and atomic counts beside the
// workgroup-partial kernels of sk_apply.hip.
//
// Every thread owns one (row, column pair) at a time.  It hashes its row
// (hash version 1, the same words as every other kernel), and for each of the
// s blocks forms the exact FP32 value v = fl32(rho * fl32(1/sqrt(s)) * x) of
// both columns (Section 4.1: the stored S value times the element).  FP32
// output adds v with FP32 atomics (Section 4.1's scatter).  FP16 output
// rounds v to FP16 with the handle's rule (RN, exact SR or dither, Section
// 4.2) and adds the pair with one packed FP16 atomic, as the vectorised
// Section 4.2 kernel does; the atomic's own addition rounds to nearest.
// SR and dither draw site q = (i*s + j)*n + c of the rounding stream, i the
// global row, j the block, c the column.
#include "sk_device.hpp"
#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr int kContribThreads = 256;

template <typename AT> __device__ __forceinline__ float elem_f32(const AT* p);
template <> __device__ __forceinline__ float elem_f32<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float elem_f32<__half>(const __half* p) { return __half2float(*p); }
template <> __device__ __forceinline__ float elem_f32<__hip_bfloat16>(const __hip_bfloat16* p)
{
    return __uint_as_float((uint32_t)__builtin_bit_cast(unsigned short, *p) << 16);
}

template <typename AT, bool F16OUT>
__global__ __launch_bounds__(kContribThreads) void contrib_kernel(ApplyArgs p)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const uint64_t npairs = (uint64_t)(p.n + 1) / 2;
    const uint64_t total = (uint64_t)p.rows * npairs;
    const uint64_t stride = (uint64_t)gridDim.x * kContribThreads;
    const float cs = p.scale;
    const uint32_t W = p.W;
    for (uint64_t t = (uint64_t)blockIdx.x * kContribThreads + threadIdx.x; t < total; t += stride) {
        const uint64_t r = t / npairs;
        const int c = 2 * (int)(t - r * npairs);
        const bool two = c + 1 < p.n;
        const AT* row = (const AT*)p.A + (int64_t)r * p.lda;
        const float x0 = elem_f32<AT>(row + c);
        const float x1 = two ? elem_f32<AT>(row + c + 1) : 0.0f;
        const uint64_t gr = (uint64_t)p.row_offset + r;
        for (int j = 0; j < p.s; ++j) {
            const uint4 w4 = row_words(gr, (uint32_t)j >> 2, p.k0, p.k1);
            const uint32_t w = word_of(w4, (uint32_t)j & 3u);
            const int64_t b = (int64_t)j * W + bucket_in_block(w, W);
            const float sv = (w & 1u) ? -cs : cs;          // the stored value of S
            const float v0 = sv * x0, v1 = sv * x1;
            if constexpr (F16OUT) {
                const uint64_t q = ((gr * (uint64_t)p.s + (uint64_t)j) * (uint64_t)p.n) + (uint64_t)c;
                uint32_t u0 = 0, u1 = 0;
                if (p.mode >= 2) {
                    u0 = round_bits(q, p.epoch, p.k0, p.k1);
                    u1 = round_bits(q + 1, p.epoch, p.k0, p.k1);
                }
                const uint16_t h0 = quantize(p.mode, v0, u0);
                // -0.0 leaves the neighbouring half unchanged (x + -0 == x for every x)
                const uint16_t h1 = two ? quantize(p.mode, v1, u1) : (uint16_t)0x8000u;
                const h2 hv = __builtin_bit_cast(h2, (uint32_t)h0 | ((uint32_t)h1 << 16));
                __builtin_amdgcn_global_atomic_fadd_v2f16((h2*)((uint16_t*)p.SA + b * p.ldsa + c), hv);
            } else {
                float* dst = (float*)p.SA + b * p.ldsa + c;
                __hip_atomic_fetch_add(dst, v0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (two) __hip_atomic_fetch_add(dst + 1, v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// FP16 finish of the workspace path: SA[b][c] += RN16-add of the rounding of
// fl32(scale * ws[b][c]), one rounding per entry at site q = site0 + b*n + c
// (the partial-sum scheme's rule for a unit that starts at global row
// site0 / (d*n) and spans the whole call).
__global__ __launch_bounds__(kContribThreads) void finish16_kernel(const float* ws, int64_t d, int32_t n,
                                                                   uint16_t* SA, int64_t ldsa, int32_t mode,
                                                                   float scale, uint64_t site0, uint32_t epoch,
                                                                   uint32_t k0, uint32_t k1)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const int64_t npairs = (n + 1) / 2;
    const int64_t total = d * npairs;
    for (int64_t e = (int64_t)blockIdx.x * kContribThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kContribThreads) {
        const int64_t b = e / npairs;
        const int c = 2 * (int)(e - b * npairs);
        const bool two = c + 1 < n;
        const uint64_t q = site0 + (uint64_t)b * (uint64_t)n + (uint64_t)c;
        uint32_t u0 = 0, u1 = 0;
        if (mode >= 2) {
            u0 = round_bits(q, epoch, k0, k1);
            u1 = round_bits(q + 1, epoch, k0, k1);
        }
        const uint16_t h0 = quantize(mode, as_fp32(ws[b * n + c] * scale), u0);
        const uint16_t h1 = two ? quantize(mode, as_fp32(ws[b * n + c + 1] * scale), u1) : (uint16_t)0x8000u;
        const h2 hv = __builtin_bit_cast(h2, (uint32_t)h0 | ((uint32_t)h1 << 16));
        __builtin_amdgcn_global_atomic_fadd_v2f16((h2*)(SA + b * ldsa + c), hv);
    }
}

// BF16 finish: SA[b][c] = rounding of fl32(scale * ws[b][c]) to BF16 (mode 4
// RN, 5 SR, 6 dither; site q = site0 + b*n + c), or with `accumulate` the
// round-to-nearest BF16 sum of SA[b][c] and that rounding.  One thread per
// entry, plain stores.  Two BF16 values add exactly in FP32 whenever their
// exponents differ by at most 16; otherwise the smaller is below a quarter
// of the larger's spacing and FP32 rounding cannot reach a BF16 midpoint,
// so the FP32 sum rounded to BF16 is the correctly rounded BF16 sum.
__global__ __launch_bounds__(kContribThreads) void finish_bf16_kernel(const float* ws, int64_t d, int32_t n,
                                                                      uint16_t* SA, int64_t ldsa, int32_t mode,
                                                                      float scale, uint64_t site0, uint32_t epoch,
                                                                      uint32_t k0, uint32_t k1, int32_t accumulate)
{
    const int64_t total = d * n;
    for (int64_t e = (int64_t)blockIdx.x * kContribThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kContribThreads) {
        const int64_t b = e / n;
        const int c = (int)(e - b * n);
        const uint64_t q = site0 + (uint64_t)b * (uint64_t)n + (uint64_t)c;
        const uint32_t u = mode != 4 ? round_bits(q, epoch, k0, k1) : 0u;
        uint16_t h = quantize_bf16(mode, as_fp32(ws[e] * scale), u);
        uint16_t* dst = SA + b * ldsa + c;
        if (accumulate) h = b16_rn(b16_val(*dst) + b16_val(h));
        *dst = h;
    }
}

template <typename AT>
hipError_t contrib_typed(const ApplyArgs& a, hipStream_t st)
{
    const uint64_t total = (uint64_t)a.rows * (uint64_t)((a.n + 1) / 2);
    if (total == 0) return hipSuccess;
    const uint64_t blocks = (total + kContribThreads - 1) / kContribThreads;
    const unsigned grid = (unsigned)(blocks < 16384 ? blocks : 16384);
    if (a.mode == 0)
        hipLaunchKernelGGL((contrib_kernel<AT, false>), dim3(grid), dim3(kContribThreads), 0, st, a);
    else
        hipLaunchKernelGGL((contrib_kernel<AT, true>), dim3(grid), dim3(kContribThreads), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_finish16(const float* ws, int64_t d, int32_t n, uint16_t* SA, int64_t ldsa, int32_t mode,
                           float scale, uint64_t site0, uint32_t epoch, uint32_t k0, uint32_t k1, hipStream_t st)
{
    const int64_t total = d * ((n + 1) / 2);
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + kContribThreads - 1) / kContribThreads;
    hipLaunchKernelGGL(finish16_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kContribThreads), 0,
                       st, ws, d, n, SA, ldsa, mode, scale, site0, epoch, k0, k1);
    return hipGetLastError();
}

hipError_t launch_finish_bf16(const float* ws, int64_t d, int32_t n, uint16_t* SA, int64_t ldsa, int32_t mode,
                              float scale, uint64_t site0, uint32_t epoch, uint32_t k0, uint32_t k1, bool accumulate,
                              hipStream_t st)
{
    const int64_t total = d * n;
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + kContribThreads - 1) / kContribThreads;
    hipLaunchKernelGGL(finish_bf16_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kContribThreads), 0,
                       st, ws, d, n, SA, ldsa, mode, scale, site0, epoch, k0, k1, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_contrib(int a_dtype, const ApplyArgs& a, hipStream_t st)
{
    switch (a_dtype) {
    case SK_F32: return contrib_typed<float>(a, st);
    case SK_F16: return contrib_typed<__half>(a, st);
    case SK_BF16: return contrib_typed<__hip_bfloat16>(a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sk
