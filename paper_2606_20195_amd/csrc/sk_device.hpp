// Device-side primitives of the sketch library (gfx950 / CDNA4).
//
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): the counter-based
//    generator behind both the sketch hash and the rounding noise.
//  * The row hash that defines S (hash version 1): SparseStack puts the j-th
//    nonzero of column i in block j, rows [j*W, (j+1)*W) with W = d/s, with a
//    Rademacher sign (paper Section 2.2, SparseStack definition; Section 4.1
//    for the block ranges).  The paper draws these i.i.d. from an unnamed
//    generator; here counter = (lo32 i, hi32 i, j/4, TAG_SKETCH) under key
//    (lo32 seed, hi32 seed), w = word j%4, bucket = j*W + hi32(w*W),
//    sign = -1 iff w&1.
//  * The three FP32 -> FP16 rounding rules of Section 4.2: round-to-nearest
//    (hardware conversion), exact stochastic rounding (round up iff
//    u*2^-24 * (up - down) < x - down, with 24 random bits u), and dithered
//    rounding (RN of fma(u*2^-24 - 1/2, x*2^-10, x); the paper leaves the ULP
//    scale unset, 2^-10 is this library's reading).  Rounding noise for
//    quantisation site q: word q%4 of Philox((lo32 q/4, hi32 q/4, epoch,
//    TAG_ROUND), key).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace sk {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kTagSketch = 0x534B4348u;
constexpr uint32_t kTagRound = 0x524E4446u;

// One Philox4x32 block: 10 rounds, key advanced by the Weyl constants between
// rounds.  The key is uniform across the wave, so its schedule lives in SGPRs.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t rk0 = k0 + (uint32_t)r * kPhiloxW0;
        const uint32_t rk1 = k1 + (uint32_t)r * kPhiloxW1;
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ rk0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ rk1, (uint32_t)p0);
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(const uint4& w, uint32_t i)
{
    // three selects on the bits of i (a per-lane index must not become a branch)
    const uint32_t a = (i & 1u) ? w.y : w.x;
    const uint32_t b = (i & 1u) ? w.w : w.z;
    return (i & 2u) ? b : a;
}

// Hash words of row i, Philox call g (blocks 4g .. 4g+3).
__device__ __forceinline__ uint4 row_words(uint64_t i, uint32_t g, uint32_t k0, uint32_t k1)
{
    return philox10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), g, kTagSketch), k0, k1);
}

// Bucket offset inside its block (multiply-shift) for hash word w, block height W.
__device__ __forceinline__ uint32_t bucket_in_block(uint32_t w, uint32_t W)
{
    return __umulhi(w, W);
}

// 24 random bits for quantisation site q.
__device__ __forceinline__ uint32_t round_bits(uint64_t q, uint32_t epoch, uint32_t k0, uint32_t k1)
{
    const uint64_t call = q >> 2;
    const uint4 w = philox10(make_uint4((uint32_t)call, (uint32_t)(call >> 32), epoch, kTagRound), k0, k1);
    return word_of(w, (uint32_t)(q & 3)) & 0xFFFFFFu;
}

// The rounding bits of sites q and q + 1 (one Philox block when both fall in it).
__device__ __forceinline__ void round_bits2(uint64_t q, uint32_t epoch, uint32_t k0, uint32_t k1, uint32_t& u0,
                                            uint32_t& u1)
{
    const uint64_t call = q >> 2;
    const uint4 w = philox10(make_uint4((uint32_t)call, (uint32_t)(call >> 32), epoch, kTagRound), k0, k1);
    const uint32_t i = (uint32_t)(q & 3);
    u0 = word_of(w, i) & 0xFFFFFFu;
    u1 = (i != 3u) ? (word_of(w, i + 1u) & 0xFFFFFFu) : round_bits(q + 1, epoch, k0, k1);
}

// x as a materialised FP32 value: the compiler may not fold the operation
// that produced it into a following conversion (an FP32 product followed by
// an FP16 conversion would otherwise become one mixed-precision FMA with a
// single rounding).
__device__ __forceinline__ float as_fp32(float x)
{
    asm("" : "+v"(x));
    return x;
}

// ---- FP32 -> FP16 rounding rules -----------------------------------------

__device__ __forceinline__ uint16_t f16_bits(__half h) { return __half_as_ushort(h); }
__device__ __forceinline__ __half f16_from_bits(uint16_t b) { return __ushort_as_half(b); }

// Round-to-nearest-even (v_cvt_f16_f32 in the default rounding mode).
__device__ __forceinline__ uint16_t q_rn(float x)
{
    return f16_bits(__float2half_rn(x));
}

// Adjacent FP16 values (bit patterns) toward +inf / -inf.
__device__ __forceinline__ uint16_t f16_next_up(uint16_t h)
{
    if (h == 0x8000u) return 0x0001u;
    return (h & 0x8000u) ? (uint16_t)(h - 1u) : (uint16_t)(h + 1u);
}
__device__ __forceinline__ uint16_t f16_next_down(uint16_t h)
{
    if (h == 0x0000u) return 0x8001u;
    return (h & 0x8000u) ? (uint16_t)(h + 1u) : (uint16_t)(h - 1u);
}

// Exact stochastic rounding with 24 random bits u.  All FP32 operations below
// are exact: up - down is a power of two, x - down drops x's low bits, and
// u*2^-24 times a power of two stays in range.
__device__ __forceinline__ uint16_t q_sr(float x, uint32_t u)
{
    const uint16_t hn = q_rn(x);
    if (!(fabsf(x) <= 65504.0f)) return hn;           // beyond FP16 range, or NaN
    const float xn = __half2float(f16_from_bits(hn));
    if (xn == x) return hn;
    uint16_t lo, hi;
    if (xn < x) { lo = hn; hi = f16_next_up(hn); }
    else        { hi = hn; lo = f16_next_down(hn); }
    const float flo = __half2float(f16_from_bits(lo));
    const float fhi = __half2float(f16_from_bits(hi));
    const float gap = fhi - flo;
    const float dist = x - flo;
    const float t = (float)(u & 0xFFFFFFu) * 0x1p-24f;
    return (t * gap < dist) ? hi : lo;
}

// Dithered rounding: RN16(fma(u*2^-24 - 1/2, x*2^-10, x)).
__device__ __forceinline__ uint16_t q_dither(float x, uint32_t u)
{
    if (!isfinite(x)) return q_rn(x);                 // +-inf and NaN pass through
    const float t = (float)(u & 0xFFFFFFu) * 0x1p-24f - 0.5f;
    const float y = __builtin_fmaf(t, x * 0x1p-10f, x);
    return q_rn(y);
}

// mode: 1 RN, 2 SR, 3 dither.
__device__ __forceinline__ uint16_t quantize(int mode, float x, uint32_t u)
{
    if (mode == 2) return q_sr(x, u);
    if (mode == 3) return q_dither(x, u);
    return q_rn(x);
}

// ---- FP32 -> BF16 rounding rules (BF16 = the high 16 bits of an FP32) -------

__device__ __forceinline__ float b16_val(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round-to-nearest-even; NaN stays NaN (quiet, sign kept), overflow gives inf.
__device__ __forceinline__ uint16_t b16_rn(float x)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((b >> 16) | 0x40u);
    return (uint16_t)((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
}

// Exact stochastic rounding (the rule of the FP16 one with BF16 neighbours):
// x lies between trunc (toward zero) and the next BF16 away from zero at
// fraction f/2^16 of the spacing, f = the low 16 bits of x, so with 24 random
// bits the test u*2^-24 * (ru - rd) < x - rd is the integer test u < dist*2^8,
// dist = f for x > 0 and 2^16 - f for x < 0.  Beyond the largest finite BF16
// (and for inf / NaN) the result is the round-to-nearest one.
__device__ __forceinline__ uint16_t b16_sr(float x, uint32_t u)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7FFFFFFFu) > 0x7F7F0000u) return b16_rn(x);
    const uint32_t f = b & 0xFFFFu;
    const uint16_t trunc = (uint16_t)(b >> 16);
    if (f == 0) return trunc;
    const uint16_t away = (uint16_t)(trunc + 1u);     // one spacing further from zero
    const bool neg = (b >> 31) != 0;
    const uint32_t dist = neg ? 0x10000u - f : f;
    const uint16_t ru = neg ? trunc : away, rd = neg ? away : trunc;
    return ((u & 0xFFFFFFu) < (dist << 8)) ? ru : rd;
}

// Dithered rounding with the BF16 epsilon: RN_bf16(fma(u*2^-24 - 1/2, x*2^-7, x)).
__device__ __forceinline__ uint16_t b16_dither(float x, uint32_t u)
{
    if (!isfinite(x)) return b16_rn(x);
    const float t = (float)(u & 0xFFFFFFu) * 0x1p-24f - 0.5f;
    const float y = __builtin_fmaf(t, x * 0x1p-7f, x);
    return b16_rn(y);
}

// mode: 4 RN, 5 SR, 6 dither (BF16 output).
__device__ __forceinline__ uint16_t quantize_bf16(int mode, float x, uint32_t u)
{
    if (mode == 5) return b16_sr(x, u);
    if (mode == 6) return b16_dither(x, u);
    return b16_rn(x);
}

}  // namespace sk
