// Device side of sketch_apply for gfx950: the work item (apply_item), the
// single-call and persistent kernels, and their launch templates.  Each
// element type's kernels are instantiated in a source file of their own
// (sk_apply_f32.hip, sk_apply_f16.hip, sk_apply_bf16.hip).
//
//
// SA = S * A with S a SparseStack operator (paper Section 2.2; s = 1 is
// CountSketch), formed by scattering every row of A into its s hashed target
// rows (Section 4.1).  The paper does one global atomic per contribution;
// here each workgroup accumulates an FP32 partial of its rows in LDS and adds
// it into SA once (FP32 atomics, or after FP16 quantisation with the rounding
// rules of Section 4.2, packed FP16 atomics).
//
// Decomposition.  A workgroup owns one unit of consecutive rows, one tile of
// 32 columns and a group of BG SparseStack blocks; its LDS partial holds
// BG * (d/s) bucket rows of 32 FP32 values.  Each wave streams 64-row tiles:
// lane (k, q) = (lane / 16, lane % 16) handles row slot k and column pair
// 2q, 2q+1, so one wave instruction covers 4 rows of 64 contiguous bytes
// (FP16) or 128 bytes (FP32).  Lane (k, q) also hashes row 4q + k of the
// tile; in group g the 16 lanes of DPP row k read that row's bucket offsets
// and signs from lane (k, g) with a row_newbcast DPP broadcast, so the hash is
// computed once per row and no LDS traffic is spent distributing it.
//
// Bank-conflict-free scatter.  In instruction jj the lanes of slot k update
// local block (jj + k) mod BG, so the four slots of a wave instruction hit
// four different blocks.  Block lb's bucket rows start at an LDS word
// offset congruent to 32*(lb & 1) + ((lb >> 1) & 1) modulo 64, so with 64
// banks the four slots' even (then odd) columns land on four disjoint
// 16-bank sets whatever the buckets are.
#pragma once

#include <type_traits>

#include "sk_device.hpp"
#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr int kNT = 32;     // the widest column tile (and the per-column control arrays)
constexpr int kTile = 64;   // rows per wave tile

// Geometry of a column tile of NT columns: L = NT/2 lanes per row slot (one
// column pair each), K = 64/L row slots per wave instruction, G = L wave
// instructions per 64-row tile.  NT = 32 (16-lane slots, row_newbcast
// broadcasts) is the main path; NT = 8, 4 and 2 (quad_perm broadcasts, or
// none) let larger d/s fit in LDS and keep lanes busy on narrow matrices.
template <int NT>
struct Geom {
    static constexpr int L = NT / 2;
    static constexpr int K = 64 / L;
    static constexpr int G = L;
};

template <int BG, int NT>
__host__ __device__ constexpr uint32_t lds_row(uint32_t lb, uint32_t o, uint32_t W)
{
    return NT != kNT ? (lb * W + o) * NT
           : BG == 1 ? o * kNT
                     : (lb >> 1) * (W * 64u + 64u) + o * 64u + 32u * (lb & 1u) + ((lb >> 1) & 1u);
}

template <int BG, int NT>
__host__ __device__ constexpr size_t lds_words(uint32_t W)
{
    return NT != kNT ? (size_t)BG * W * NT
           : BG == 1 ? (size_t)W * kNT : (size_t)(BG / 2) * ((size_t)W * 64u + 64u);
}

// Raw storage of one lane's column pair and its conversion to FP32.
template <typename AT> struct PairRaw;
template <> struct PairRaw<float> { float2 v; };
template <> struct PairRaw<__half> { uint32_t v; };
template <> struct PairRaw<__hip_bfloat16> { uint32_t v; };

__device__ __forceinline__ void to_f32(const PairRaw<float>& r, float& lo, float& hi)
{
    lo = r.v.x;
    hi = r.v.y;
}
__device__ __forceinline__ void to_f32(const PairRaw<__half>& r, float& lo, float& hi)
{
    lo = __half2float(__ushort_as_half((unsigned short)(r.v & 0xFFFFu)));
    hi = __half2float(__ushort_as_half((unsigned short)(r.v >> 16)));
}
__device__ __forceinline__ void to_f32(const PairRaw<__hip_bfloat16>& r, float& lo, float& hi)
{
    lo = __uint_as_float(r.v << 16);
    hi = __uint_as_float(r.v & 0xFFFF0000u);
}

// Buffer loads of the lane's column pair (columns c and c+1 of one row).  The
// resource covers exactly the workgroup's unit of rows, so loads of rows past
// its end return zero.  VEC: one vector load (needs even n and lda and an
// aligned base); otherwise two scalar loads, the second `d1` elements further
// (1, or 0 when c+1 is past the last column; such values only reach LDS
// columns that are never flushed).
template <bool VEC, typename AT>
__device__ __forceinline__ PairRaw<AT> load_pair(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so, uint32_t d1);

template <>
__device__ __forceinline__ PairRaw<float> load_pair<true, float>(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so,
                                                                 uint32_t)
{
    PairRaw<float> r;
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)vo, (int)so, 0);
    r.v = __builtin_bit_cast(float2, v);
    return r;
}
template <>
__device__ __forceinline__ PairRaw<float> load_pair<false, float>(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so,
                                                                  uint32_t d1)
{
    PairRaw<float> r;
    r.v.x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)vo, (int)so, 0));
    r.v.y = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(vo + 4u * d1), (int)so, 0));
    return r;
}
template <bool VEC, typename AT>
__device__ __forceinline__ PairRaw<AT> load_pair16(__amdgpu_buffer_rsrc_t rs, uint32_t vo, uint32_t so, uint32_t d1)
{
    PairRaw<AT> r;
    if constexpr (VEC) {
        r.v = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vo, (int)so, 0);
    } else {
        const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)vo, (int)so, 0);
        const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)(vo + 2u * d1), (int)so, 0);
        r.v = lo | (hi << 16);
    }
    return r;
}
template <>
__device__ __forceinline__ PairRaw<__half> load_pair<true, __half>(__amdgpu_buffer_rsrc_t rs, uint32_t vo,
                                                                   uint32_t so, uint32_t d1)
{
    return load_pair16<true, __half>(rs, vo, so, d1);
}
template <>
__device__ __forceinline__ PairRaw<__half> load_pair<false, __half>(__amdgpu_buffer_rsrc_t rs, uint32_t vo,
                                                                    uint32_t so, uint32_t d1)
{
    return load_pair16<false, __half>(rs, vo, so, d1);
}
template <>
__device__ __forceinline__ PairRaw<__hip_bfloat16> load_pair<true, __hip_bfloat16>(__amdgpu_buffer_rsrc_t rs,
                                                                                   uint32_t vo, uint32_t so,
                                                                                   uint32_t d1)
{
    return load_pair16<true, __hip_bfloat16>(rs, vo, so, d1);
}
template <>
__device__ __forceinline__ PairRaw<__hip_bfloat16> load_pair<false, __hip_bfloat16>(__amdgpu_buffer_rsrc_t rs,
                                                                                    uint32_t vo, uint32_t so,
                                                                                    uint32_t d1)
{
    return load_pair16<false, __hip_bfloat16>(rs, vo, so, d1);
}


// Every lane of a row slot takes the value of the slot's lane G: for 16-lane
// slots row_newbcast:G, for 4-lane slots quad_perm [G,G,G,G], for 2-lane
// slots quad_perm [G,G,2+G,2+G]; one-lane slots hold their own row.
template <int NT, int G>
__device__ __forceinline__ uint32_t bcast_slot(uint32_t v)
{
    // bound_ctrl set and old = 0 let the compiler fold the move into the consumer
    // (v_add_u32_dpp / v_xor_b32_dpp); no lane is out of range for these patterns.
    if constexpr (NT == 32) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + G, 0xF, 0xF, true);
    else if constexpr (NT == 8)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, G | (G << 2) | (G << 4) | (G << 6), 0xF, 0xF, true);
    else if constexpr (NT == 4)
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, G | (G << 2) | ((G + 2) << 4) | ((G + 2) << 6), 0xF,
                                                     0xF, true);
    else return v;
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// FP32 input doubles the registers of the load pipeline, so its kernels are
// built for 8 waves per workgroup (the same bytes in flight as 16 FP16 waves).
template <typename AT>
constexpr int kMaxThreads = sizeof(AT) == 4 ? 512 : 1024;
// Single-call kernels: eight blocks per workgroup, or the two scalar loads per
// column pair of unaligned input, need more than the 128 registers a
// 1024-thread workgroup leaves each lane, so they run at most 8 waves.
template <typename AT, int BG, bool VEC>
constexpr int kApplyThreads = (BG >= 8 || !VEC) ? 512 : kMaxThreads<AT>;
// The persistent kernel keeps the 128-register budget of 1024 threads: its
// work items are small, and several workgroups per CU (more waves in flight)
// measured faster than 8 waves with 256 registers (4.33 against 3.60 ms for
// 512 sketches), even though the two inlined work items spill a few values.
constexpr int kBatchThreads = 1024;

// Fixed-point LDS partials.
//
// LDS floating-point atomics run at about 1/25 of the rate of 64-bit integer
// atomics on this GPU (ds_add_f32 and ds_pk_add_f16 take about 190 clocks per
// wave instruction, ds_add_u64 about 8), so each unit is accumulated exactly
// in integer fixed point.  Column c of a work item has its own exponent E_c:
// a contribution x with |x| < 2^(E_c+1) becomes q = rne(x * 2^S_c),
// S_c = 19 - h - E_c, |q| <= 2^(20-h), and is added as the offset-binary
// field B + sigma*q (B = 2^(21-h)) into one 32-bit half of a 64-bit LDS word;
// the two columns of a lane's pair share one ds_add_u64.  The conversion is a
// single FMA, y = x * 2^S_c + 2^23 + B, whose low 23 bits are B + q; XOR with
// 0x4B000000 (sign +) or 0x4B000000 | (2B - 1) (sign -) turns y's bits into
// the field value, the negative case being B - q - 1.  A per-bucket-row
// counter (64 bits) holds the number K of contributions (low 32 bits) and of
// negative ones N (high 32 bits), so the field sum F decodes exactly to
// sum(sigma*q) = F - K*B + N as long as no field exceeds 2^32 (K < 2^(10+h);
// the count headroom h starts at initial_headroom(rows of the unit, W) and
// grows if a bucket row takes 2^(10+h) or more contributions in the unit;
// beyond h = 16 the unit takes the float path).
//
// E_c comes from a sample, the first 64-row tile of every wave: each lane's
// largest |x| in the column over its 16 rows of that tile, and
// E_c = binade(4th largest of those lane maxima) + 2.  A contribution with
// |x| >= 2^(E_c+1) (an outlier: a few rows far above the rest of their
// column, such as identity rows stacked on a small dense block) adds zero to
// the field and is appended instead, as (LDS entry, sign * x), to a list in
// LDS; the list is added to the decoded FP32 partial before the flush.  If the
// list overflows, the unit is recomputed with E_c = binade of the column's
// true maximum (then no contribution is an outlier); if a bucket row breaks
// the K bound, with a larger h.  Non-finite input falls back to FP32 LDS
// atomics.
constexpr uint32_t kMagicBits = 0x4B000000u;   // bit pattern of 2^23
constexpr int kListCap = 1024;                 // outlier records per work item
constexpr int kSampleRank = 4;                 // rank of the lane maximum that sets E_c
constexpr int kHeadroom = 2;                   // binades of E_c above that lane maximum
constexpr int kMaxHeadroom = 16;               // largest count headroom h (K < 2^26)

// Count headroom a unit starts with: with a = ceil(rows / W), the average
// count of a bucket row, the smallest h with 3a/2 + 64 < 2^(10 + h), at most
// kMaxHeadroom.  Starting from h = 0 would recompute every unit whose
// average alone reaches 1024 (8 bucket rows per block with 16384-row units:
// each unit streamed twice).  The bound leaves the usual shapes at h = 0
// (256 bucket rows, 32768-row units: 256 < 1024).
__host__ __device__ constexpr int initial_headroom(int64_t rows, uint32_t W)
{
    const int64_t a = (rows + (int64_t)W - 1) / (int64_t)W;
    int h = 0;
    while (h < kMaxHeadroom && 3 * a / 2 + 64 >= ((int64_t)1 << (10 + h))) ++h;
    return h;
}
constexpr int kCtlWords = 8 + 2 * kNT;         // control words, per-column S, per-column maximum
constexpr int kAuxWords = 2 * kListCap;        // the outlier list; before the pass, the sample
static_assert(kAuxWords >= 16 * 4 * kNT, "the sample of 16 waves must fit the list area");

template <int BG, int NT>
__device__ __forceinline__ uint32_t lds_row_fixed(uint32_t lb, uint32_t o, uint32_t W)
{
    // 64-bit words: no one-word shift; with two 32-lane passes per wave
    // instruction, slots 0/1 and 2/3 update blocks of opposite parity.
    return NT != kNT ? (lb * W + o) * NT
           : BG == 1 ? o * kNT : (lb >> 1) * (W * 64u + 64u) + o * 64u + 32u * (lb & 1u);
}

// Largest |x| of each column of one lane's pair, as sign-cleared bit patterns
// in the element format (monotone in |x|; infinities and NaNs compare above
// every finite value).  FP32: one word per column; 16-bit types: the two
// 16-bit magnitudes packed in one word.
template <typename AT> struct MagOf { typedef uint32_t type; };
template <> struct MagOf<float> { typedef uint2 type; };

__device__ __forceinline__ uint2 pair_mag(const PairRaw<float>& r, uint2 m)
{
    return make_uint2(max(m.x, __float_as_uint(r.v.x) & 0x7FFFFFFFu), max(m.y, __float_as_uint(r.v.y) & 0x7FFFFFFFu));
}
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
template <typename AT>
__device__ __forceinline__ uint32_t pair_mag(const PairRaw<AT>& r, uint32_t m)
{
    // per-half 16-bit maximum of the magnitudes (v_pk_max_u16)
    const u16x2 a = __builtin_bit_cast(u16x2, r.v & 0x7FFF7FFFu);
    const u16x2 b = __builtin_bit_cast(u16x2, m);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(a, b));
}
template <>
__device__ __forceinline__ uint32_t pair_mag<__half>(const PairRaw<__half>& r, uint32_t m)
{
    // FP16: m = maximum3(m, x, -x) per half, one instruction; the IEEE maximum
    // propagates NaN, so non-finite input still shows up as >= 0x7C00.
    uint32_t out;
    asm volatile("v_pk_maximum3_f16 %0, %1, %2, %2 neg_lo:[0,0,1] neg_hi:[0,0,1]"
                 : "=v"(out) : "v"(m), "v"(r.v));
    return out;
}
__device__ __forceinline__ uint2 mag_max(uint2 a, uint2 b) { return make_uint2(max(a.x, b.x), max(a.y, b.y)); }
__device__ __forceinline__ uint32_t mag_max(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}
// true if either column's magnitude reaches its threshold
__device__ __forceinline__ bool mag_reaches(uint2 m, uint2 t) { return m.x >= t.x || m.y >= t.y; }
__device__ __forceinline__ bool mag_reaches(uint32_t m, uint32_t t)
{
    return (m & 0xFFFFu) >= (t & 0xFFFFu) || (m >> 16) >= (t >> 16);
}

// The two columns' magnitudes as FP32 magnitude bits.
template <typename AT>
__device__ __forceinline__ void mag_cols(uint32_t m, uint32_t& a, uint32_t& b)
{
    if constexpr (std::is_same<AT, __hip_bfloat16>::value) {
        a = (m & 0xFFFFu) << 16;
        b = m & 0xFFFF0000u;
    } else {
        a = __float_as_uint(__half2float(__ushort_as_half((unsigned short)(m & 0xFFFFu))));
        b = __float_as_uint(__half2float(__ushort_as_half((unsigned short)(m >> 16))));
    }
}
template <typename AT>
__device__ __forceinline__ void mag_cols(uint2 m, uint32_t& a, uint32_t& b)
{
    a = m.x;
    b = m.y;
}

// floor(log2 v) of a finite FP32 magnitude given as bits (subnormals exact);
// -1000 for zero, 128 for infinities and NaNs.
__device__ __forceinline__ int binade_exact(uint32_t b)
{
    if (b == 0) return -1000;
    const int e = (int)(b >> 23);
    if (e) return e - 127;
    return (31 - __clz((int)b)) - 149;
}

// Magnitude bits, in the element format, of 2^e (e clamped to the format's
// range: beyond the largest finite value every finite magnitude is below it,
// below the smallest subnormal every nonzero magnitude reaches it).
template <typename AT>
__device__ __forceinline__ uint32_t pow2_bits(int e)
{
    if constexpr (sizeof(AT) == 4) {
        if (e > 127) return 0x7F800000u;
        if (e < -149) return 1u;
        if (e < -126) return 1u << (e + 149);
        return (uint32_t)(e + 127) << 23;
    } else if constexpr (std::is_same<AT, __hip_bfloat16>::value) {
        if (e > 127) return 0x7F80u;
        if (e < -133) return 1u;
        if (e < -126) return 1u << (e + 133);
        return (uint32_t)(e + 127) << 7;
    } else {
        if (e > 15) return 0x7C00u;
        if (e < -24) return 1u;
        if (e < -14) return 1u << (e + 24);
        return (uint32_t)(e + 15) << 10;
    }
}

// Per-lane fixed-point parameters of one attempt.
template <typename AT>
struct Fixed {
    float slo, shi;                   // 2^S of the lane's two columns
    typename MagOf<AT>::type thr;     // outlier thresholds 2^(E+1), element format
    float magic;                      // 2^23 + B
    uint32_t xneg;                    // 0x4B000000 | (2B - 1)
    uint32_t B;
    int Slo, Shi;
};

__device__ __forceinline__ int clamp_exponent(int E, int h)
{
    // keeps S = 19 - h - E a normal FP32 exponent
    return max(min(E, 145 - h), -108 - h);
}

template <typename AT>
__device__ __forceinline__ Fixed<AT> fixed_params(int Elo, int Ehi, int h)
{
    Fixed<AT> f;
    Elo = clamp_exponent(Elo, h);
    Ehi = clamp_exponent(Ehi, h);
    f.Slo = 19 - h - Elo;
    f.Shi = 19 - h - Ehi;
    f.slo = __uint_as_float((uint32_t)(f.Slo + 127) << 23);
    f.shi = __uint_as_float((uint32_t)(f.Shi + 127) << 23);
    if constexpr (sizeof(AT) == 4) f.thr = make_uint2(pow2_bits<AT>(Elo + 1), pow2_bits<AT>(Ehi + 1));
    else f.thr = pow2_bits<AT>(Elo + 1) | (pow2_bits<AT>(Ehi + 1) << 16);
    f.B = 1u << (21 - h);
    f.magic = 8388608.0f + (float)f.B;
    f.xneg = kMagicBits | (2u * f.B - 1u);
    return f;
}

// Whether each element of a pair is an outlier (magnitude bits >= threshold).
__device__ __forceinline__ void elem_out(const PairRaw<float>& r, uint2 t, bool& olo, bool& ohi)
{
    olo = (__float_as_uint(r.v.x) & 0x7FFFFFFFu) >= t.x;
    ohi = (__float_as_uint(r.v.y) & 0x7FFFFFFFu) >= t.y;
}
template <typename AT>
__device__ __forceinline__ void elem_out(const PairRaw<AT>& r, uint32_t t, bool& olo, bool& ohi)
{
    olo = (r.v & 0x7FFFu) >= (t & 0xFFFFu);
    ohi = ((r.v >> 16) & 0x7FFFu) >= (t >> 16);
}

// Replace the flagged elements of a pair by +0.
__device__ __forceinline__ void zero_halves(PairRaw<float>& r, bool lo, bool hi)
{
    if (lo) r.v.x = 0.0f;
    if (hi) r.v.y = 0.0f;
}
template <typename AT>
__device__ __forceinline__ void zero_halves(PairRaw<AT>& r, bool lo, bool hi)
{
    r.v &= (lo ? 0xFFFF0000u : 0xFFFFFFFFu) & (hi ? 0x0000FFFFu : 0xFFFFFFFFu);
}

// ACC: 0 = FP32 LDS atomics, 1 = one fixed-point field per element (FP16
// modes), 2 = two fields per element (FP32 mode): the rounded value and its
// residual at 2^-21 finer resolution, kept in two LDS arrays with the same
// layout, so each unit is summed with about 41 significant bits below
// 2^(E_c+1).
// Maximum of v over the wave, in every lane: DPP shifts within each row of 16
// lanes (lanes shifted in from outside the row read 0, the identity), then
// row broadcasts carry the row maxima up to lane 63.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// One work item: the partial sketch of unit `unit` (rows [unit * chunk_rows,
// ...)), column tile `ct` and block group `bgi`, accumulated in LDS and added
// into SA.  Called by every thread of the workgroup; ends with LDS free.
template <typename AT, int BG, bool VEC, int ACC, int NT>
__device__ __forceinline__ void apply_item(const ApplyArgs& p, int unit, int ct, int bgi, float* lds)
{
    typedef typename MagOf<AT>::type Mag;
    constexpr int LL = Geom<NT>::L, KK = Geom<NT>::K, GG = Geom<NT>::G;
    const int nwaves = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // uniform: tile arithmetic stays scalar
    const int lane = (int)(threadIdx.x & 63);
    const int64_t r_begin = (int64_t)unit * p.chunk_rows;
    const int64_t r_end = min(r_begin + (int64_t)p.chunk_rows, p.rows);
    const int c0 = ct * NT;
    const uint32_t j0 = (uint32_t)bgi * BG;
    const uint32_t W = p.W;
    const size_t nw = lds_words<BG, NT>(W);
    const size_t narr = (ACC == 2) ? 2 : 1;       // fixed-point arrays
    uint64_t* cnt = (uint64_t*)((uint32_t*)lds + narr * nw);   // per bucket row, K | N << 32
    uint32_t* ctl = (uint32_t*)(cnt + (size_t)BG * W);         // [0] outliers, [1] non-finite, [2] max K
    int* colS = (int*)ctl + 8;                    // per column: E (sample), then S
    uint32_t* colmax = ctl + 8 + kNT;             // per column: largest |x| (FP32 bits)
    uint32_t* aux = ctl + kCtlWords;              // sample, then outlier list
    const uint32_t lo_off = (uint32_t)(nw * 4);   // byte offset of the residual array

    const int k = lane / LL;                 // row slot within a wave instruction
    const int q = lane % LL;                 // column pair within the tile
    const int col = c0 + 2 * q;
    // Lanes past the last column read columns 0 and 1 of their row; what they
    // add lands in LDS columns >= n, which are never flushed.
    const int colc = (col < p.n) ? col : 0;
    const uint32_t d1 = (colc + 1 < p.n) ? 1u : 0u;
    const bool live_lo = col < p.n, live_hi = col + 1 < p.n;
    const uint32_t laneoff = (uint32_t)(2 * q) * 4u;
    const int64_t span = r_end - r_begin;
    const int64_t ntiles = span > 0 ? (span + kTile - 1) / kTile : 0;

    // One buffer resource per workgroup covering its unit (the planner keeps a
    // unit below 2 GiB); vector offset = the lane's row and column, scalar
    // offset = the row group within the tile.
    constexpr uint32_t esz = (uint32_t)sizeof(AT);
    const AT* ubase = (const AT*)p.A + r_begin * p.lda;
    const uint32_t nrec = (uint32_t)(span > 0 ? span * p.lda * (int64_t)esz : 0);
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)ubase, (short)0, (int)nrec, 0x00020000);
    const uint32_t lane_vo = ((uint32_t)k * (uint32_t)p.lda + (uint32_t)colc) * esz;
    const uint32_t gstep = (uint32_t)KK * (uint32_t)p.lda * esz;
    const uint32_t tstep = (uint32_t)kTile * (uint32_t)p.lda * esz;

    // Clears the partial (and, with the fixed-point arrays, the counters and
    // control words).
    auto zero_lds = [&](bool with_counters) {
        const uint32_t base = (uint32_t)(with_counters ? narr * nw : nw);
        const uint32_t words = base + (with_counters ? 2u * (uint32_t)BG * W + (uint32_t)kCtlWords : 0u);
        float4* l4 = (float4*)lds;
        for (uint32_t e = threadIdx.x; e < base / 4; e += blockDim.x) l4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (uint32_t e = base + threadIdx.x; e < words; e += blockDim.x) lds[e] = 0.f;
    };

    auto load_tile = [&](PairRaw<AT> (&buf)[GG], int64_t tile) {
        const uint32_t vo = lane_vo + (uint32_t)tile * tstep;
#pragma unroll
        for (int g = 0; g < GG; ++g) buf[g] = load_pair<VEC, AT>(rsrc, vo, (uint32_t)g * gstep, d1);
    };

    auto tile_mag = [&](const PairRaw<AT> (&buf)[GG]) {
        Mag m{};
#pragma unroll
        for (int g = 0; g < GG; ++g) m = pair_mag(buf[g], m);
        return m;
    };

    // Lane (k, q) hashes row K q + k of the tile and keeps, for instruction jj,
    // the LDS byte offset and the sign word of local block (jj + k) mod BG.
    // Float path: sign word = sign-bit mask.  Fixed path: the XOR word, and the
    // row's contribution is counted per bucket row.
    auto hash_tile = [&](uint32_t (&hoff)[BG], uint32_t (&hsgn)[BG], int64_t tile, bool fixed,
                         uint32_t xneg) {
        const uint64_t grow = (uint64_t)(p.row_offset + r_begin + tile * kTile + KK * q + k);
        uint4 w4a = row_words(grow, j0 >> 2, p.k0, p.k1);
        uint4 w4b = w4a;
        if (BG == 8 || (BG > 1 && ((j0 & 3u) + BG > 4u))) w4b = row_words(grow, (j0 >> 2) + 1u, p.k0, p.k1);
        if (fixed) {
#pragma unroll
            for (int lb = 0; lb < BG; ++lb) {
                const uint32_t wi = (j0 & 3u) + (uint32_t)lb;
                const uint32_t w = (wi < 4u) ? word_of(w4a, wi) : word_of(w4b, wi - 4u);
                __hip_atomic_fetch_add(&cnt[(uint32_t)lb * W + bucket_in_block(w, W)],
                                       (uint64_t)1u + ((uint64_t)(w & 1u) << 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int jj = 0; jj < BG; ++jj) {
            const uint32_t lb = (uint32_t)(jj + k) & (uint32_t)(BG - 1);
            const uint32_t wi = (j0 & 3u) + lb;            // word index from the first call
            const uint32_t w = (wi < 4u) ? word_of(w4a, wi) : word_of(w4b, wi - 4u);
            const uint32_t o = bucket_in_block(w, W);
            if (fixed) {
                hoff[jj] = lds_row_fixed<BG, NT>(lb, o, W) * 4u;
                hsgn[jj] = (w & 1u) ? xneg : kMagicBits;
            } else {
                hoff[jj] = lds_row<BG, NT>(lb, o, W) * 4u;
                hsgn[jj] = w << 31;
            }
        }
    };

    auto scatter_float = [&](const PairRaw<AT> (&buf)[GG], const uint32_t (&hoff)[BG],
                             const uint32_t (&hsgn)[BG]) {
        static_for<0, GG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            float lo, hi;
            to_f32(buf[g], lo, hi);
#pragma unroll
            for (int jj = 0; jj < BG; ++jj) {
                const uint32_t off = bcast_slot<NT, g>(hoff[jj]) + laneoff;
                const uint32_t sg = bcast_slot<NT, g>(hsgn[jj]);
                float* dst = (float*)__builtin_assume_aligned((char*)lds + off, 4);
                __hip_atomic_fetch_add(dst, __uint_as_float(__float_as_uint(lo) ^ sg),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(dst + 1, __uint_as_float(__float_as_uint(hi) ^ sg),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        });
    };

    // Appends an outlier record: word index of the entry in array 0, signed value.
    auto push_outlier = [&](uint32_t word, float v) {
        const uint32_t i = __hip_atomic_fetch_add(&ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (i < (uint32_t)kListCap) {
            aux[2 * i] = word;
            aux[2 * i + 1] = __float_as_uint(v);
        }
    };

    // Fixed-point scatter of one tile.  ACC == 1: y = x*2^S + (2^23 + B) is the
    // field.  ACC == 2: y rounds x*2^S to an integer Q = y - 2^23 - B, the FMA
    // x*2^S - Q is the exact residual (|r| <= 1/2), and z = r*2^21 + (2^23 + B)
    // is its field in the second array.
    auto scatter_fixed = [&](const PairRaw<AT> (&buf)[GG], const uint32_t (&hoff)[BG],
                             const uint32_t (&hsgn)[BG], const Fixed<AT>& fx) {
        static_for<0, GG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            float lo, hi;
            to_f32(buf[g], lo, hi);
            const float ylo = __builtin_fmaf(lo, fx.slo, fx.magic);
            const float yhi = __builtin_fmaf(hi, fx.shi, fx.magic);
            uint32_t zlo = 0, zhi = 0;
            if constexpr (ACC == 2) {
                const float rlo = __builtin_fmaf(lo, fx.slo, -(ylo - fx.magic));
                const float rhi = __builtin_fmaf(hi, fx.shi, -(yhi - fx.magic));
                zlo = __float_as_uint(__builtin_fmaf(rlo, 2097152.0f, fx.magic));
                zhi = __float_as_uint(__builtin_fmaf(rhi, 2097152.0f, fx.magic));
            }
            const uint32_t alo = __float_as_uint(ylo), ahi = __float_as_uint(yhi);
#pragma unroll
            for (int jj = 0; jj < BG; ++jj) {
                const uint32_t off = bcast_slot<NT, g>(hoff[jj]) + laneoff;
                const uint32_t x = bcast_slot<NT, g>(hsgn[jj]);
                const uint64_t v = ((uint64_t)(ahi ^ x) << 32) | (uint64_t)(alo ^ x);
                unsigned long long* dst = (unsigned long long*)__builtin_assume_aligned((char*)lds + off, 8);
                __hip_atomic_fetch_add(dst, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if constexpr (ACC == 2) {
                    const uint64_t w = ((uint64_t)(zhi ^ x) << 32) | (uint64_t)(zlo ^ x);
                    unsigned long long* dst2 =
                        (unsigned long long*)__builtin_assume_aligned((char*)lds + off + lo_off, 8);
                    __hip_atomic_fetch_add(dst2, (unsigned long long)w, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        });
    };

    // A tile in which some lane of the wave holds an outlier: append each
    // outlier (of a live column) to the list, once per block, and replace it
    // by zero in the tile, which then goes through the ordinary scatter.
    auto strip_outliers = [&](PairRaw<AT> (&buf)[GG], const uint32_t (&hoff)[BG], const uint32_t (&hsgn)[BG],
                              const Fixed<AT>& fx) {
        static_for<0, GG>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            bool olo, ohi;
            elem_out(buf[g], fx.thr, olo, ohi);
            if (__builtin_amdgcn_ballot_w64(olo || ohi) != 0) {
                float vlo, vhi;
                to_f32(buf[g], vlo, vhi);
                const bool rlo = olo && live_lo, rhi = ohi && live_hi;
#pragma unroll
                for (int jj = 0; jj < BG; ++jj) {
                    // broadcasts with every lane active, then the per-lane pushes
                    const uint32_t word = (bcast_slot<NT, g>(hoff[jj]) + laneoff) >> 2;
                    const bool neg = bcast_slot<NT, g>(hsgn[jj]) != kMagicBits;
                    if (rlo) push_outlier(word, neg ? -vlo : vlo);
                    if (rhi) push_outlier(word + 1u, neg ? -vhi : vhi);
                }
                zero_halves(buf[g], olo, ohi);
            }
        });
    };

    PairRaw<AT> bufA[GG], bufB[GG];
    uint32_t offA[BG], sgnA[BG], offB[BG], sgnB[BG];

    // One tile: fixed point (outliers stripped first when a lane of the wave
    // holds one) or float atomics.  Returns the lane's column maxima so far.
    auto process = [&](int acc, PairRaw<AT> (&buf)[GG], const uint32_t (&hoff)[BG], const uint32_t (&hsgn)[BG],
                       const Fixed<AT>& fx, Mag mag) {
        if constexpr (ACC != 0) {
            if (acc != 0) {
                const Mag tm = tile_mag(buf);
                if (__builtin_amdgcn_ballot_w64(mag_reaches(tm, fx.thr)) != 0) strip_outliers(buf, hoff, hsgn, fx);
                scatter_fixed(buf, hoff, hsgn, fx);
                return mag_max(mag, tm);
            }
        }
        scatter_float(buf, hoff, hsgn);
        return mag;
    };

    // Stream the unit once; `acc` selects the accumulation.  bufA and bufB
    // hold the wave's first two tiles on entry when `preloaded`.  Returns the
    // lane's column maxima.
    auto run = [&](int acc, bool preloaded, const Fixed<AT>& fx) {
        const bool fixed = acc != 0;
        Mag mag{};
        int64_t tile = wave;
        if (tile < ntiles) {
            if (!preloaded) {
                load_tile(bufA, tile);
                load_tile(bufB, min(tile + nwaves, ntiles));   // tile ntiles lies wholly past the unit
            }
            hash_tile(offA, sgnA, tile, fixed, fx.xneg);
        }
        // Software pipeline: the next tile's loads are in flight while the
        // current tile is scattered; unrolled twice to ping-pong the buffers.
        // Rows past the unit's end load as zero and add nothing.  The tile
        // after next is loaded unconditionally (past the last tile every row
        // is out of the buffer's range and reads zero without touching
        // memory): a load behind a branch would make the compiler wait for it
        // before the next tile's values could be used.
        while (tile < ntiles) {
            int64_t nxt = tile + nwaves;
            mag = process(acc, bufA, offA, sgnA, fx, mag);
            if (nxt >= ntiles) break;
            load_tile(bufA, min(nxt + nwaves, ntiles));
            hash_tile(offB, sgnB, nxt, fixed, fx.xneg);
            tile = nxt;
            nxt = tile + nwaves;
            mag = process(acc, bufB, offB, sgnB, fx, mag);
            if (nxt >= ntiles) break;
            load_tile(bufB, min(nxt + nwaves, ntiles));
            hash_tile(offA, sgnA, nxt, fixed, fx.xneg);
            tile = nxt;
        }
        return mag;
    };

    auto wave_max = [&](uint32_t v) { return wave_max_u32(v); };

    bool fixed_ok = false;
    uint32_t nout = 0;            // outlier records to add before the flush
    uint32_t Bfix = 0;
    Fixed<AT> fx = fixed_params<AT>(0, 0, 0);
    if constexpr (ACC != 0) {
        // The sample: every lane's column maxima over its rows of the wave's
        // first tile, column-major with Ls = K * nwaves values per column.
        // The wave's second tile is requested with the first, so the memory
        // stays busy while the exponents are chosen.
        const int Ls = KK * nwaves;
        Mag m0{};
        if (wave < ntiles) {
            load_tile(bufA, wave);
            load_tile(bufB, min((int64_t)wave + nwaves, ntiles));
        }
        zero_lds(true);
        if (wave < ntiles) m0 = tile_mag(bufA);
        {
            uint32_t a0, a1;
            mag_cols<AT>(m0, a0, a1);
            aux[(2 * q) * Ls + wave * KK + k] = a0;
            aux[(2 * q + 1) * Ls + wave * KK + k] = a1;
        }
        __syncthreads();
        // The kSampleRank-th largest lane maximum of each column (with
        // multiplicity): wave w takes columns w, w + nwaves, ...; each lane
        // keeps the largest kSampleRank values of its share in order, then
        // kSampleRank rounds each take the wave's maximum and drop one
        // instance of it (from the lowest lane holding it).
        for (int c = wave; c < NT; c += nwaves) {
            uint32_t t[kSampleRank] = {};
            for (int i = lane; i < Ls; i += 64) {
                uint32_t v = aux[c * Ls + i];
#pragma unroll
                for (int r = 0; r < kSampleRank; ++r) {
                    const uint32_t a = max(t[r], v);
                    v = min(t[r], v);
                    t[r] = a;
                }
            }
            uint32_t top = 0;
            for (int r = 0; r < kSampleRank; ++r) {
                top = wave_max(t[0]);
                const uint64_t holders = __builtin_amdgcn_ballot_w64(t[0] == top);
                if (lane == (int)__builtin_ctzll(holders)) {
#pragma unroll
                    for (int i = 0; i + 1 < kSampleRank; ++i) t[i] = t[i + 1];
                    t[kSampleRank - 1] = 0;
                }
            }
            if (lane == 0) colS[c] = binade_exact(top) + kHeadroom;
        }
        __syncthreads();
        int Elo = colS[2 * q], Ehi = colS[2 * q + 1];
        int h = initial_headroom(span, W);
        for (int attempt = 0; attempt < 2 && !fixed_ok; ++attempt) {
            if (attempt > 0) {
                zero_lds(true);
                __syncthreads();
            }
            fx = fixed_params<AT>(Elo, Ehi, h);
            const Mag m = run(ACC, attempt == 0, fx);
            uint32_t a0, a1;
            mag_cols<AT>(m, a0, a1);
            if (a0 >= 0x7F800000u || a1 >= 0x7F800000u) ctl[1] = 1u;
            if (live_lo) atomicMax(&colmax[2 * q], a0);
            if (live_hi) atomicMax(&colmax[2 * q + 1], a1);
            uint32_t kmax = 0;
            __syncthreads();
            for (uint32_t e = threadIdx.x; e < (uint32_t)BG * W; e += blockDim.x) kmax = max(kmax, (uint32_t)cnt[e]);
            kmax = wave_max(kmax);
            if (lane == 0) atomicMax(&ctl[2], kmax);
            __syncthreads();
            const uint32_t kall = ctl[2];
            nout = ctl[0];
            if (ctl[1]) break;                                  // non-finite input
            fixed_ok = (uint64_t)kall < (1ull << (10 + h)) && nout <= (uint32_t)kListCap;
            if (!fixed_ok) {
                if (nout > (uint32_t)kListCap) {
                    // no outliers at the columns' true maxima
                    Elo = binade_exact(colmax[2 * q]);
                    Ehi = binade_exact(colmax[2 * q + 1]);
                }
                while (h <= kMaxHeadroom && (uint64_t)kall >= (1ull << (10 + h))) ++h;
                if (h > kMaxHeadroom) break;                   // too many rows in one bucket row
            }
            __syncthreads();
        }
        if (fixed_ok) {
            Bfix = fx.B;
            if (wave == 0 && k == 0) {
                colS[2 * q] = fx.Slo;
                colS[2 * q + 1] = fx.Shi;
            }
        } else {
            zero_lds(false);
            __syncthreads();
            run(0, false, fx);
        }
    } else {
        zero_lds(false);
        __syncthreads();
        run(0, false, fx);
    }
    __syncthreads();

    // Each thread keeps one column pair of the tile (cp) and walks bucket rows
    // o0, o0 + ostep, ... of every local block.
    constexpr uint32_t NP = NT / 2;
    const uint32_t cp = threadIdx.x % NP;
    const uint32_t o0 = threadIdx.x / NP, ostep = blockDim.x / NP;
    const int cpair = c0 + 2 * (int)cp;                     // first column of the pair in A
    int S0 = 0, S1 = 0;
    uint32_t bsh = 0;                                        // B = 2^bsh
    if (fixed_ok) {
        S0 = colS[2 * cp];
        S1 = colS[2 * cp + 1];
        bsh = (uint32_t)__builtin_ctz(Bfix);
    }
    // body(lb, o, b): bucket row o of local block lb, b = its row of SA.
    auto for_rows = [&](auto&& body) {
        for (uint32_t lb = 0; lb < (uint32_t)BG; ++lb) {
            int64_t b = (int64_t)(j0 + lb) * W + o0;
#pragma unroll 4
            for (uint32_t o = o0; o < W; o += ostep, b += ostep) body(lb, o, b);
        }
    };

    // The unit's exact fixed-point sums of the pair's two entries in bucket row
    // (lb, o), each rounded once to FP32.  F - K*B + N is evaluated modulo
    // 2^32: every field sum is below 2^32 and the signed result below 2^30 in
    // magnitude (K < 2^(10+h), |q| <= 2^(20-h)), so the wrapped difference is
    // the exact integer.
    auto decode2 = [&](uint32_t lb, uint32_t o) -> float2 {
        const uint32_t wi = lds_row_fixed<BG, NT>(lb, o, W) + 2u * cp;
        const uint64_t cv = cnt[lb * W + o];
        const uint32_t kb = ((uint32_t)cv << bsh) - (uint32_t)(cv >> 32);
        const uint2 f = *(const uint2*)((const uint32_t*)lds + wi);
        const int32_t a = (int32_t)(f.x - kb), b = (int32_t)(f.y - kb);
        if constexpr (ACC == 2) {
            // value = (a * 2^21 + residual) * 2^-(S + 21); the sum is exact in FP64
            const uint2 g = *(const uint2*)((const uint32_t*)lds + nw + wi);
            const double va = __builtin_fma((double)a, 2097152.0, (double)(int32_t)(g.x - kb));
            const double vb = __builtin_fma((double)b, 2097152.0, (double)(int32_t)(g.y - kb));
            return make_float2((float)ldexp(va, -(S0 + 21)), (float)ldexp(vb, -(S1 + 21)));
        } else {
            return make_float2(ldexpf((float)a, -S0), ldexpf((float)b, -S1));
        }
    };
    if (fixed_ok && nout > 0) {
        // Decode the partial to FP32 in place (array 0), then add the outliers.
        // (each entry is read and rewritten by one thread: no other entry shares its words)
        for_rows([&](uint32_t lb, uint32_t o, int64_t) {
            *(float2*)(lds + lds_row_fixed<BG, NT>(lb, o, W) + 2u * cp) = decode2(lb, o);
        });
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nout; i += blockDim.x)
            __hip_atomic_fetch_add(lds + aux[2 * i], __uint_as_float(aux[2 * i + 1]), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
    }
    // The pair's two entries of the finished partial in bucket row (lb, o).
    // DEC: the fixed-point sums are decoded here (the common case, compiled
    // into branch-free flush loops); otherwise the partial holds FP32 values,
    // decoded in place (fixed layout) or from the float path (whose rows may
    // start at an odd word).
    auto entry2 = [&](auto dec_c, uint32_t lb, uint32_t o) -> float2 {
        if constexpr (decltype(dec_c)::value) {
            return decode2(lb, o);
        } else {
            if (fixed_ok) return *(const float2*)(lds + lds_row_fixed<BG, NT>(lb, o, W) + 2u * cp);
            const float* e = lds + lds_row<BG, NT>(lb, o, W) + 2u * cp;
            return make_float2(e[0], e[1]);
        }
    };
    const bool dec = fixed_ok && nout == 0;

    // ---- flush the partial into SA -----------------------------------------
    if (cpair >= p.n) return;
    const bool has1 = cpair + 1 < p.n;
    const int64_t r0g = p.row_offset + r_begin;             // first global row of the unit
    if (p.mode == 0) {
        float* SA = (float*)p.SA;
        auto flush32 = [&](auto dec_c) {
            for_rows([&](uint32_t lb, uint32_t o, int64_t b) {
                const float2 v = entry2(dec_c, lb, o);
                float* dst = SA + b * p.ldsa + cpair;
                unsafeAtomicAdd(dst, v.x * p.scale);
                if (has1) unsafeAtomicAdd(dst + 1, v.y * p.scale);
            });
        };
        if (dec) flush32(std::true_type{});
        else flush32(std::false_type{});
    } else {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        uint16_t* SA = (uint16_t*)p.SA;
        const uint64_t site0 = (uint64_t)r0g * ((uint64_t)p.d * (uint64_t)p.n) + (uint64_t)cpair;
        // MODE: the rounding rule, fixed per loop in the common case so the
        // body has no branches (0: taken from p.mode at run time)
        auto flush16 = [&](auto mode_c, auto dec_c) {
            constexpr int MODE = decltype(mode_c)::value;
            const int mode = MODE ? MODE : p.mode;
            for_rows([&](uint32_t lb, uint32_t o, int64_t b) {
                const float2 v = entry2(dec_c, lb, o);
                uint32_t u0 = 0, u1 = 0;
                if (MODE == 0 ? mode >= 2 : MODE >= 2)
                    round_bits2(site0 + (uint64_t)b * (uint64_t)p.n, p.epoch, p.k0, p.k1, u0, u1);
                // the scaled value is rounded to FP32 before its rounding to
                // FP16 (the opaque copy keeps the two roundings apart)
                const uint16_t h0 = quantize(mode, as_fp32(v.x * p.scale), u0);
                // -0.0 leaves the neighbouring half unchanged (x + -0 == x for every x)
                const uint16_t h1 = has1 ? quantize(mode, as_fp32(v.y * p.scale), u1) : (uint16_t)0x8000u;
                const uint32_t packed = (uint32_t)h0 | ((uint32_t)h1 << 16);
                h2 hv = __builtin_bit_cast(h2, packed);
                __builtin_amdgcn_global_atomic_fadd_v2f16((h2*)(SA + b * p.ldsa + cpair), hv);
            });
        };
        if (!dec) flush16(std::integral_constant<int, 0>{}, std::false_type{});
        else if (p.mode == 2) flush16(std::integral_constant<int, 2>{}, std::true_type{});
        else if (p.mode == 3) flush16(std::integral_constant<int, 3>{}, std::true_type{});
        else flush16(std::integral_constant<int, 1>{}, std::true_type{});
    }
}

template <typename AT, int BG, bool VEC, int ACC, int NT>
__global__ __launch_bounds__((kApplyThreads<AT, BG, VEC>)) void apply_kernel(ApplyArgs p)
{
    extern __shared__ float lds[];
    const int per_unit = p.col_tiles * p.bgroups;
    int unit, t;
    if (p.xcd_remap) {
        // Consecutive workgroup ids go to different XCDs; give all tiles of a
        // unit the same id modulo 8 so they read the unit's rows through one L2.
        const int x = (int)(blockIdx.x & 7u), sidx = (int)(blockIdx.x >> 3);
        unit = (sidx / per_unit) * 8 + x;
        t = sidx % per_unit;
    } else {
        unit = (int)blockIdx.x / per_unit;
        t = (int)blockIdx.x % per_unit;
    }
    apply_item<AT, BG, VEC, ACC, NT>(p, unit, t % p.col_tiles, t / p.col_tiles, lds);
}

// Persistent form for many problems: each workgroup takes work items from a
// device counter until the batch's items run out.  descs[] is sorted so the
// largest problems' items come first; item0 is a problem's first flat item.
// A problem's column tile is 32 or 8 columns (a.nt).
template <typename AT, int BG, bool VEC, int ACC>
__global__ __launch_bounds__(kBatchThreads) void apply_batched_kernel(const BatchDesc* descs, int32_t count,
                                                                         int64_t total_items, uint32_t* counter)
{
    extern __shared__ float lds[];
    __shared__ int64_t s_item;
    __shared__ int32_t s_prob;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t it = (int64_t)atomicAdd(counter, 1u);
            int lo = 0, hi = count - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (descs[mid].item0 <= it) lo = mid;
                else hi = mid - 1;
            }
            s_item = it;
            s_prob = lo;
        }
        __syncthreads();
        const int64_t it = s_item;
        const int pi = __builtin_amdgcn_readfirstlane(s_prob);
        if (it >= total_items) break;
        const BatchDesc* bd = descs + pi;
        const int local = __builtin_amdgcn_readfirstlane((int)(it - bd->item0));
        const int per_unit = bd->a.col_tiles * bd->a.bgroups;
        const int t = local % per_unit;
        if (bd->a.nt == 8)
            apply_item<AT, BG, VEC, ACC, 8>(bd->a, local / per_unit, t % bd->a.col_tiles, t / bd->a.col_tiles, lds);
        else
            apply_item<AT, BG, VEC, ACC, kNT>(bd->a, local / per_unit, t % bd->a.col_tiles, t / bd->a.col_tiles,
                                              lds);
        __syncthreads();
    }
}

template <typename AT, int BG, bool VEC, int ACC, int NT>
hipError_t launch_kernel(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    static size_t attr_bytes = 0;
    auto kern = apply_kernel<AT, BG, VEC, ACC, NT>;
    if (plan.lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)plan.lds_bytes);
        if (e != hipSuccess) return e;
        attr_bytes = plan.lds_bytes;
    }
    const int64_t grid = plan.units * (int64_t)plan.col_tiles * plan.bgroups;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((unsigned)(64 * plan.waves)), plan.lds_bytes, st, a);
    return hipGetLastError();
}

template <typename AT, int BG, bool VEC, int NT>
hipError_t launch_typed(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    return a.mode == 0 ? launch_kernel<AT, BG, VEC, 2, NT>(plan, a, st)
                       : launch_kernel<AT, BG, VEC, 1, NT>(plan, a, st);
}

// (column tile, block group) pairs with kernels: 32 x {1,2,4,8}, 8 x {1,2,4},
// 4 x {1,2}, 2 x {1} (narrow tiles serve large d/s, where few blocks fit).
template <typename AT, bool VEC>
hipError_t launch_bg(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    switch (plan.nt * 16 + plan.bg) {
    case 32 * 16 + 1: return launch_typed<AT, 1, VEC, 32>(plan, a, st);
    case 32 * 16 + 2: return launch_typed<AT, 2, VEC, 32>(plan, a, st);
    case 32 * 16 + 4: return launch_typed<AT, 4, VEC, 32>(plan, a, st);
    case 32 * 16 + 8: return launch_typed<AT, 8, VEC, 32>(plan, a, st);
    case 8 * 16 + 1: return launch_typed<AT, 1, VEC, 8>(plan, a, st);
    case 8 * 16 + 2: return launch_typed<AT, 2, VEC, 8>(plan, a, st);
    case 8 * 16 + 4: return launch_typed<AT, 4, VEC, 8>(plan, a, st);
    case 4 * 16 + 1: return launch_typed<AT, 1, VEC, 4>(plan, a, st);
    case 4 * 16 + 2: return launch_typed<AT, 2, VEC, 4>(plan, a, st);
    case 2 * 16 + 1: return launch_typed<AT, 1, VEC, 2>(plan, a, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename AT>
hipError_t launch_vec(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    return a.aligned ? launch_bg<AT, true>(plan, a, st) : launch_bg<AT, false>(plan, a, st);
}

// grid == 0: only raise the kernel's dynamic-LDS limit (done before a graph capture).
template <typename AT, int BG, bool VEC, int ACC>
hipError_t launch_batched_kernel(const BatchDesc* descs, int32_t count, int64_t total_items, uint32_t* counter,
                                 int grid, int waves, size_t lds_bytes, hipStream_t st)
{
    static size_t attr_bytes = 0;
    auto kern = apply_batched_kernel<AT, BG, VEC, ACC>;
    if (lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds_bytes);
        if (e != hipSuccess) return e;
        attr_bytes = lds_bytes;
    }
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3((unsigned)(64 * waves)), lds_bytes, st, descs, count,
                       total_items, counter);
    return hipGetLastError();
}

template <typename AT, bool VEC, int ACC>
hipError_t batched_bg(int bg, const BatchDesc* descs, int32_t count, int64_t total_items, uint32_t* counter,
                      int grid, int waves, size_t lds_bytes, hipStream_t st)
{
    switch (bg) {
    case 1: return launch_batched_kernel<AT, 1, VEC, ACC>(descs, count, total_items, counter, grid, waves, lds_bytes, st);
    case 2: return launch_batched_kernel<AT, 2, VEC, ACC>(descs, count, total_items, counter, grid, waves, lds_bytes, st);
    case 4: return launch_batched_kernel<AT, 4, VEC, ACC>(descs, count, total_items, counter, grid, waves, lds_bytes, st);
    case 8: return launch_batched_kernel<AT, 8, VEC, ACC>(descs, count, total_items, counter, grid, waves, lds_bytes, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename AT>
hipError_t batched_typed(int bg, bool vec, bool dual, const BatchDesc* descs, int32_t count, int64_t total_items,
                         uint32_t* counter, int grid, int waves, size_t lds_bytes, hipStream_t st)
{
    if (dual)
        return vec ? batched_bg<AT, true, 2>(bg, descs, count, total_items, counter, grid, waves, lds_bytes, st)
                   : batched_bg<AT, false, 2>(bg, descs, count, total_items, counter, grid, waves, lds_bytes, st);
    return vec ? batched_bg<AT, true, 1>(bg, descs, count, total_items, counter, grid, waves, lds_bytes, st)
               : batched_bg<AT, false, 1>(bg, descs, count, total_items, counter, grid, waves, lds_bytes, st);
}

}  // namespace
}  // namespace sk
