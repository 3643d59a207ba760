// sketch_apply kernels for gfx950.
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
#include <type_traits>

#include "sk_device.hpp"
#include "sk_internal.hpp"

namespace sk {
namespace {

constexpr int kNT = 32;     // columns per workgroup tile
constexpr int kTile = 64;   // rows per wave tile
constexpr int kGroups = 16; // wave instructions (4 rows each) per tile

template <int BG>
__host__ __device__ constexpr uint32_t lds_row(uint32_t lb, uint32_t o, uint32_t W)
{
    return BG == 1 ? o * kNT
                   : (lb >> 1) * (W * 64u + 64u) + o * 64u + 32u * (lb & 1u) + ((lb >> 1) & 1u);
}

template <int BG>
__host__ __device__ constexpr size_t lds_words(uint32_t W)
{
    return BG == 1 ? (size_t)W * kNT : (size_t)(BG / 2) * ((size_t)W * 64u + 64u);
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


// row_newbcast:G -- every lane of each 16-lane row takes lane G of that row.
template <int G>
__device__ __forceinline__ uint32_t bcast16(uint32_t v)
{
    // bound_ctrl set and old = 0 let the compiler fold the move into the consumer
    // (v_add_u32_dpp / v_xor_b32_dpp); no lane is out of range for this pattern.
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + G, 0xF, 0xF, true);
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

// Fixed-point LDS partials (the FP16 modes).
//
// LDS floating-point atomics are two orders of magnitude slower than integer
// ones on this GPU, so the FP16 modes accumulate each unit exactly in integer
// fixed point: a contribution x becomes q = round(x * 2^S) with |q| < 2^(20-c)
// and is added as the offset-binary field B + sigma*q (B = 2^(21-c)) into one
// 32-bit half of a 64-bit LDS word; the two columns of a lane's pair share
// one ds_add_u64.  The conversion is a single FMA, y = x * 2^S + 2^23 + B,
// whose low 23 bits are B + q; XOR with 0x4B000000 (sign +) or
// 0x4B000000 | (2B - 1) (sign -) turns y's bits into the field value, the
// negative case being B - q - 1.  A per-bucket-row counter holds the number
// K of contributions (low 16 bits) and of negative ones N (high 16 bits), so
// the field sum F decodes exactly to sum(sigma*q) = F - K*B + N as long as no
// field exceeds 2^32 (K < 2^(10+c)).  S comes from the largest |x| of the
// first tiles (one binade of headroom); the workgroup tracks the true maximum
// and the largest K and, if either bound was broken, recomputes the unit with
// the exact parameters.  Non-finite input falls back to FP32 LDS atomics.
constexpr uint32_t kMagicBits = 0x4B000000u;   // bit pattern of 2^23

template <int BG>
__device__ __forceinline__ uint32_t lds_row_fixed(uint32_t lb, uint32_t o, uint32_t W)
{
    // 64-bit words: no one-word shift; with two 32-lane passes per wave
    // instruction, slots 0/1 and 2/3 update blocks of opposite parity.
    return BG == 1 ? o * kNT : (lb >> 1) * (W * 64u + 64u) + o * 64u + 32u * (lb & 1u);
}

// Largest |x| of one lane's pair so far, as sign-cleared bit patterns (monotone
// in |x|; infinities and NaNs compare above every finite value).
__device__ __forceinline__ uint32_t pair_mag(const PairRaw<float>& r, uint32_t m)
{
    return max(m, max(__float_as_uint(r.v.x) & 0x7FFFFFFFu, __float_as_uint(r.v.y) & 0x7FFFFFFFu));
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
__device__ __forceinline__ uint32_t mag16_to_f32bits(uint32_t m, bool bf16)
{
    const uint32_t a = max(m & 0xFFFFu, m >> 16);
    if (bf16) return a << 16;
    return __float_as_uint(__half2float(__ushort_as_half((unsigned short)a)));
}

struct FixedParams {
    float scale;      // 2^S
    float magic;      // 2^23 + B
    uint32_t xneg;    // 0x4B000000 | (2B - 1)
    uint32_t B;
    int S;
};

__device__ __forceinline__ FixedParams fixed_params(int E, int c)
{
    FixedParams f;
    int S = 19 - c - E;
    S = S > 127 ? 127 : (S < -126 ? -126 : S);
    f.S = S;
    f.scale = __uint_as_float((uint32_t)(S + 127) << 23);
    f.B = 1u << (21 - c);
    f.magic = 8388608.0f + (float)f.B;
    f.xneg = kMagicBits | (2u * f.B - 1u);
    return f;
}

__device__ __forceinline__ int binade_of(uint32_t magbits)
{
    if (magbits == 0) return 0;
    const int e = (int)((magbits >> 23) & 0xFFu) - 127;
    return e < -126 ? -126 : e;
}

// ACC: 0 = FP32 LDS atomics, 1 = one fixed-point field per element (FP16
// modes), 2 = two fields per element (FP32 mode): the rounded value and its
// residual at 2^-21 finer resolution, kept in two LDS arrays with the same
// layout, so each unit is summed with about 41 significant bits.
// One work item: the partial sketch of unit `unit` (rows [unit * chunk_rows,
// ...)), column tile `ct` and block group `bgi`, accumulated in LDS and added
// into SA.  Called by every thread of the workgroup; ends with LDS free.
template <typename AT, int BG, bool VEC, int ACC>
__device__ __forceinline__ void apply_item(const ApplyArgs& p, int unit, int ct, int bgi, float* lds)
{
    const int nwaves = (int)(blockDim.x >> 6);
    const int wave = (int)(threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    const int64_t r_begin = (int64_t)unit * p.chunk_rows;
    const int64_t r_end = min(r_begin + (int64_t)p.chunk_rows, p.rows);
    const int c0 = ct * kNT;
    const uint32_t j0 = (uint32_t)bgi * BG;
    const uint32_t W = p.W;
    const size_t nw = lds_words<BG>(W);
    const size_t narr = (ACC == 2) ? 2 : 1;       // fixed-point arrays
    uint32_t* cnt = (uint32_t*)lds + narr * nw;   // per bucket row, K | N << 16
    uint32_t* ctl = cnt + (size_t)BG * W;         // [0] first max, [1] max, [2] max K
    const uint32_t lo_off = (uint32_t)(nw * 4);   // byte offset of the residual array

    const int k = lane >> 4;                 // row slot within a wave instruction
    const int q = lane & 15;                 // column pair within the tile
    const int col = c0 + 2 * q;
    // Lanes past the last column read columns 0 and 1 of their row; what they
    // add lands in LDS columns >= n, which are never flushed.
    const int colc = (col < p.n) ? col : 0;
    const uint32_t d1 = (colc + 1 < p.n) ? 1u : 0u;
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
    const uint32_t gstep = 4u * (uint32_t)p.lda * esz;
    const uint32_t tstep = (uint32_t)kTile * (uint32_t)p.lda * esz;

    auto zero_lds = [&](bool with_counters) {
        const size_t base = with_counters ? narr * nw : nw;
        const size_t words = base + (with_counters ? (size_t)BG * W + 4 : 0);
        float4* l4 = (float4*)lds;
        for (size_t e = threadIdx.x; e < base / 4; e += blockDim.x) l4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (size_t e = base + threadIdx.x; e < words; e += blockDim.x) lds[e] = 0.f;
    };

    auto load_tile = [&](PairRaw<AT> (&buf)[kGroups], int64_t tile) {
        const uint32_t vo = lane_vo + (uint32_t)tile * tstep;
#pragma unroll
        for (int g = 0; g < kGroups; ++g) buf[g] = load_pair<VEC, AT>(rsrc, vo, (uint32_t)g * gstep, d1);
    };

    auto tile_mag = [&](const PairRaw<AT> (&buf)[kGroups], uint32_t m) {
#pragma unroll
        for (int g = 0; g < kGroups; ++g) m = pair_mag(buf[g], m);
        return m;
    };

    // Lane (k, q) hashes row 4q + k of the tile and keeps, for instruction jj,
    // the LDS byte offset and the sign word of local block (jj + k) mod BG.
    // Float path: sign word = sign-bit mask.  Fixed path: the XOR word, and the
    // row's contribution is counted per bucket row.
    auto hash_tile = [&](uint32_t (&hoff)[BG], uint32_t (&hsgn)[BG], int64_t tile, bool fixed,
                         uint32_t xneg) {
        const uint64_t grow = (uint64_t)(p.row_offset + r_begin + tile * kTile + 4 * q + k);
        uint4 w4a = row_words(grow, j0 >> 2, p.k0, p.k1);
        uint4 w4b = w4a;
        if (BG == 8 || (BG > 1 && ((j0 & 3u) + BG > 4u))) w4b = row_words(grow, (j0 >> 2) + 1u, p.k0, p.k1);
        if (fixed) {
#pragma unroll
            for (int lb = 0; lb < BG; ++lb) {
                const uint32_t wi = (j0 & 3u) + (uint32_t)lb;
                const uint32_t w = (wi < 4u) ? word_of(w4a, wi) : word_of(w4b, wi - 4u);
                __hip_atomic_fetch_add(&cnt[(uint32_t)lb * W + bucket_in_block(w, W)], 1u + ((w & 1u) << 16),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
#pragma unroll
        for (int jj = 0; jj < BG; ++jj) {
            const uint32_t lb = (uint32_t)(jj + k) & (uint32_t)(BG - 1);
            const uint32_t wi = (j0 & 3u) + lb;            // word index from the first call
            const uint32_t w = (wi < 4u) ? word_of(w4a, wi) : word_of(w4b, wi - 4u);
            const uint32_t o = bucket_in_block(w, W);
            if (fixed) {
                hoff[jj] = lds_row_fixed<BG>(lb, o, W) * 4u;
                hsgn[jj] = (w & 1u) ? xneg : kMagicBits;
            } else {
                hoff[jj] = lds_row<BG>(lb, o, W) * 4u;
                hsgn[jj] = w << 31;
            }
        }
    };

    auto scatter_float = [&](const PairRaw<AT> (&buf)[kGroups], const uint32_t (&hoff)[BG],
                             const uint32_t (&hsgn)[BG]) {
        static_for<0, kGroups>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            float lo, hi;
            to_f32(buf[g], lo, hi);
#pragma unroll
            for (int jj = 0; jj < BG; ++jj) {
                const uint32_t off = bcast16<g>(hoff[jj]) + laneoff;
                const uint32_t sg = bcast16<g>(hsgn[jj]);
                float* dst = (float*)__builtin_assume_aligned((char*)lds + off, 4);
                __hip_atomic_fetch_add(dst, __uint_as_float(__float_as_uint(lo) ^ sg),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(dst + 1, __uint_as_float(__float_as_uint(hi) ^ sg),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        });
    };

    auto scatter_fixed = [&](const PairRaw<AT> (&buf)[kGroups], const uint32_t (&hoff)[BG],
                             const uint32_t (&hsgn)[BG], float scale, float magic) {
        static_for<0, kGroups>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            float lo, hi;
            to_f32(buf[g], lo, hi);
            const uint32_t ylo = __float_as_uint(__builtin_fmaf(lo, scale, magic));
            const uint32_t yhi = __float_as_uint(__builtin_fmaf(hi, scale, magic));
#pragma unroll
            for (int jj = 0; jj < BG; ++jj) {
                const uint32_t off = bcast16<g>(hoff[jj]) + laneoff;
                const uint32_t x = bcast16<g>(hsgn[jj]);
                const uint64_t v = ((uint64_t)(yhi ^ x) << 32) | (uint64_t)(ylo ^ x);
                unsigned long long* dst = (unsigned long long*)__builtin_assume_aligned((char*)lds + off, 8);
                __hip_atomic_fetch_add(dst, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        });
    };

    // Two fields per element: y = x*2^S + (2^23 + B) rounds x*2^S to an integer
    // Q = y - 2^23 - B, the FMA x*2^S - Q is the exact residual (|r| <= 1/2),
    // and z = r*2^21 + (2^23 + B) is its fixed-point form.
    auto scatter_dual = [&](const PairRaw<AT> (&buf)[kGroups], const uint32_t (&hoff)[BG],
                            const uint32_t (&hsgn)[BG], float scale, float magic) {
        static_for<0, kGroups>([&](auto gc) {
            constexpr int g = decltype(gc)::value;
            float lo, hi;
            to_f32(buf[g], lo, hi);
            const float ylo = __builtin_fmaf(lo, scale, magic);
            const float yhi = __builtin_fmaf(hi, scale, magic);
            const float rlo = __builtin_fmaf(lo, scale, -(ylo - magic));
            const float rhi = __builtin_fmaf(hi, scale, -(yhi - magic));
            const uint32_t zlo = __float_as_uint(__builtin_fmaf(rlo, 2097152.0f, magic));
            const uint32_t zhi = __float_as_uint(__builtin_fmaf(rhi, 2097152.0f, magic));
            const uint32_t alo = __float_as_uint(ylo), ahi = __float_as_uint(yhi);
#pragma unroll
            for (int jj = 0; jj < BG; ++jj) {
                const uint32_t off = bcast16<g>(hoff[jj]) + laneoff;
                const uint32_t x = bcast16<g>(hsgn[jj]);
                const uint64_t v = ((uint64_t)(ahi ^ x) << 32) | (uint64_t)(alo ^ x);
                const uint64_t w = ((uint64_t)(zhi ^ x) << 32) | (uint64_t)(zlo ^ x);
                unsigned long long* dst = (unsigned long long*)__builtin_assume_aligned((char*)lds + off, 8);
                unsigned long long* dst2 = (unsigned long long*)__builtin_assume_aligned((char*)lds + off + lo_off, 8);
                __hip_atomic_fetch_add(dst, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_fetch_add(dst2, (unsigned long long)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        });
    };

    PairRaw<AT> bufA[kGroups], bufB[kGroups];
    uint32_t offA[BG], sgnA[BG], offB[BG], sgnB[BG];

    // Stream the unit once; `fixed` selects the accumulation.  bufA holds the
    // wave's first tile on entry when `preloaded`.  Returns the lane's largest
    // input magnitude bits.
    auto run = [&](int acc, bool preloaded, const FixedParams& fp) {
        const bool fixed = acc != 0;
        uint32_t mag = 0;
        int64_t tile = wave;
        if (tile < ntiles) {
            if (!preloaded) load_tile(bufA, tile);
            hash_tile(offA, sgnA, tile, fixed, fp.xneg);
        }
        // Software pipeline: the next tile's loads are in flight while the
        // current tile is scattered; unrolled twice to ping-pong the buffers.
        // Rows past the unit's end load as zero and add nothing.  The next
        // tile is loaded unconditionally (past the last tile every row is out
        // of the buffer's range and reads zero without touching memory): a
        // load behind a branch would make the compiler wait for it before
        // the current tile's values could be used.
        while (tile < ntiles) {
            int64_t nxt = tile + nwaves;
            load_tile(bufB, min(nxt, ntiles));     // tile ntiles lies wholly past the unit
            if (acc == 2) {
                if constexpr (ACC == 2) {
                    mag = tile_mag(bufA, mag);
                    scatter_dual(bufA, offA, sgnA, fp.scale, fp.magic);
                }
            } else if (acc == 1) {
                if constexpr (ACC == 1) {
                    mag = tile_mag(bufA, mag);
                    scatter_fixed(bufA, offA, sgnA, fp.scale, fp.magic);
                }
            } else {
                scatter_float(bufA, offA, sgnA);
            }
            if (nxt >= ntiles) break;
            hash_tile(offB, sgnB, nxt, fixed, fp.xneg);
            tile = nxt;
            nxt = tile + nwaves;
            load_tile(bufA, min(nxt, ntiles));
            if (acc == 2) {
                if constexpr (ACC == 2) {
                    mag = tile_mag(bufB, mag);
                    scatter_dual(bufB, offB, sgnB, fp.scale, fp.magic);
                }
            } else if (acc == 1) {
                if constexpr (ACC == 1) {
                    mag = tile_mag(bufB, mag);
                    scatter_fixed(bufB, offB, sgnB, fp.scale, fp.magic);
                }
            } else {
                scatter_float(bufB, offB, sgnB);
            }
            if (nxt >= ntiles) break;
            hash_tile(offA, sgnA, nxt, fixed, fp.xneg);
            tile = nxt;
        }
        return mag;
    };

    auto wave_max = [&](uint32_t v) {
        for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
        return v;
    };
    auto to_f32bits = [&](uint32_t m) -> uint32_t {
        if constexpr (sizeof(AT) == 4) return m;
        else return mag16_to_f32bits(m, std::is_same<AT, __hip_bfloat16>::value);
    };

    bool fixed_ok = false;
    FixedParams fp = fixed_params(0, 0);
    if constexpr (ACC != 0) {
        zero_lds(true);
        __syncthreads();
        // Scale from the first tile of every wave, with one binade of headroom.
        uint32_t m0 = 0;
        if (wave < ntiles) {
            load_tile(bufA, wave);
            m0 = to_f32bits(tile_mag(bufA, 0u));
        }
        m0 = wave_max(m0);
        if (lane == 0) atomicMax(&ctl[0], m0);
        __syncthreads();
        const uint32_t first = ctl[0];
        if (first < 0x7F800000u) {
            int E = binade_of(first) + 1;
            int c = 0;
            for (int attempt = 0; attempt < 2 && !fixed_ok; ++attempt) {
                if (attempt > 0) {
                    zero_lds(true);
                    __syncthreads();
                }
                fp = fixed_params(E, c);
                uint32_t m = to_f32bits(run(ACC, attempt == 0, fp));
                m = wave_max(m);
                if (lane == 0) atomicMax(&ctl[1], m);
                __syncthreads();
                uint32_t kmax = 0;
                for (uint32_t e = threadIdx.x; e < (uint32_t)BG * W; e += blockDim.x) kmax = max(kmax, cnt[e] & 0xFFFFu);
                kmax = wave_max(kmax);
                if (lane == 0) atomicMax(&ctl[2], kmax);
                __syncthreads();
                const uint32_t mall = ctl[1], kall = ctl[2];
                if (mall >= 0x7F800000u) break;                    // non-finite input
                const bool mag_ok = binade_of(mall) <= E;          // |x| < 2^(E+1)
                const bool cnt_ok = kall < (1u << (10 + c));
                fixed_ok = mag_ok && cnt_ok;
                if (!fixed_ok) {
                    E = max(E, binade_of(mall));
                    while (kall >= (1u << (10 + c))) ++c;
                }
                __syncthreads();
                if (!fixed_ok && threadIdx.x == 0) { ctl[1] = 0; ctl[2] = 0; }
            }
        }
        if (!fixed_ok) {
            zero_lds(false);
            __syncthreads();
            run(0, false, fp);
        }
    } else {
        zero_lds(false);
        __syncthreads();
        run(0, false, fp);
    }
    __syncthreads();

    // ---- flush the partial into SA -----------------------------------------
    const int64_t r0g = p.row_offset + r_begin;             // first global row of the unit
    if (p.mode == 0) {
        float* SA = (float*)p.SA;
        const uint32_t total = (uint32_t)BG * W * kNT;
        for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
            const uint32_t c = e % kNT, o = (e / kNT) % W, lb = e / (kNT * W);
            const int cc = c0 + (int)c;
            if (cc >= p.n) continue;
            float v;
            if (ACC == 2 && fixed_ok) {
                // exact unit sum sum(q_hi) * 2^21 + sum(q_lo), rounded once to FP32
                const uint32_t wi = lds_row_fixed<BG>(lb, o, W) + c;
                const uint32_t cv = cnt[lb * W + o];
                const int64_t kb = (int64_t)(cv & 0xFFFFu) * (int64_t)fp.B - (int64_t)(cv >> 16);
                const int64_t hi = (int64_t)((const uint32_t*)lds)[wi] - kb;
                const int64_t lo = (int64_t)((const uint32_t*)lds)[nw + wi] - kb;
                v = (float)ldexp((double)(hi * 2097152 + lo), -(fp.S + 21));
            } else {
                v = lds[lds_row<BG>(lb, o, W) + c];
            }
            const int64_t b = (int64_t)(j0 + lb) * W + o;
            unsafeAtomicAdd(SA + b * p.ldsa + cc, v * p.scale);
        }
    } else {
        typedef _Float16 h2 __attribute__((ext_vector_type(2)));
        uint16_t* SA = (uint16_t*)p.SA;
        const uint32_t total = (uint32_t)BG * W * (kNT / 2);
        const uint64_t dn = (uint64_t)p.d * (uint64_t)p.n;
        for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
            const uint32_t cp = e % (kNT / 2), o = (e / (kNT / 2)) % W, lb = e / ((kNT / 2) * W);
            const int cc = c0 + 2 * (int)cp;
            if (cc >= p.n) continue;
            const int64_t b = (int64_t)(j0 + lb) * W + o;
            float v0, v1;
            if (fixed_ok) {
                // exact sums of the unit, rounded once to FP32
                const uint32_t* wrd = (const uint32_t*)lds + lds_row_fixed<BG>(lb, o, W) + 2 * cp;
                const uint32_t cv = cnt[lb * W + o];
                const int64_t kb = (int64_t)(cv & 0xFFFFu) * (int64_t)fp.B - (int64_t)(cv >> 16);
                v0 = ldexpf((float)((int64_t)wrd[0] - kb), -fp.S);
                v1 = ldexpf((float)((int64_t)wrd[1] - kb), -fp.S);
            } else {
                const uint32_t li = lds_row<BG>(lb, o, W) + 2 * cp;
                v0 = lds[li];
                v1 = lds[li + 1];
            }
            const uint64_t site = (uint64_t)r0g * dn + (uint64_t)b * (uint64_t)p.n + (uint64_t)cc;
            uint32_t u0 = 0, u1 = 0;
            if (p.mode >= 2) {
                u0 = round_bits(site, p.epoch, p.k0, p.k1);
                u1 = round_bits(site + 1, p.epoch, p.k0, p.k1);
            }
            const uint16_t h0 = quantize(p.mode, v0 * p.scale, u0);
            // -0.0 leaves the neighbouring half unchanged (x + -0 == x for every x)
            const uint16_t h1 = (cc + 1 < p.n) ? quantize(p.mode, v1 * p.scale, u1) : (uint16_t)0x8000u;
            const uint32_t packed = (uint32_t)h0 | ((uint32_t)h1 << 16);
            h2 hv = __builtin_bit_cast(h2, packed);
            __builtin_amdgcn_global_atomic_fadd_v2f16((h2*)(SA + b * p.ldsa + cc), hv);
        }
    }
}

template <typename AT, int BG, bool VEC, int ACC>
__global__ __launch_bounds__(kMaxThreads<AT>) void apply_kernel(ApplyArgs p)
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
    apply_item<AT, BG, VEC, ACC>(p, unit, t % p.col_tiles, t / p.col_tiles, lds);
}

// Persistent form for many problems: each workgroup takes work items from a
// device counter until the batch's items run out.  descs[] is sorted so the
// largest problems' items come first; item0 is a problem's first flat item.
template <typename AT, int BG, bool VEC, int ACC>
__global__ __launch_bounds__(kMaxThreads<AT>) void apply_batched_kernel(const BatchDesc* descs, int32_t count,
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
        apply_item<AT, BG, VEC, ACC>(bd->a, local / per_unit, t % bd->a.col_tiles, t / bd->a.col_tiles, lds);
        __syncthreads();
    }
}

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

template <typename AT, int BG, bool VEC, int ACC>
hipError_t launch_kernel(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    static size_t attr_bytes = 0;
    auto kern = apply_kernel<AT, BG, VEC, ACC>;
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

template <typename AT, int BG, bool VEC>
hipError_t launch_typed(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    return a.mode == 0 ? launch_kernel<AT, BG, VEC, 2>(plan, a, st) : launch_kernel<AT, BG, VEC, 1>(plan, a, st);
}

template <typename AT, bool VEC>
hipError_t launch_bg(const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    switch (plan.bg) {
    case 1: return launch_typed<AT, 1, VEC>(plan, a, st);
    case 2: return launch_typed<AT, 2, VEC>(plan, a, st);
    case 4: return launch_typed<AT, 4, VEC>(plan, a, st);
    case 8: return launch_typed<AT, 8, VEC>(plan, a, st);
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

unsigned grid_for(int64_t work, int threads)
{
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

}  // namespace

int apply_max_waves(int32_t a_dtype)
{
    return (a_dtype == SK_F32 ? kMaxThreads<float> : kMaxThreads<__half>) / 64;
}

size_t apply_lds_bytes(int32_t bg, int64_t W, bool dual)
{
    // fixed-point array(s) + per-bucket-row counters + 4 control words
    const size_t extra = ((size_t)bg * (size_t)W + 4) * 4;
    const size_t narr = dual ? 2 : 1;
    switch (bg) {
    case 1: return narr * lds_words<1>((uint32_t)W) * 4 + extra;
    case 2: return narr * lds_words<2>((uint32_t)W) * 4 + extra;
    case 4: return narr * lds_words<4>((uint32_t)W) * 4 + extra;
    case 8: return narr * lds_words<8>((uint32_t)W) * 4 + extra;
    default: return (size_t)-1;
    }
}

hipError_t launch_apply(int a_dtype, const Plan& plan, const ApplyArgs& a, hipStream_t st)
{
    switch (a_dtype) {
    case SK_F32: return launch_vec<float>(plan, a, st);
    case SK_F16: return launch_vec<__half>(plan, a, st);
    case SK_BF16: return launch_vec<__hip_bfloat16>(plan, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t prepare_batched(int a_dtype, int bg, bool vec, bool dual, size_t lds_bytes)
{
    switch (a_dtype) {
    case SK_F32: return batched_typed<float>(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
    case SK_F16: return batched_typed<__half>(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
    case SK_BF16: return batched_typed<__hip_bfloat16>(bg, vec, dual, nullptr, 0, 0, nullptr, 0, 8, lds_bytes, nullptr);
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
    case SK_F32: e = batched_typed<float>(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    case SK_F16: e = batched_typed<__half>(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    case SK_BF16: e = batched_typed<__hip_bfloat16>(bg, vec, dual, descs, count, total_items, counter, grid, waves, lds_bytes, st); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || !post_scale) return e;
    hipLaunchKernelGGL(batch_scale_kernel, dim3(fx, (unsigned)count), dim3(256), 0, st, descs, count);
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
