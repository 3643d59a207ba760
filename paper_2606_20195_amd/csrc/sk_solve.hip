// Least squares by sketch-and-precondition with FP64 iterative refinement,
// and the FP32 Householder QR and triangular inverse it is built on.
//
// The paper solves the sketched problem min ||SAx - Sb|| with an FP32 reduced
// QR and a triangular solve (Section 5.1).  Here that solution is only the
// start: R of the QR is the right preconditioner of LSQR (Paige and Saunders,
// ACM TOMS 8(1), 1982, Section 4) run in FP32 on the correction equation of
// FP64 iterative refinement, so the answer is the FP64 least-squares solution
// for the stored A whatever the precision of the sketch.
//
// Device work per solve:
//   sketch      SA (the handle's mode) and Sb (FP32) into M = [SA | Sb]
//   factor      blocked Householder QR of M in FP32 (one-workgroup panel
//               kernel + multi-workgroup trailing update per panel), P = R^-1
//               and P^T in FP32, x0 = P (Q^T Sb) in FP64
//   refine      per step one FP64 row pass (r = b - A x, A^T r, norms) and
//               one row pass per LSQR iteration; a row pass reads A once and
//               forms both A t and A^T u (the row of A needed for the second
//               product is the one just read), and its last workgroup to
//               finish reduces the per-workgroup partials and runs the
//               O(n^2) vector recurrences, so an LSQR iteration is one launch.
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>

#include "sk_internal.hpp"

namespace sk {

namespace {

constexpr int kT = 1024;           // threads of the row passes and one-workgroup kernels
constexpr int kWaves = kT / 64;
constexpr int kTI = 256;           // threads of the triangular inverse (one column per wave)
constexpr int kQB = 32;            // columns per tile of the tiled trailing update
constexpr int kQNRB = 16;          // row blocks of its partial W = V^T C (at least 64 rows each)
constexpr int kQR2 = 64;           // rows per workgroup of its C -= V (T^T W)
constexpr int kMaxN = 1024;
constexpr int64_t kQRRows = 16384;   // rows of one QR factorisation (LDS panel kernel)
// QR scratch: T (kQB x kQB) and the partials of the tiled update (kQNRB row
// blocks x kQB reflectors x padded columns of at most kMaxN + 1)
constexpr int64_t kQRScratchFloats =
    (int64_t)kQB * kQB + (int64_t)kQNRB * kQB * (((int64_t)kMaxN + 1 + kQB - 1) / kQB * kQB);
constexpr int64_t kMaxD = 131072;    // sketch rows of sketch_solve (taller sketches: two-level QR)

// Device-resident state of the refinement and of the running LSQR.
struct SolveState {
    double fro2;        // ||A||_F^2
    double bnorm2;      // ||b||^2
    double rnorm;       // ||b - A x|| of the current x
    double crit;        // ||A^T r|| / (||A||_F ||r||)
    double rel;         // ||r|| / ||b||
    double alpha, rhobar, phibar, anorm2, coef, beta1;
    double alpha1;      // ||(A P)^T r/||r|| || at the start of the current LSQR run
    double rfro2;       // ||R||_F^2 of the triangular factor of the sketch
    double tol, inner_tol;
    int32_t outer_done, inner_done, inner_iter, total_inner;
    int32_t bad, max_inner, pad0, pad1;
};

// ------------------------------------------------------------ reductions

// Sums over aligned groups of W lanes (W a power of two <= 64), every lane of
// a group receiving the same bits: each step adds a lane's value to its
// partner's, so both partners add the same two numbers.  Steps within a row
// of 16 lanes are DPP (quad swaps, half-row and row mirrors), the 16-lane
// exchange is a ds_swizzle, the 32-lane one v_permlane32_swap.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

template <int W>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (W >= 2) v += __uint_as_float(dpp32<0xB1>(__float_as_uint(v)));    // quad_perm [1,0,3,2]
    if constexpr (W >= 4) v += __uint_as_float(dpp32<0x4E>(__float_as_uint(v)));    // quad_perm [2,3,0,1]
    if constexpr (W >= 8) v += __uint_as_float(dpp32<0x141>(__float_as_uint(v)));   // row_half_mirror
    if constexpr (W >= 16) v += __uint_as_float(dpp32<0x140>(__float_as_uint(v)));  // row_mirror
    if constexpr (W >= 32) v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
    if constexpr (W >= 64) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
        v = __int_as_float(r[0]) + __int_as_float(r[1]);
    }
    return v;
}

template <int CTRL>
__device__ __forceinline__ double dpp64(double v)
{
    const uint64_t b = __double_as_longlong(v);
    const uint64_t lo = dpp32<CTRL>((uint32_t)b), hi = dpp32<CTRL>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

template <int W>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (W >= 2) v += dpp64<0xB1>(v);
    if constexpr (W >= 4) v += dpp64<0x4E>(v);
    if constexpr (W >= 8) v += dpp64<0x141>(v);
    if constexpr (W >= 16) v += dpp64<0x140>(v);
    if constexpr (W >= 32) {
        const uint64_t b = __double_as_longlong(v);
        const uint64_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)b, 0x401F);
        const uint64_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), 0x401F);
        v += __longlong_as_double((long long)(lo | (hi << 32)));
    }
    if constexpr (W >= 64) {
        const uint64_t b = __double_as_longlong(v);
        const auto rl = __builtin_amdgcn_permlane32_swap((int)(uint32_t)b, (int)(uint32_t)b, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap((int)(uint32_t)(b >> 32), (int)(uint32_t)(b >> 32), false,
                                                         false);
        const double a0 = __longlong_as_double((long long)((uint64_t)(uint32_t)rl[0] | ((uint64_t)(uint32_t)rh[0] << 32)));
        const double a1 = __longlong_as_double((long long)((uint64_t)(uint32_t)rl[1] | ((uint64_t)(uint32_t)rh[1] << 32)));
        v = a0 + a1;
    }
    return v;
}

// Sum over groups of 32 or 64 lanes (the QR panel's column groups).
__device__ __forceinline__ float sum_lanes(float v, int width)
{
    return width == 32 ? group_sum<32>(v) : group_sum<64>(v);
}

// Sum over all kT threads; every thread receives the total.  `sh` holds kWaves
// doubles; all threads must call it.
template <int NT = kT>
__device__ double block_sum(double v, double* sh)
{
    v = group_sum<64>(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) t += sh[i];
    return t;
}

// ------------------------------------------------------------ element loads

template <typename AT> struct ET;
template <> struct ET<float> { static constexpr int C = 4; static constexpr int B = 4; };
template <> struct ET<__half> { static constexpr int C = 8; static constexpr int B = 2; };
template <> struct ET<__hip_bfloat16> { static constexpr int C = 8; static constexpr int B = 2; };

template <typename AT> __device__ __forceinline__ float lo16(uint32_t w);
template <typename AT> __device__ __forceinline__ float hi16(uint32_t w);
template <> __device__ __forceinline__ float lo16<__half>(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
}
template <> __device__ __forceinline__ float hi16<__half>(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}
template <> __device__ __forceinline__ float lo16<__hip_bfloat16>(uint32_t w) { return __uint_as_float(w << 16); }
template <> __device__ __forceinline__ float hi16<__hip_bfloat16>(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// C consecutive elements (16 bytes) at byte offset `off` of the buffer.  With
// vec = false the bytes are read with element-sized loads (any element
// alignment).  Offsets past the buffer's end read as zero.
template <typename AT>
__device__ __forceinline__ void load_raw(__amdgpu_buffer_rsrc_t rs, uint32_t off, bool vec, uint32_t (&w)[4])
{
    if (vec) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
        w[0] = q[0];
        w[1] = q[1];
        w[2] = q[2];
        w[3] = q[3];
    } else if constexpr (ET<AT>::B == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4u * e), 0, 0);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t l = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)(off + 4u * e), 0, 0);
            const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)(off + 4u * e + 2u), 0, 0);
            w[e] = (l & 0xFFFFu) | (h << 16);
        }
    }
}

// The C elements of a raw chunk as FP32.  The row passes keep chunks raw
// while their loads are in flight (16-bit elements take half the registers)
// and convert them where they are used.
template <typename AT>
__device__ __forceinline__ void unpack(const uint32_t (&w)[4], float (&a)[ET<AT>::C])
{
    if constexpr (ET<AT>::B == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = __uint_as_float(w[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            a[2 * e] = lo16<AT>(w[e]);
            a[2 * e + 1] = hi16<AT>(w[e]);
        }
    }
}

// load_raw then unpack: C elements as FP32.
template <typename AT>
__device__ __forceinline__ void load_chunk(__amdgpu_buffer_rsrc_t rs, uint32_t off, bool vec,
                                           float (&a)[ET<AT>::C])
{
    uint32_t w[4];
    load_raw<AT>(rs, off, vec, w);
    unpack<AT>(w, a);
}

// ------------------------------------------------------------ row passes

struct RowArgs {
    const void* A;
    int64_t lda, m, rpw;       // rows per workgroup
    int32_t n, vec, mask, first;
    const double* b;
    double* x;                 // FP64 solution (n)
    float* u;                  // m: r in FP32 after a residual pass, then LSQR's unnormalised u
    float* t;                  // n: P v, the direction of the next product by A (FP32 copy of tv)
    const float* M;            // n x n: P P^T (symmetric, dense)
    const float* PT;           // P^T (n x n): x0 and nothing per iteration
    int64_t ldp;
    double* tv;                // LSQR in the t = P v form (n each): t, W = P w, Y = P y
    double* W;
    double* Y;
    double* part;              // per-workgroup partials, stride pst doubles
    int32_t pst;
    SolveState* st;
    uint32_t* ticket;
};

// Dynamic LDS of a row pass: per-wave column sums, then the epilogue's vectors.
size_t row_lds_bytes(int n, bool fp64)
{
    const size_t pass = (size_t)kWaves * n * (fp64 ? 8 : 4);
    const size_t epi = (size_t)(3 * (n + 4) + kT + kWaves) * 8;
    return std::max(pass, epi);
}

// Reduce `nv` values over the workgroup partials into out[0..nv) (LDS).  The
// loads of one thread are issued eight at a time.
__device__ void reduce_partials(const double* part, int pst, int nwg, int nv, double* out, double* tmp)
{
    const int tid = threadIdx.x;
    const int parts = nv > kT / 2 ? 1 : kT / nv;
    const int nj = parts == 1 ? (nv + kT - 1) / kT : 1;
    for (int jj = 0; jj < nj; ++jj) {
        const int idx = tid + jj * kT;
        const int j = parts == 1 ? idx : tid % nv;
        const int q = parts == 1 ? 0 : tid / nv;
        double acc = 0.0;
        if (j < nv && q < parts) {
            double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int w = q;
            for (; w + 7 * parts < nwg; w += 8 * parts) {
#pragma unroll
                for (int e = 0; e < 8; ++e) s[e] += part[(int64_t)(w + e * parts) * pst + j];
            }
            for (; w < nwg; w += parts) s[0] += part[(int64_t)w * pst + j];
            acc = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
        }
        if (parts == 1) {
            if (j < nv) out[j] = acc;
        } else if (tid < parts * nv) {
            tmp[tid] = acc;
        }
    }
    __syncthreads();
    if (parts > 1) {
        for (int j = tid; j < nv; j += kT) {
            double sum = 0.0;
            for (int q = 0; q < parts; ++q) sum += tmp[q * nv + j];
            out[j] = sum;
        }
        __syncthreads();
    }
}

// out = S in for an n x n matrix S read through columns (S symmetric, or S
// given transposed): out_i = sum_j S[j][i] in_j.  Loads issued eight at a time.
__device__ void matvec_cols(const float* S, int64_t lds_, int n, const double* in, double* out, double* tmp)
{
    const int tid = threadIdx.x;
    const int parts = kT / n;
    if (tid < parts * n) {
        const int i = tid % n, q = tid / n;
        double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int j = q;
        for (; j + 7 * parts < n; j += 8 * parts) {
#pragma unroll
            for (int e = 0; e < 8; ++e) s[e] = fma((double)S[(int64_t)(j + e * parts) * lds_ + i], in[j + e * parts], s[e]);
        }
        for (; j < n; j += parts) s[0] = fma((double)S[(int64_t)j * lds_ + i], in[j], s[0]);
        tmp[tid] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    }
    __syncthreads();
    for (int i = tid; i < n; i += kT) {
        double sum = 0.0;
        for (int q = 0; q < parts; ++q) sum += tmp[q * n + i];
        out[i] = sum;
    }
    __syncthreads();
}

// First row of the next block of `rows` rows of the workgroup's range, from
// the workgroup's block counter (one LDS atomic per wave, lane 0's result
// read by every lane).  Row passes take their blocks this way, so the waves of
// a workgroup stream until its rows run out and finish within one block of
// each other: with blocks dealt out in a fixed order, the first wave
// measured some 60 us (a quarter of the pass) ahead of the workgroup's last.
__device__ __forceinline__ int64_t next_block(uint32_t* ctr, int lane, int64_t row0, int64_t rows)
{
    uint32_t v = 0u;
    if (lane == 0) v = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    v = (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
    return row0 + (int64_t)v * rows;
}

// True in exactly one workgroup, the last to finish; partials written before
// the call are visible to it.  Each wave first waits for its own stores to be
// acknowledged; after the barrier one thread takes a ticket with an
// agent-scope release add, so each workgroup writes its XCD's L2 back once (a
// fence in every wave would write back and invalidate the L2 once per wave,
// which also evicts the data of kernels running beside this one).  Only the
// last workgroup then invalidates (acquire fence after the add that read the
// final count), to read the other XCDs' partials.
__device__ bool last_workgroup(uint32_t* ticket)
{
    __shared__ int last;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0)
        last = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *ticket = 0u;
    return true;
}

// LSQR (Paige and Saunders, Section 4) on A P, kept in the variables
// t = P v, W = P w, Y = P y so that an iteration needs one product by
// M = P P^T and no final product: with g = A^T u / beta,
//   P^T g - beta v = q,  alpha^2 = ||q||^2 = g^T M g - 2 beta t^T g + beta^2,
//   t' = P q / alpha = (M g - beta t) / alpha,
// and the solution update is x += ||r|| Y.  Start (step 1 with
// beta_1 u_1 = r / ||r||): g = A^T r / ||r||, alpha_1 = sqrt(g^T M g),
// t_1 = M g / alpha_1, W = t_1, Y = 0.
__device__ void lsqr_start(const RowArgs& p, double* g, double rnorm)
{
    const int n = p.n, tid = threadIdx.x;
    double* mg = g + (n + 4);
    double* tmp = mg + 2 * (n + 4);
    double* sh = tmp + kT;
    const double ib = rnorm > 0.0 ? 1.0 / rnorm : 0.0;
    for (int j = tid; j < n; j += kT) g[j] *= ib;
    __syncthreads();
    matvec_cols(p.M, p.ldp, n, g, mg, tmp);
    double ss = 0.0;
    for (int j = tid; j < n; j += kT) ss = fma(g[j], mg[j], ss);
    const double alpha = sqrt(fmax(block_sum(ss, sh), 0.0));
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    for (int j = tid; j < n; j += kT) {
        const double tj = mg[j] * ia;
        p.tv[j] = tj;
        p.W[j] = tj;
        p.Y[j] = 0.0;
        p.t[j] = (float)tj;
    }
    if (tid == 0) {
        SolveState* st = p.st;
        st->alpha = alpha;
        st->alpha1 = alpha;
        st->rhobar = alpha;
        st->phibar = 1.0;
        st->anorm2 = 0.0;
        st->beta1 = rnorm;
        st->coef = rnorm > 0.0 ? alpha / rnorm : 0.0;
        st->inner_iter = 0;
        st->inner_done = (alpha == 0.0 || rnorm == 0.0) ? 1 : 0;
    }
}

// FP64 residual pass: r = b - A x, writes r (FP32) into u and reduces A^T r,
// ||r||^2 (and on the first pass ||A||_F^2, ||b||^2); the last workgroup
// evaluates the stopping test and starts LSQR.  Loads of the next rows are in
// flight while the current ones are used.
template <typename AT, int LR, int CP>
__global__ __launch_bounds__(kT) void resid_pass(RowArgs p)
{
    constexpr int C = ET<AT>::C, B = ET<AT>::B, RW = 64 / LR, U = CP >= 2 ? 1 : (ET<AT>::B == 4 ? 3 : 2);
    extern __shared__ double dsh[];
    __shared__ double xs[kMaxN + 16];          // x in FP64, zero past n
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rs = lane / LR, cl = lane % LR;
    const int n = p.n;

    // With two or more chunks per lane the A^T r sums live in LDS (each wave
    // owns a row of red[], each lane its columns) instead of registers.
    constexpr bool GL = CP >= 2;
    double* red = dsh;
    for (int c = tid; c < kMaxN + 16; c += kT) xs[c] = c < n ? p.x[c] : 0.0;
    if constexpr (GL)
        for (int c = tid; c < kWaves * n; c += kT) red[c] = 0.0;
    double g[GL ? 1 : CP][C];
    int col0[CP];
#pragma unroll
    for (int pp = 0; pp < CP; ++pp) {
        col0[pp] = C * (cl + LR * pp);
#pragma unroll
        for (int e = 0; e < C; ++e)
            if constexpr (!GL) g[pp][e] = 0.0;
    }
    __shared__ uint32_t blk_ctr;
    if (tid == 0) blk_ctr = 0u;
    __syncthreads();
    const int64_t row0 = (int64_t)blockIdx.x * p.rpw;
    const int64_t row1 = row0 >= p.m ? row0 : (row0 + p.rpw < p.m ? row0 + p.rpw : p.m);
    const uint32_t rowbytes = (uint32_t)(p.lda * B);
    const uint32_t nrec = (uint32_t)((row1 - row0) * rowbytes);
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const char*)p.A + row0 * (int64_t)rowbytes), (short)0, (int)nrec, 0x00020000);
    const bool vec = p.vec != 0, mask = p.mask != 0, first = p.first != 0;
    double rr = 0.0, aa = 0.0, bb = 0.0;
    // blocks of U * RW consecutive rows, dealt out by the workgroup's counter
    const int64_t step = RW;
    auto next = [&]() { return next_block(&blk_ctr, lane, row0, (int64_t)U * RW); };

    uint32_t aA[U][CP][4], aB[U][CP][4];
    double bA[U], bB[U];
    auto load = [&](uint32_t (&w)[U][CP][4], double (&bv)[U], int64_t rb) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t row = rb + uu * step + rs;
            const bool valid = row < row1;
            const uint32_t off = valid ? (uint32_t)(row - row0) * rowbytes : nrec;
#pragma unroll
            for (int pp = 0; pp < CP; ++pp) load_raw<AT>(rsrc, off + (uint32_t)(col0[pp] * B), vec, w[uu][pp]);
            bv[uu] = valid ? p.b[row] : 0.0;
        }
    };
    auto use = [&](const uint32_t (&w)[U][CP][4], const double (&bv)[U], int64_t rb) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t row = rb + uu * step + rs;
            const bool valid = row < row1;
            float a[CP][C];
#pragma unroll
            for (int pp = 0; pp < CP; ++pp) unpack<AT>(w[uu][pp], a[pp]);
            double dot = 0.0;
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    if (mask && col0[pp] + e >= n) a[pp][e] = 0.0f;
                    const int c = min(col0[pp] + e, kMaxN + 15);
                    dot = fma((double)a[pp][e], xs[c], dot);
                }
            dot = group_sum<LR>(dot);
            const double r = valid ? bv[uu] - dot : 0.0;
            if (valid && cl == 0) p.u[row] = (float)r;
            if (cl == 0) rr = fma(r, r, rr);
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    if constexpr (GL) {
                        const int c = col0[pp] + e;
                        if (c < n) red[wave * n + c] = fma(r, (double)a[pp][e], red[wave * n + c]);
                    } else {
                        g[pp][e] = fma(r, (double)a[pp][e], g[pp][e]);
                    }
                }
            if (first) {
                if (cl == 0) bb = fma(bv[uu], bv[uu], bb);
#pragma unroll
                for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                    for (int e = 0; e < C; ++e) aa = fma((double)a[pp][e], (double)a[pp][e], aa);
            }
        }
    };
    int64_t rb = next();
    if (rb < row1) load(aA, bA, rb);
    int64_t nx = next();
    while (rb < row1) {
        if (nx < row1) load(aB, bB, nx);
        int64_t nn = nx < row1 ? next() : nx;
        use(aA, bA, rb);
        if (nx >= row1) break;
        rb = nx;
        nx = nn;
        if (nx < row1) load(aA, bA, nx);
        nn = nx < row1 ? next() : nx;
        use(aB, bB, rb);
        if (nx >= row1) break;
        rb = nx;
        nx = nn;
    }
    // column sums: over the RW row slots of the wave, then over the waves
    if constexpr (!GL) {
#pragma unroll
        for (int o = LR; o < 64; o <<= 1)
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e) g[pp][e] += __shfl_xor(g[pp][e], o, 64);
    }
    rr = group_sum<64>(rr);
    aa = group_sum<64>(aa);
    bb = group_sum<64>(bb);
    __shared__ double wsum[kWaves][3];
    if constexpr (!GL) {
        if (rs == 0) {
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e)
                    if (col0[pp] + e < n) red[wave * n + col0[pp] + e] = g[pp][e];
        }
    }
    if (lane == 0) {
        wsum[wave][0] = rr;
        wsum[wave][1] = aa;
        wsum[wave][2] = bb;
    }
    __syncthreads();
    double* mine = p.part + (int64_t)blockIdx.x * p.pst;
    for (int j = tid; j < n; j += kT) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kWaves; ++w2) s += red[w2 * n + j];
        mine[j] = s;
    }
    if (tid < 3) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kWaves; ++w2) s += wsum[w2][tid];
        mine[n + tid] = s;
    }
    if (!last_workgroup(p.ticket)) return;

    // ---- epilogue (one workgroup)
    double* g64 = dsh;                   // n + 3 values
    double* tmp = dsh + 3 * (n + 4);
    double* sh = tmp + kT;
    reduce_partials(p.part, p.pst, gridDim.x, n + 3, g64, tmp);
    SolveState* st = p.st;
    if (first && tid == 0) {
        st->fro2 = g64[n + 1];
        st->bnorm2 = g64[n + 2];
    }
    double gs = 0.0;
    for (int j = tid; j < n; j += kT) gs = fma(g64[j], g64[j], gs);
    const double gnorm = sqrt(block_sum(gs, sh));
    const double fro2 = first ? g64[n + 1] : st->fro2;
    const double bn2 = first ? g64[n + 2] : st->bnorm2;
    const double rnorm = sqrt(g64[n]);
    const double crit = (rnorm > 0.0 && fro2 > 0.0) ? gnorm / (sqrt(fro2) * rnorm) : 0.0;
    const double rel = bn2 > 0.0 ? rnorm / sqrt(bn2) : 0.0;
    const bool done = crit <= st->tol || rel <= st->tol;
    __syncthreads();
    if (tid == 0) {
        st->rnorm = rnorm;
        st->crit = crit;
        st->rel = rel;
        st->outer_done = done ? 1 : 0;
        if (!(crit == crit) || !(rnorm == rnorm)) st->bad = 2;
    }
    if (done) return;
    lsqr_start(p, g64, rnorm);
}

// One LSQR iteration (Paige-Saunders, Section 4, steps 3-6) on the operator
// A P: u' = A t - coef u (u = beta u' from the previous iteration), A^T u' and
// ||u'||^2 in the same pass; the last workgroup finishes the iteration in the
// t-form of lsqr_start and, at termination, adds ||r|| Y to x in FP64.
template <typename AT, int LR, int CP>
__global__ __launch_bounds__(kT) void lsqr_pass(RowArgs p)
{
    constexpr int C = ET<AT>::C, B = ET<AT>::B, RW = 64 / LR, U = CP >= 2 ? 1 : 4;
    extern __shared__ double dsh[];
    SolveState* st = p.st;
    if (st->inner_done != 0 || st->outer_done != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rs = lane / LR, cl = lane % LR;
    const int n = p.n;

    float tr[CP][C], g[CP][C];
    int col0[CP];
#pragma unroll
    for (int pp = 0; pp < CP; ++pp) {
        col0[pp] = C * (cl + LR * pp);
#pragma unroll
        for (int e = 0; e < C; ++e) {
            const int c = col0[pp] + e;
            tr[pp][e] = c < n ? p.t[c] : 0.0f;
            g[pp][e] = 0.0f;
        }
    }
    const float coef = (float)st->coef;
    const int64_t row0 = (int64_t)blockIdx.x * p.rpw;
    const int64_t row1 = row0 >= p.m ? row0 : (row0 + p.rpw < p.m ? row0 + p.rpw : p.m);
    const uint32_t rowbytes = (uint32_t)(p.lda * B);
    const uint32_t nrec = (uint32_t)((row1 - row0) * rowbytes);
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void*)((const char*)p.A + row0 * (int64_t)rowbytes), (short)0, (int)nrec, 0x00020000);
    const bool vec = p.vec != 0, mask = p.mask != 0;
    float ss = 0.0f;
    // A wave takes U * RW consecutive rows at a time (slot uu, row slot rs =
    // row uu * RW + rs of the block).  With BL it moves their u in one load
    // and one store of U * RW lanes, handing values between lanes; otherwise
    // every row loads and stores its own u.
    constexpr bool BL = U * RW <= 64 && U <= LR;
    const int64_t step = RW;
    __shared__ uint32_t blk_ctr;
    if (tid == 0) blk_ctr = 0u;
    __syncthreads();
    auto next = [&]() { return next_block(&blk_ctr, lane, row0, (int64_t)U * RW); };

    float aA[U][CP][C], aB[U][CP][C];
    float uA[U], uB[U];
    auto load = [&](float (&a)[U][CP][C], float (&uo)[U], int64_t rb) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t row = rb + uu * step + rs;
            const bool valid = row < row1;
            const uint32_t off = valid ? (uint32_t)(row - row0) * rowbytes : nrec;
#pragma unroll
            for (int pp = 0; pp < CP; ++pp) load_chunk<AT>(rsrc, off + (uint32_t)(col0[pp] * B), vec, a[uu][pp]);
            if constexpr (!BL) uo[uu] = valid ? p.u[row] : 0.0f;
        }
        if constexpr (BL) {
            const int64_t r = rb + lane;
            const float uv = (lane < U * RW && r < row1) ? p.u[r] : 0.0f;
#pragma unroll
            for (int uu = 0; uu < U; ++uu) uo[uu] = __shfl(uv, uu * RW + rs, 64);
        }
    };
    auto use = [&](float (&a)[U][CP][C], const float (&uo)[U], int64_t rb) {
        float unv[U];
#pragma unroll
        for (int uu = 0; uu < U; ++uu) {
            const int64_t row = rb + uu * step + rs;
            const bool valid = row < row1;
            float dot = 0.0f;
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    if (mask && col0[pp] + e >= n) a[uu][pp][e] = 0.0f;
                    dot = __builtin_fmaf(a[uu][pp][e], tr[pp][e], dot);
                }
            dot = group_sum<LR>(dot);
            const float un = valid ? __builtin_fmaf(-coef, uo[uu], dot) : 0.0f;
            if constexpr (!BL)
                if (valid && cl == 0) p.u[row] = un;
            if (cl == 0) ss = __builtin_fmaf(un, un, ss);
#pragma unroll
            for (int pp = 0; pp < CP; ++pp)
#pragma unroll
                for (int e = 0; e < C; ++e) g[pp][e] = __builtin_fmaf(un, a[uu][pp][e], g[pp][e]);
            unv[uu] = un;
        }
        if constexpr (BL) {
            // row l of the block (slot l / RW, row slot l % RW): lane (l % RW) * LR + l / RW
            // holds its value once each lane has picked un[cl] (cl < U)
            float v = unv[0];
#pragma unroll
            for (int uu = 1; uu < U; ++uu) v = cl == uu ? unv[uu] : v;
            const int l = lane & (U * RW - 1);
            const float o = __shfl(v, (l % RW) * LR + l / RW, 64);
            const int64_t r = rb + lane;
            if (lane < U * RW && r < row1) p.u[r] = o;
        }
    };
    // Blocks are handed out in turn from an LDS counter (the index of the
    // block after next is taken while the current one is used), so the waves
    // of a workgroup finish together whatever the arbitration between them.
    int64_t rb = next();
    if (rb < row1) load(aA, uA, rb);
    int64_t nx = next();
    while (rb < row1) {
        if (nx < row1) load(aB, uB, nx);
        int64_t nn = nx < row1 ? next() : nx;
        use(aA, uA, rb);
        if (nx >= row1) break;
        rb = nx;
        nx = nn;
        if (nx < row1) load(aA, uA, nx);
        nn = nx < row1 ? next() : nx;
        use(aB, uB, rb);
        if (nx >= row1) break;
        rb = nx;
        nx = nn;
    }
#pragma unroll
    for (int o = LR; o < 64; o <<= 1)
#pragma unroll
        for (int pp = 0; pp < CP; ++pp)
#pragma unroll
            for (int e = 0; e < C; ++e) g[pp][e] += __shfl_xor(g[pp][e], o, 64);
    ss = group_sum<64>(ss);
    float* red = (float*)dsh;
    __shared__ float wss[kWaves];
    if (rs == 0) {
#pragma unroll
        for (int pp = 0; pp < CP; ++pp)
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (col0[pp] + e < n) red[wave * n + col0[pp] + e] = g[pp][e];
    }
    if (lane == 0) wss[wave] = ss;
    __syncthreads();
    double* mine = p.part + (int64_t)blockIdx.x * p.pst;
    for (int j = tid; j < n; j += kT) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kWaves; ++w2) s += (double)red[w2 * n + j];
        mine[j] = s;
    }
    if (tid == 0) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kWaves; ++w2) s += (double)wss[w2];
        mine[n] = s;
    }
    if (!last_workgroup(p.ticket)) return;

    // ---- epilogue (one workgroup)
    double* g64 = dsh;                       // A^T u' (n), ||u'||^2
    double* mg = g64 + (n + 4);
    double* tmp = mg + 2 * (n + 4);
    double* sh = tmp + kT;
    reduce_partials(p.part, p.pst, gridDim.x, n + 1, g64, tmp);
    const double beta = sqrt(g64[n]);
    const double alpha_old = st->alpha;
    const double anorm2 = st->anorm2 + alpha_old * alpha_old + beta * beta;
    const double ib = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int j = tid; j < n; j += kT) g64[j] *= ib;
    __syncthreads();
    matvec_cols(p.M, p.ldp, n, g64, mg, tmp);
    double s_gmg = 0.0, s_tg = 0.0;
    for (int j = tid; j < n; j += kT) {
        s_gmg = fma(g64[j], mg[j], s_gmg);
        s_tg = fma(p.tv[j], g64[j], s_tg);
    }
    const double gmg = block_sum(s_gmg, sh);
    const double tg = block_sum(s_tg, sh);
    const double alpha = sqrt(fmax(gmg - 2.0 * beta * tg + beta * beta, 0.0));
    const double ia = alpha > 0.0 ? 1.0 / alpha : 0.0;
    // plane rotation (no damping)
    const double rhobar0 = st->rhobar, phibar0 = st->phibar;
    const double rho = hypot(rhobar0, beta);
    const double c = rho > 0.0 ? rhobar0 / rho : 1.0;
    const double sn = rho > 0.0 ? beta / rho : 0.0;
    const double theta = sn * alpha;
    const double rhobar = -c * alpha;
    const double phi = c * phibar0;
    const double phibar = sn * phibar0;
    const double t1 = rho > 0.0 ? phi / rho : 0.0;
    const double t2 = rho > 0.0 ? -theta / rho : 0.0;
    const int iter = st->inner_iter + 1;
    const double itol = st->inner_tol;
    // Stopping: the correction problem's normal-equations residual
    // ||(A P)^T (r^ - A P y)|| = phibar alpha |c| (Paige-Saunders, Section 5)
    // has fallen by inner_tol from its start alpha_1, or (consistent
    // corrections) the residual estimate phibar has fallen by inner_tol.  The
    // test is relative to the start, not to ||r^||: near the solution r^ is
    // almost orthogonal to the range of A, and a test relative to ||r^|| would
    // stop after one iteration.
    //   It also stops once the same estimate bounds the outer criterion below
    // half its tolerance: with A = (A P) R, the updated residual r' satisfies
    // ||A^T r'|| <= ||R||_2 ||(A P)^T r'||, and ||r'|| = phibar ||r||, so
    // ||A^T r'|| / (||A||_F ||r'||) <= (||R||_F / ||A||_F) alpha |c|.  The
    // estimate holds until FP32 rounding in the products dominates; the FP64
    // residual of the next outer step decides convergence either way.
    const double test2 = st->alpha1 > 0.0 ? phibar * alpha * fabs(c) / st->alpha1 : 0.0;
    const double crit_est = st->fro2 > 0.0 ? sqrt(st->rfro2 / st->fro2) * alpha * fabs(c) : 1.0;
    const bool done = beta == 0.0 || alpha == 0.0 || test2 <= itol || phibar <= itol || crit_est <= 0.5 * st->tol ||
                      iter >= st->max_inner;
    const double scale = st->beta1;
    for (int j = tid; j < n; j += kT) {
        const double tn = (mg[j] - beta * p.tv[j]) * ia;      // P v_{k+1}
        const double wj = p.W[j];
        const double yj = fma(t1, wj, p.Y[j]);
        p.W[j] = fma(t2, wj, tn);
        p.tv[j] = tn;
        p.t[j] = (float)tn;
        if (done) p.x[j] = fma(scale, yj, p.x[j]);
        else p.Y[j] = yj;
    }
    if (tid == 0) {
        st->alpha = alpha;
        st->rhobar = rhobar;
        st->phibar = phibar;
        st->anorm2 = anorm2;
        st->coef = beta > 0.0 ? alpha / beta : 0.0;
        st->inner_iter = iter;
        st->total_inner += 1;
        st->inner_done = done ? 1 : 0;
        if (!(alpha == alpha) || !(beta == beta)) st->bad = 2;
    }
}

// M = P P^T from P^T (n x n): M[i][j] = sum_k PT[k][i] PT[k][j], k >= max(i, j),
// accumulated in FP64 and stored in FP32.
__global__ void gram_kernel(const float* PT, int64_t ldp, int32_t n, float* M)
{
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= n || j >= n) return;
    double s = 0.0;
    for (int k = max(i, j); k < n; ++k) s = fma((double)PT[(int64_t)k * ldp + i], (double)PT[(int64_t)k * ldp + j], s);
    M[(int64_t)i * ldp + j] = (float)s;
}

// ------------------------------------------------------------ QR (FP32)

// Row i of the triangular factor T of a panel's block reflector (forward,
// columnwise): T[i][i] = tau_i and T[i][j] = -tau_j sum_{i <= l < j} T[i][l]
// gv[l][j] for i < j, where gv[l][j] = v_l . v_j; the lane keeps its row in
// registers, so each step reads only its own lane and gv.  T[i][l] = 0 for
// l < i, so the sums may run over all l < j.
__device__ __forceinline__ void form_t(int i, int nb, const float* gv, const float* s_tau, float* Tout)
{
    float trow[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        float val = 0.0f;
        if (j < nb) {
            const float tj = s_tau[j];
            if (i == j) {
                val = tj;
            } else if (i < j) {
                float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int l = 0; l < j; ++l) acc[l & 3] = __builtin_fmaf(trow[l], gv[l * 33 + j], acc[l & 3]);
                val = -tj * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
            }
        }
        trow[j] = val;
    }
#pragma unroll
    for (int j = 0; j < 32; ++j)
        if (j < nb) Tout[i * nb + j] = trow[j];
}

// Householder factorisation of the panel M[k0:rows, k0:k0+nb] in LDS by one
// workgroup (LAPACK slarfg convention: beta = -sign(x0) ||x||, v[0] = 1).
__global__ __launch_bounds__(kT) void qr_panel_kernel(float* M, int64_t ldm, int32_t rows_total, int32_t k0,
                                                       int32_t nb, float* tau, float* Tout)
{
    extern __shared__ float pan[];
    __shared__ float s_tau[32];
    const int rows = rows_total - k0;
    const int ldl = rows | 1;            // odd column stride: the transposing stores hit distinct banks
    const int tid = threadIdx.x;
    // staged eight loads at a time per thread
    for (int base = 0; base < rows * nb; base += 8 * kT) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = base + e * kT + tid;
            const int r = idx / nb, c = idx - r * nb;
            v[e] = idx < rows * nb ? M[(int64_t)(k0 + r) * ldm + k0 + c] : 0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = base + e * kT + tid;
            const int r = idx / nb, c = idx - r * nb;
            if (idx < rows * nb) pan[c * ldl + r] = v[e];
        }
    }
    __syncthreads();
    // Narrow panels (nb <= 8: tall matrices) take step j as the register
    // kernel does, with the panel in LDS: every thread sums
    // S_c = sum_{r > j} y_rj y_rc over its rows for the columns c >= j at once
    // (S_j is the squared norm below the diagonal), one block reduction gives
    // beta, tau, scal = 1 / (x0 - beta) and the coefficients tau w_c with
    // w_c = y_jc + scal S_c (v_j . y_c), and every thread updates its rows
    // (8192 x 4 panels: 73 -> 60 us).  Wider panels keep one lane group per
    // column, so the columns' dot products run side by side (2048 x 16: the
    // block-wide form measured 1.3x slower).
    __shared__ float wsum[kT / 64][32];
    __shared__ float ssum[32];
    __shared__ float coefv[32];
    __shared__ float step_s[2];          // scal, beta
    const int lane = tid & 63, wv = tid >> 6;
    if (nb <= 8) {
        for (int j = 0; j < nb; ++j) {
            const int nc = nb - j;           // columns j .. nb - 1
            float part[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) part[c] = 0.0f;
            for (int r = j + 1 + tid; r < rows; r += kT) {
                const float yj = pan[j * ldl + r];
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if (c < nc) part[c] = __builtin_fmaf(yj, pan[(j + c) * ldl + r], part[c]);
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                if (c < nc) {
                    float v = part[c];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
                    if (lane == 0) wsum[wv][c] = v;
                }
            }
            __syncthreads();
            if (tid < nc) {
                float sum = 0.0f;
#pragma unroll
                for (int w = 0; w < kT / 64; ++w) sum += wsum[w][tid];
                ssum[tid] = sum;
            }
            __syncthreads();
            if (tid == 0) {
                const float x0 = pan[j * ldl + j];
                const float sig = ssum[0];
                float t = 0.0f, beta = x0, scal = 0.0f;
                if (sig > 0.0f) {
                    beta = -copysignf(sqrtf(__builtin_fmaf(x0, x0, sig)), x0);
                    t = (beta - x0) / beta;
                    scal = 1.0f / (x0 - beta);
                }
                s_tau[j] = t;
                step_s[0] = scal;
                step_s[1] = beta;
            }
            __syncthreads();
            if (tid > 0 && tid < nc)
                coefv[tid] = s_tau[j] * __builtin_fmaf(step_s[0], ssum[tid], pan[(j + tid) * ldl + j]);
            __syncthreads();
            const float scal = step_s[0];
            if (tid == 0) {
                for (int c = 1; c < nc; ++c) pan[(j + c) * ldl + j] -= coefv[c];
                pan[j * ldl + j] = step_s[1];
            }
            for (int r = j + 1 + tid; r < rows; r += kT) {
                const float v = pan[j * ldl + r] * scal;
                pan[j * ldl + r] = v;
#pragma unroll
                for (int c = 1; c < 8; ++c)
                    if (c < nc) pan[(j + c) * ldl + r] = __builtin_fmaf(-coefv[c], v, pan[(j + c) * ldl + r]);
            }
            __syncthreads();
        }
    } else {
        // One sweep per step: the pivot's norm comes from the previous step's
        // update of that column (its group sums the squares as it writes
        // them), the other columns use the unscaled pivot with the scale
        // folded into their coefficients, and the pivot column is scaled one
        // step later, when no group reads it.
        const int G = nb > 16 ? 32 : 64;     // lanes per column group: kT / G >= nb groups
        const int grp = tid / G, gl = tid % G;
        __shared__ float sig_s[32];
        __shared__ float scal_s[32];
        if (grp == 0) {
            const float* x = pan;
            float s4 = 0.0f;
            for (int r = 1 + gl; r < rows; r += G) s4 = __builtin_fmaf(x[r], x[r], s4);
            s4 = sum_lanes(s4, G);
            if (gl == 0) sig_s[0] = s4;
        }
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            if (tid == 0) {
                float* x = pan + j * ldl;
                const float x0 = x[j], sig = sig_s[j];
                float t = 0.0f, beta = x0, scal = 0.0f;
                if (sig > 0.0f) {
                    beta = -copysignf(sqrtf(__builtin_fmaf(x0, x0, sig)), x0);
                    t = (beta - x0) / beta;
                    scal = 1.0f / (x0 - beta);
                }
                x[j] = beta;
                s_tau[j] = t;
                scal_s[j] = scal;
            }
            __syncthreads();
            if (j >= 1 && grp == j - 1) {
                float* x = pan + (j - 1) * ldl;
                const float scal = scal_s[j - 1];
                for (int r = j + gl; r < rows; r += G) x[r] *= scal;
            }
            if (grp > j && grp < nb) {
                const float t = s_tau[j], scal = scal_s[j];
                const float* x = pan + j * ldl;
                float* yc = pan + grp * ldl;
                float ss = 0.0f;
                if (t != 0.0f) {
                    float w4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    int r = j + 1 + gl;
                    for (; r + 3 * G < rows; r += 4 * G) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) w4[e] = __builtin_fmaf(x[r + e * G], yc[r + e * G], w4[e]);
                    }
                    for (; r < rows; r += G) w4[0] = __builtin_fmaf(x[r], yc[r], w4[0]);
                    const float dot = sum_lanes((w4[0] + w4[1]) + (w4[2] + w4[3]), G);
                    const float w = __builtin_fmaf(scal, dot, yc[j]) * t;
                    if (gl == 0) yc[j] -= w;
                    const float ws = w * scal;
                    for (int r2 = j + 1 + gl; r2 < rows; r2 += G) {
                        const float y = __builtin_fmaf(-ws, x[r2], yc[r2]);
                        yc[r2] = y;
                        if (r2 > j + 1) ss = __builtin_fmaf(y, y, ss);
                    }
                } else if (grp == j + 1) {
                    for (int r2 = j + 2 + gl; r2 < rows; r2 += G) ss = __builtin_fmaf(yc[r2], yc[r2], ss);
                }
                if (grp == j + 1) {
                    ss = sum_lanes(ss, G);
                    if (gl == 0) sig_s[j + 1] = ss;
                }
            }
            __syncthreads();
        }
        if (grp == nb - 1) {
            float* x = pan + (nb - 1) * ldl;
            const float scal = scal_s[nb - 1];
            for (int r = nb + gl; r < rows; r += G) x[r] *= scal;
        }
    }
    __syncthreads();
    for (int idx = tid; idx < rows * nb; idx += kT) {
        const int r = idx / nb, c = idx - r * nb;
        M[(int64_t)(k0 + r) * ldm + k0 + c] = pan[c * ldl + r];
    }
    if (tid < nb) tau[k0 + tid] = s_tau[tid];
    if (!Tout) return;
    // Triangular factor of the block reflector (forward, columnwise):
    // H_0 H_1 ... H_{nb-1} = I - V T V^T with T[j][j] = tau_j and
    // T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j).  First the Gram
    // entries gv[l][j] = v_l . v_j (l < j; v_j is 0 above row j and 1 on it),
    // one wave per entry, then the recurrence with lane i holding row i of T
    // in registers, so each step reads only its own lane and gv.
    __shared__ float gv[32 * 33];
    const int wave = wv;
    const int npairs = nb * (nb - 1) / 2;
    for (int pi = wave; pi < npairs; pi += kT / 64) {
        int j = 1;
        while ((j * (j + 1)) / 2 <= pi) ++j;
        const int l = pi - j * (j - 1) / 2;
        const float* vl = pan + l * ldl;
        const float* vj = pan + j * ldl;
        float acc = 0.0f;
        for (int r = j + 1 + lane; r < rows; r += 64) acc = __builtin_fmaf(vl[r], vj[r], acc);
        acc = group_sum<64>(acc);
        if (lane == 0) gv[l * 33 + j] = acc + vl[j];
    }
    __syncthreads();
    if (wave == 0 && lane < nb) form_t(lane, nb, gv, s_tau, Tout);
}

// Register-resident panel factorisation for panels of at most 4 * kPT rows:
// thread t holds rows t, t + kPT, ... (R of them) of the nb <= 32 panel
// columns in registers.  Step j needs one block reduction: with
// S_c = sum_{r > j} y_rj y_rc for every column c, S_j is the squared norm
// below the diagonal that fixes beta, tau and scal = 1 / (x0 - beta)
// (x0 = y_jj), and
// w_c = y_jc + scal S_c is v_j . y_c for c > j (the dot product of the
// trailing column with the reflector v_j = (1, scal * y_{r > j, j})) and
// v_c . v_j for c < j (the Gram column of T).  The update
// y_rc -= tau w_c v_r then touches registers only.  A wave folds its 32 sums
// by halving (each exchange sends the half the partner keeps), leaving sum c
// on lanes 2c and 2c + 1; 128 threads add the waves' sums and form the step's
// coefficients.  LDS buffers alternate between steps, so two barriers a step
// suffice.
constexpr int kPT = 256;

template <int CTRL>
__device__ __forceinline__ float dppf(float v)
{
    return __uint_as_float(dpp32<CTRL>(__float_as_uint(v)));
}

// One halving step of the wave fold: lanes with `hi` keep values [H, 2H), the
// others [0, H); each adds what the partner (reached by X) sends.
template <int H, typename X>
__device__ __forceinline__ void fold_half(float* p, bool hi, X exch)
{
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float keep = hi ? p[k + H] : p[k];
        const float send = hi ? p[k] : p[k + H];
        p[k] = keep + exch(send);
    }
}

template <int R>
__global__ __launch_bounds__(kPT) void qr_panel_reg_kernel(float* M, int64_t ldm, int32_t rows_total, int32_t k0,
                                                           int32_t nb, float* tau, float* Tout)
{
    __shared__ float red[2][kPT / 64][32];
    __shared__ float piv[2][32];
    __shared__ float coef[2][32];
    __shared__ float stepv[2][2];
    __shared__ float gv[32 * 33];
    __shared__ float s_tau[32];
    const int rows = rows_total - k0;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float y0[32], y1[32], y2[32], y3[32];
    auto each = [&](auto&& f) {
        f(y0, 0);
        if constexpr (R > 1) f(y1, 1);
        if constexpr (R > 2) {
            f(y2, 2);
            f(y3, 3);
        }
    };
    each([&](float* y, int i) {
        const int r = tid + i * kPT;
        const float* src = M + (int64_t)(k0 + (r < rows ? r : 0)) * ldm + k0;
        if (nb == 32) {
#pragma unroll
            for (int c = 0; c < 32; ++c) y[c] = src[c];
        } else {
#pragma unroll
            for (int c = 0; c < 32; ++c) y[c] = src[c < nb ? c : 0];
#pragma unroll
            for (int c = 0; c < 32; ++c) y[c] = c < nb ? y[c] : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 32; ++c) y[c] = r < rows ? y[c] : 0.0f;
    });
    for (int j = 0; j < nb; ++j) {
        const int b = j & 1;
        float p[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) p[c] = 0.0f;
        each([&](float* y, int i) {
            const int r = tid + i * kPT;
            const float a = r > j ? y[j] : 0.0f;
#pragma unroll
            for (int c = 0; c < 32; ++c) p[c] = __builtin_fmaf(a, y[c], p[c]);
            if (r == j) {
#pragma unroll
                for (int c = 0; c < 32; ++c) piv[b][c] = y[c];
            }
        });
        fold_half<16>(p, lane & 32, [](float v) { return __shfl_xor(v, 32); });
        fold_half<8>(p, lane & 16,
                     [](float v) { return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)); });
        fold_half<4>(p, lane & 8, [](float v) { return dppf<0x140>(v); });   // row_mirror: flips lane bit 3
        fold_half<2>(p, lane & 4, [](float v) { return dppf<0x141>(v); });   // row_half_mirror: flips bit 2
        fold_half<1>(p, lane & 2, [](float v) { return dppf<0x4E>(v); });    // quad_perm [2,3,0,1]: bit 1
        p[0] += dppf<0xB1>(p[0]);                                            // quad_perm [1,0,3,2]: bit 0
        if ((lane & 1) == 0) red[b][wave][lane >> 1] = p[0];
        __syncthreads();
        if (tid < 32 * (kPT / 64)) {
            const int c = tid / (kPT / 64), w = tid % (kPT / 64);
            const float sc = group_sum<kPT / 64>(red[b][w][c]);
            const float sig = group_sum<kPT / 64>(red[b][w][j]);
            const float x0 = piv[b][j];
            float t = 0.0f, beta = x0, scal = 1.0f;
            if (sig > 0.0f) {
                beta = -copysignf(sqrtf(__builtin_fmaf(x0, x0, sig)), x0);
                t = (beta - x0) / beta;
                scal = 1.0f / (x0 - beta);
            }
            const float wc = __builtin_fmaf(scal, sc, piv[b][c]);
            if (w == 0) {
                coef[b][c] = c > j ? t * wc : 0.0f;
                if (c < j) gv[c * 33 + j] = wc;
                if (c == 0) {
                    stepv[b][0] = scal;
                    stepv[b][1] = beta;
                    s_tau[j] = t;
                }
            }
        }
        __syncthreads();
        float cf[32];
#pragma unroll
        for (int c = 0; c < 32; ++c) cf[c] = coef[b][c];
        const float scal = stepv[b][0], beta = stepv[b][1];
        each([&](float* y, int i) {
            const int r = tid + i * kPT;
            const float yj = y[j];
            const float v = r > j ? scal * yj : (r == j ? 1.0f : 0.0f);
#pragma unroll
            for (int c = 0; c < 32; ++c) y[c] = __builtin_fmaf(-cf[c], v, y[c]);   // cf[j] = 0
            y[j] = r > j ? v : (r == j ? beta : yj);
        });
    }
    each([&](float* y, int i) {
        const int r = tid + i * kPT;
        if (r < rows) {
            float* dst = M + (int64_t)(k0 + r) * ldm + k0;
            if (nb == 32) {
#pragma unroll
                for (int c = 0; c < 32; ++c) dst[c] = y[c];
            } else {
#pragma unroll
                for (int c = 0; c < 32; ++c)
                    if (c < nb) dst[c] = y[c];
            }
        }
    });
    __syncthreads();
    if (tid < nb) tau[k0 + tid] = s_tau[tid];
    if (Tout && wave == 0 && lane < nb) form_t(lane, nb, gv, s_tau, Tout);
}

// Tiled trailing update, first half: for column tile x (kQB columns of the
// trailing block, from c0) and row block y (rpb rows of the panel), the
// partial Wp[y][i][x kQB + c] = sum over the block's rows r of V[r][i] C[r][c],
// V the panel's reflectors (unit diagonal, zero above it), C the trailing
// columns; padded columns and reflectors past nb hold zeros.  Rows pass
// through LDS 64 at a time (32 lanes per row, coalesced), the next 64 in
// registers meanwhile; thread (i, c4) owns W entries (i, 4 c4 .. 4 c4 + 3).
__global__ __launch_bounds__(256) void qr_upd_w_kernel(const float* M, int64_t ldm, int32_t rows_total, int32_t k0,
                                                       int32_t nb, int32_t c0, int32_t ncols, float* Wp, int64_t ncp,
                                                       int32_t rpb)
{
    __shared__ float Vs[64][kQB + 1];
    __shared__ float Cs[64][kQB + 1];
    const int rows = rows_total - k0;
    const int tid = threadIdx.x;
    const int cb0 = blockIdx.x * kQB;
    const int r_begin = blockIdx.y * rpb;
    const int r_end = min(r_begin + rpb, rows);
    const int oi = tid >> 3, oc = (tid & 7) * 4;
    const int lj = tid & 31, lr = tid >> 5;          // staging: column lj of rows lr, lr + 8, ...
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float pv[8], pc[8];
    auto fetch = [&](int rb) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int r = rb + lr + 8 * u;
            float v = 0.0f, c = 0.0f;
            if (r < r_end) {
                const float* row = M + (int64_t)(k0 + r) * ldm;
                if (lj < nb) v = r > lj ? row[k0 + lj] : (r == lj ? 1.0f : 0.0f);
                if (cb0 + lj < ncols) c = row[c0 + cb0 + lj];
            }
            pv[u] = v;
            pc[u] = c;
        }
    };
    if (r_begin < r_end) fetch(r_begin);
    for (int rb = r_begin; rb < r_end; rb += 64) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            Vs[lr + 8 * u][lj] = pv[u];
            Cs[lr + 8 * u][lj] = pc[u];
        }
        __syncthreads();
        if (rb + 64 < r_end) fetch(rb + 64);
#pragma unroll 8
        for (int rr = 0; rr < 64; ++rr) {
            const float v = Vs[rr][oi];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = __builtin_fmaf(v, Cs[rr][oc + q], acc[q]);
        }
        __syncthreads();
    }
    float* dst = Wp + ((int64_t)blockIdx.y * kQB + oi) * ncp + cb0 + oc;
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = acc[q];
}

// Second half: W = the nrb partials of the tile summed in row-block order,
// W2 = T^T W (T upper triangular, nb x nb row-major), then rows of the block
// eight at a time: lane c of row slot rr subtracts sum_i V[r][i] W2[i][c]
// from column c (the row's V staged in LDS, the tile's columns coalesced).
__global__ __launch_bounds__(256) void qr_upd_c_kernel(float* M, int64_t ldm, int32_t rows_total, int32_t k0,
                                                       int32_t nb, int32_t c0, int32_t ncols, const float* Wp,
                                                       int32_t nrb, int64_t ncp, const float* Tg)
{
    __shared__ float W[kQB][kQB + 1];
    __shared__ float W2[kQB][kQB + 1];
    __shared__ float Ts[kQB][kQB + 1];
    __shared__ float Vs[2][8][kQB + 1];
    const int rows = rows_total - k0;
    const int tid = threadIdx.x;
    const int cb0 = blockIdx.x * kQB;
    for (int e = tid; e < kQB * kQB; e += 256) {
        const int i = e >> 5, c = e & 31;
        float sum = 0.0f;
        for (int y = 0; y < nrb; ++y) sum += Wp[((int64_t)y * kQB + i) * ncp + cb0 + c];
        W[i][c] = sum;
        Ts[i][c] = (i < nb && c < nb) ? Tg[i * nb + c] : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < kQB * kQB; e += 256) {
        const int i = e >> 5, c = e & 31;
        float a = 0.0f;
        for (int l = 0; l <= i; ++l) a = __builtin_fmaf(Ts[l][i], W[l][c], a);
        W2[i][c] = a;
    }
    const int c = tid & 31, rr = tid >> 5;
    const bool live = cb0 + c < ncols;
    const int r_begin = blockIdx.y * kQR2, r_end = min(r_begin + kQR2, rows);
    int buf = 0;
    for (int rb = r_begin; rb < r_end; rb += 8, buf ^= 1) {
        const int r = rb + rr;
        float* row = M + (int64_t)(k0 + r) * ldm;
        float v = 0.0f, cv = 0.0f;
        if (r < r_end) {
            if (c < nb) v = r > c ? row[k0 + c] : (r == c ? 1.0f : 0.0f);
            if (live) cv = row[c0 + cb0 + c];
        }
        Vs[buf][rr][c] = v;
        __syncthreads();        // also orders W2 before its first use
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < kQB; ++i) a = __builtin_fmaf(Vs[buf][rr][i], W2[i][c], a);
        if (r < r_end && live) row[c0 + cb0 + c] = cv - a;
    }
}

// P = R^-1 (and P^T) by back substitution: wave w of workgroup b computes
// column j = 4 b + w, lane l holding x_k for k = l + 64 q, q < Q (64 Q >= n);
// rows of R are staged through LDS 16 at a time.  Four waves a workgroup
// spread the columns over n / 4 compute units.  The last workgroup stages
// all of R; if rfro2 is given it stores ||R||_F^2 there.
template <int Q>
__global__ __launch_bounds__(kTI) void trinv_kernel(const float* R, int64_t ldr, int32_t n, float* P, float* PT,
                                                     int64_t ldp, int32_t* bad, double* rfro2)
{
    extern __shared__ float rp[];        // [16][J]
    __shared__ double red[kTI / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x * (kTI / 64) + wave;
    const int J = min(n, (int)(blockIdx.x + 1) * (kTI / 64));
    double sq = 0.0;                     // squares of the staged entries (all of R in the last workgroup)
    float xv[Q];                         // x_k, k = lane + 64 q: zero until solved, and for k > j
#pragma unroll
    for (int q = 0; q < Q; ++q) xv[q] = 0.0f;
    bool ok = true;
    for (int hi = J - 1; hi >= 0; hi -= 16) {
        const int lo = max(0, hi - 15);
        __syncthreads();
        const int cnt = (hi - lo + 1) * J;
        for (int base = 0; base < cnt; base += 8 * kTI) {
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int idx = base + e * kTI + tid;
                const int rr = idx / J, k = idx - rr * J;
                const int i = lo + rr;
                v[e] = (idx < cnt && k >= i) ? R[(int64_t)i * ldr + k] : 0.0f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int idx = base + e * kTI + tid;
                if (idx < cnt) rp[idx] = v[e];
                sq = fma((double)v[e], (double)v[e], sq);
            }
        }
        __syncthreads();
        if (j < n) {
            for (int i = min(hi, j); i >= lo; --i) {
                // row[k] = 0 below the diagonal and x_k = 0 for k <= i or k > j,
                // so the sum over all staged k is the one over i < k <= j
                const float* row = rp + (i - lo) * J;
                float s = 0.0f;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const int k = lane + 64 * q;
                    if (64 * (q + 1) <= J || k < J) s = __builtin_fmaf(row[k], xv[q], s);
                }
                s = group_sum<64>(s);
                const float dgl = row[i];
                const float xi = ((i == j ? 1.0f : 0.0f) - s) / dgl;
                if (!(dgl != 0.0f) || !(fabsf(xi) <= 3.0e38f)) ok = false;
#pragma unroll
                for (int q = 0; q < Q; ++q)
                    if (lane + 64 * q == i) xv[q] = xi;
            }
        }
    }
    if (j < n) {
        for (int i = lane; i < n; i += 64) {
            float val = 0.0f;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (lane + 64 * q == i) val = xv[q];
            if (i > j) val = 0.0f;
            P[(int64_t)i * ldp + j] = val;
            PT[(int64_t)j * ldp + i] = val;
        }
        if (!ok && lane == 0) *bad = 1;
    }
    if (rfro2 && blockIdx.x == gridDim.x - 1) {
        const double t = block_sum<kTI>(sq, red);
        if (tid == 0) *rfro2 = t;
    }
}

// x = P z in FP64, z = the first n entries of column zc of M (Q^T Sb).
__global__ __launch_bounds__(kT) void x0_kernel(const float* PT, int64_t ldp, int32_t n, const float* M,
                                                 int64_t ldm, int32_t zc, double* x)
{
    __shared__ double z[kMaxN];
    __shared__ double out[kMaxN];
    __shared__ double tmp[kT];
    for (int j = threadIdx.x; j < n; j += kT) z[j] = (double)M[(int64_t)j * ldm + zc];
    __syncthreads();
    matvec_cols(PT, ldp, n, z, out, tmp);       // out_i = sum_j P[i][j] z_j
    for (int j = threadIdx.x; j < n; j += kT) x[j] = out[j];
}

// dst[0:n, 0:n+1] = the upper triangle of src's first n columns (zeros below
// the diagonal) beside src's column n, for rows 0..n-1.
__global__ void copy_upper_kernel(const float* src, int64_t lds_, float* dst, int64_t ldd, int32_t n)
{
    const int64_t total = (int64_t)n * (n + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / (n + 1);
        const int c = (int)(i - r * (n + 1));
        dst[r * ldd + c] = (c < n && c < r) ? 0.0f : src[r * lds_ + c];
    }
}

__global__ void cast_f64_f32_kernel(const double* in, float* out, int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}

__global__ void f16_to_f32_kernel(const uint16_t* in, int64_t ldi, float* out, int64_t ldo, int64_t rows,
                                  int32_t cols)
{
    const int64_t total = rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols;
        const int c = (int)(i - r * cols);
        out[r * ldo + c] = (float)__builtin_bit_cast(_Float16, in[r * ldi + c]);
    }
}

__global__ void init_state_kernel(SolveState* st, double tol, double inner_tol, int32_t max_inner, uint32_t* ticket)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        SolveState s{};
        s.tol = tol;
        s.inner_tol = inner_tol;
        s.max_inner = max_inner;
        s.inner_done = 1;
        *st = s;
        *ticket = 0u;
    }
}

// ------------------------------------------------------------ host side

int hip_err(hipError_t e, const char* what)
{
    return set_error(SK_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int panel_width(int64_t rows)
{
    const int64_t ldl = rows | 1;
    for (int nb : {32, 16, 8, 4, 2, 1})
        if (ldl * nb * 4 <= 150 * 1024) return nb;
    return 0;
}

hipError_t set_lds(const void* fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// In-place QR of the first k columns of M (rows x cols).
// Blocked Householder QR.  With T (a 32 x 32 FP32 device buffer, reused by
// every panel in stream order) the trailing update applies each panel as one
// block reflector; without it, reflector by reflector.
hipError_t run_qr(float* M, int64_t rows, int64_t cols, int64_t ldm, int64_t k, float* tau, float* T,
                  hipStream_t st)
{
    hipError_t e;
    for (int64_t k0 = 0; k0 < k; ) {
        const int64_t prow = rows - k0;
        const int32_t nb = (int32_t)std::min<int64_t>(panel_width(prow), k - k0);
        const size_t lds = (size_t)(prow | 1) * nb * 4;
        const int64_t c0 = k0 + nb, ncols = cols - c0;
        float* Tp = ncols > 0 ? T : (float*)nullptr;
        if (prow <= kPT) {
            hipLaunchKernelGGL(qr_panel_reg_kernel<1>, dim3(1), dim3(kPT), 0, st, M, ldm, (int32_t)rows,
                               (int32_t)k0, nb, tau, Tp);
        } else if (prow <= 2 * kPT) {
            hipLaunchKernelGGL(qr_panel_reg_kernel<2>, dim3(1), dim3(kPT), 0, st, M, ldm, (int32_t)rows,
                               (int32_t)k0, nb, tau, Tp);
        } else if (prow <= 4 * kPT) {
            hipLaunchKernelGGL(qr_panel_reg_kernel<4>, dim3(1), dim3(kPT), 0, st, M, ldm, (int32_t)rows,
                               (int32_t)k0, nb, tau, Tp);
        } else {
            if ((e = set_lds((const void*)qr_panel_kernel, lds)) != hipSuccess) return e;
            hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(kT), lds, st, M, ldm, (int32_t)rows, (int32_t)k0,
                               (int32_t)nb, tau, Tp);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ncols > 0) {
            // C -= V T^T (V^T C) in two tiled kernels: partial V^T C per
            // (column tile, row block) into the scratch after T, then the sum
            // of the partials in row-block order and the rank-nb update
            // up to kQNRB row blocks of a multiple of 64 rows: enough workgroups
            // for short panels, a few staged chunks each for tall ones
            const int64_t ncb = (ncols + kQB - 1) / kQB, ncp = ncb * kQB;
            const int64_t rpb = ((prow + kQNRB - 1) / kQNRB + 63) / 64 * 64;
            const int64_t nrb = (prow + rpb - 1) / rpb;
            if (nrb > kQNRB || nrb * kQB * ncp > kQRScratchFloats - kQB * kQB) return hipErrorInvalidValue;
            float* Wp = T + kQB * kQB;
            hipLaunchKernelGGL(qr_upd_w_kernel, dim3((unsigned)ncb, (unsigned)nrb), dim3(256), 0, st,
                               (const float*)M, ldm, (int32_t)rows, (int32_t)k0, (int32_t)nb, (int32_t)c0,
                               (int32_t)ncols, Wp, ncp, (int32_t)rpb);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL(qr_upd_c_kernel, dim3((unsigned)ncb, (unsigned)((prow + kQR2 - 1) / kQR2)), dim3(256),
                               0, st, M, ldm, (int32_t)rows, (int32_t)k0, (int32_t)nb, (int32_t)c0, (int32_t)ncols,
                               (const float*)Wp, (int32_t)nrb, ncp, (const float*)T);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        k0 += nb;
    }
    return hipSuccess;
}

hipError_t run_trinv(const float* R, int64_t ldr, int64_t n, float* P, float* PT, int64_t ldp, int32_t* bad,
                     double* rfro2, hipStream_t st)
{
    constexpr int W = kTI / 64;
    const int64_t grid = (n + W - 1) / W;
    const size_t lds = (size_t)16 * n * 4;          // the last workgroup stages 16 full rows
    const int q = n <= 64 ? 1 : n <= 128 ? 2 : n <= 256 ? 4 : n <= 512 ? 8 : 16;
    const void* fn = q == 1 ? (const void*)trinv_kernel<1> : q == 2 ? (const void*)trinv_kernel<2>
                   : q == 4 ? (const void*)trinv_kernel<4> : q == 8 ? (const void*)trinv_kernel<8>
                   : (const void*)trinv_kernel<16>;
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    const dim3 g((unsigned)grid), b(kTI);
    switch (q) {
    case 1: hipLaunchKernelGGL(trinv_kernel<1>, g, b, lds, st, R, ldr, (int32_t)n, P, PT, ldp, bad, rfro2); break;
    case 2: hipLaunchKernelGGL(trinv_kernel<2>, g, b, lds, st, R, ldr, (int32_t)n, P, PT, ldp, bad, rfro2); break;
    case 4: hipLaunchKernelGGL(trinv_kernel<4>, g, b, lds, st, R, ldr, (int32_t)n, P, PT, ldp, bad, rfro2); break;
    case 8: hipLaunchKernelGGL(trinv_kernel<8>, g, b, lds, st, R, ldr, (int32_t)n, P, PT, ldp, bad, rfro2); break;
    default: hipLaunchKernelGGL(trinv_kernel<16>, g, b, lds, st, R, ldr, (int32_t)n, P, PT, ldp, bad, rfro2); break;
    }
    return hipGetLastError();
}

// Row-pass geometry: C elements (16 bytes) per lane chunk, LR lanes per row,
// CP chunks per lane.
struct Geo {
    int LR = 0, CP = 0, mask = 0;
};

Geo row_geometry(int esz, int64_t n)
{
    const int C = 16 / esz;
    const int64_t nc = (n + C - 1) / C;
    Geo g;
    if (nc <= 64) {
        int lr = 1;
        while (lr < nc) lr <<= 1;
        g.LR = lr;
        g.CP = 1;
    } else {
        g.LR = 64;
        g.CP = nc <= 128 ? 2 : 4;
    }
    g.mask = ((int64_t)g.LR * g.CP * C != n) ? 1 : 0;
    return g;
}

template <typename AT, int LR, int CP>
hipError_t launch_rows_t(bool resid, const RowArgs& a, int nwg, hipStream_t st)
{
    const size_t lds = row_lds_bytes(a.n, resid);
    const void* fn = resid ? (const void*)resid_pass<AT, LR, CP> : (const void*)lsqr_pass<AT, LR, CP>;
    hipError_t e = set_lds(fn, lds);
    if (e != hipSuccess) return e;
    if (resid)
        hipLaunchKernelGGL((resid_pass<AT, LR, CP>), dim3(nwg), dim3(kT), lds, st, a);
    else
        hipLaunchKernelGGL((lsqr_pass<AT, LR, CP>), dim3(nwg), dim3(kT), lds, st, a);
    return hipGetLastError();
}

template <typename AT>
hipError_t launch_rows_g(bool resid, const Geo& g, const RowArgs& a, int nwg, hipStream_t st)
{
    if (g.CP == 1) {
        switch (g.LR) {
            case 1: return launch_rows_t<AT, 1, 1>(resid, a, nwg, st);
            case 2: return launch_rows_t<AT, 2, 1>(resid, a, nwg, st);
            case 4: return launch_rows_t<AT, 4, 1>(resid, a, nwg, st);
            case 8: return launch_rows_t<AT, 8, 1>(resid, a, nwg, st);
            case 16: return launch_rows_t<AT, 16, 1>(resid, a, nwg, st);
            case 32: return launch_rows_t<AT, 32, 1>(resid, a, nwg, st);
            default: return launch_rows_t<AT, 64, 1>(resid, a, nwg, st);
        }
    }
    if (g.CP == 2) return launch_rows_t<AT, 64, 2>(resid, a, nwg, st);
    if constexpr (ET<AT>::B == 4) return launch_rows_t<AT, 64, 4>(resid, a, nwg, st);
    return hipErrorInvalidValue;   // 16-bit rows of n <= 1024 need at most two chunks per lane
}

hipError_t launch_rows(int a_dtype, bool resid, const Geo& g, const RowArgs& a, int nwg, hipStream_t st)
{
    if (a_dtype == SK_F32) return launch_rows_g<float>(resid, g, a, nwg, st);
    if (a_dtype == SK_F16) return launch_rows_g<__half>(resid, g, a, nwg, st);
    return launch_rows_g<__hip_bfloat16>(resid, g, a, nwg, st);
}

}  // namespace

// ------------------------------------------------------------ solve jobs

// One least-squares solve as a resumable sequence of asynchronous phases on
// one stream.  job_step() never blocks unless asked to: it looks at the event
// recorded after the last state copy and, once the device is there, reads
// the state and enqueues the next phase.  sketch_solve drives one job to the
// end; the request server keeps one job per slot and interleaves them.
constexpr size_t kNoWs = ~(size_t)0;

struct SolveJob {
    // problem
    sk_sketch S;                 // the S of A (its large-d/s workspace is the job's own)
    sk_sketch Sb;                // the same S in FP32 mode, for b
    const void* A = nullptr;
    int32_t a_dtype = 0;
    int64_t n = 0, lda = 0;
    const double* b = nullptr;
    double* x = nullptr;
    sk_solve_opts o{};
    // plan
    bool f16 = false;
    int64_t ldm = 0, ld16 = 0;
    int nwg = 0;
    Geo geo;
    RowArgs ra{};
    size_t oM = 0, o16 = 0, ob32 = 0, ou = 0, oP = 0, oPT = 0, otau = 0, ot = 0, ov = 0, ow = 0, oy = 0, opart = 0,
           ost = 0, otk = 0, oTq = 0, total = 0;
    size_t ows = kNoWs, owsb = kNoWs;  // sketch workspaces in the block (large d/s), or none
    size_t ws_floats = 0, wsb_floats = 0;   // their sizes in FP32 words (with the gather's lists)
    int32_t qr_blocks = 1;              // row blocks of a two-level QR (d above kQRRows)
    int64_t qr_rows = 0;                // rows per block
    size_t oZ = 0;                      // the stacked triangles [R_1 c_1; ...; R_B c_B]
    // device binding
    hipStream_t st = nullptr;
    char* base = nullptr;
    float* Mw = nullptr;
    float* Z = nullptr;
    uint16_t* SA16 = nullptr;
    float* b32 = nullptr;
    float* tau = nullptr;
    float* Tq = nullptr;         // QR scratch: the panel's 32 x 32 block-reflector factor, then update partials
    // host resources (kept across reuses)
    SolveState* host = nullptr;  // pinned
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_state = nullptr;
    uint32_t recorded = 0;       // bit i: ev[i] recorded in this run
    // progress
    int phase = 0;               // 0 idle, 1 residual in flight, 2 LSQR in flight, 3 finishing, 4 done
    int k = 0, launched = 0, steps = 0;
    double rel0 = 0.0;
    bool converged = false;
    int rc = SK_OK;
};

SolveJob* job_new() { return new (std::nothrow) SolveJob; }

void job_delete(SolveJob* j)
{
    if (!j) return;
    if (j->host) (void)hipHostFree(j->host);
    for (hipEvent_t& e : j->ev)
        if (e) (void)hipEventDestroy(e);
    if (j->ev_state) (void)hipEventDestroy(j->ev_state);
    delete j;
}

// Validate and plan; no device memory is touched.  *footprint = device bytes
// the job needs at its base pointer.
int job_prepare(SolveJob* j, const sk_sketch& S, const void* A, int32_t a_dtype, int64_t n, int64_t lda,
                const double* b, double* x, const sk_solve_opts* opts, size_t* footprint)
{
    const int esz = a_dtype == SK_F32 ? 4 : (a_dtype == SK_F16 || a_dtype == SK_BF16) ? 2 : 0;
    if (!esz) return set_error(SK_EINVAL, "unknown element type %d", a_dtype);
    if (n < 1 || lda < n) return set_error(SK_EINVAL, "bad shape n=%lld lda=%lld", (long long)n, (long long)lda);
    if (n > S.d) return set_error(SK_EINVAL, "n = %lld exceeds the sketch size d = %lld", (long long)n,
                                  (long long)S.d);
    if (n > kMaxN) return set_error(SK_EUNSUPPORTED, "n = %lld > %d", (long long)n, kMaxN);
    if (S.d > kMaxD) return set_error(SK_EUNSUPPORTED, "d = %lld > %lld", (long long)S.d, (long long)kMaxD);
    if (!A || !b || !x) return set_error(SK_EINVAL, "NULL array");
    if ((uintptr_t)A % (uintptr_t)esz) return set_error(SK_EINVAL, "A is not element aligned");
    if (((uintptr_t)b | (uintptr_t)x) & 7u) return set_error(SK_EINVAL, "b and x must be 8-byte aligned");
    sk_solve_opts o{};
    if (opts) {
        o = *opts;
        for (int i = 0; i < 3; ++i)
            if (o.reserved[i]) return set_error(SK_EINVAL, "reserved option fields must be zero");
        if (o.tol < 0 || o.inner_tol < 0 || o.max_refine < 0 || o.max_inner < 0)
            return set_error(SK_EINVAL, "negative option");
    }
    if (o.tol == 0) o.tol = 1e-10;
    if (o.inner_tol == 0) o.inner_tol = 1e-6;
    if (o.max_refine == 0) o.max_refine = 10;
    if (o.max_inner == 0) o.max_inner = 100;

    DeviceInfo dev;
    int rc = device_info(&dev);
    if (rc) return rc;
    const int64_t m = S.m, d = S.d;
    const int64_t nwg0 = std::max<int64_t>(1, std::min<int64_t>(dev.cus, (m + 1023) / 1024));
    const int64_t rpw = (m + nwg0 - 1) / nwg0;
    if (rpw * lda * esz >= ((int64_t)1 << 31))
        return set_error(SK_EUNSUPPORTED, "rows per workgroup span more than 2 GiB");
    j->S = S;
    j->S.ws = nullptr;                           // never the caller's handle workspace
    j->S.ws_floats = 0;
    j->S.ws_borrowed = true;                     // set from the job's block at start
    j->S.sw = nullptr;
    j->Sb = sk_sketch{};
    j->Sb.ws_borrowed = true;
    j->Sb.m = S.m;
    j->Sb.d = S.d;
    j->Sb.s = S.s;
    j->Sb.seed = S.seed;
    j->Sb.rounding = SK_ACC_F32;
    j->A = A;
    j->a_dtype = a_dtype;
    j->n = n;
    j->lda = lda;
    j->b = b;
    j->x = x;
    j->o = o;
    if (S.rounding >= SK_ACC_BF16_RN) return set_error(SK_EUNSUPPORTED, "sketch_solve takes FP32 or FP16 sketches");
    j->f16 = S.rounding != SK_ACC_F32;
    j->ldm = n + 1;
    j->ld16 = (n + 1) / 2 * 2;
    j->nwg = (int)((m + rpw - 1) / rpw);          // every workgroup owns at least one row
    j->geo = row_geometry(esz, n);
    const int pst = (int)((n + 3 + 3) / 4 * 4);

    size_t off = 0;
    auto take = [&](size_t b2) { const size_t at = off; off = align_up(off + b2, 256); return at; };
    j->oM = take((size_t)d * j->ldm * 4);
    j->o16 = j->f16 ? take((size_t)d * j->ld16 * 2) : 0;
    j->ob32 = take((size_t)m * 4);
    j->ou = take((size_t)m * 4);
    j->oP = take((size_t)n * n * 4);
    j->oPT = take((size_t)n * n * 4);
    j->otau = take((size_t)n * 4 + 4);
    j->oTq = take((size_t)kQRScratchFloats * 4);
    // Sketches taller than one QR: factor row blocks of at most kQRRows rows,
    // stack their triangles (with the transformed Sb) and factor the stack.
    j->qr_blocks = (int32_t)((d + kQRRows - 1) / kQRRows);
    j->qr_rows = (d + j->qr_blocks - 1) / j->qr_blocks;
    if (j->qr_blocks > 1) {
        if (j->qr_rows < n + 1 || (int64_t)j->qr_blocks * n > kQRRows)
            return set_error(SK_EUNSUPPORTED, "d = %lld with n = %lld: the stacked triangles exceed %lld rows",
                             (long long)d, (long long)n, (long long)kQRRows);
        j->oZ = take((size_t)j->qr_blocks * n * (n + 1) * 4);
    }
    j->ot = take((size_t)n * 4);
    j->ov = take((size_t)n * 8);
    j->ow = take((size_t)n * 8);
    j->oy = take((size_t)n * 8);
    j->opart = take((size_t)j->nwg * pst * 8);
    j->ost = take(sizeof(SolveState));
    j->otk = take(64);
    // Sketches whose d/s rows do not fit in LDS sum in a d x n FP32
    // workspace; it is carved from the job's block so admission by
    // footprint stays honest and a job never allocates.
    {
        DeviceInfo dv = dev;
        Plan pa, pb;
        j->ws_floats = (make_plan(&j->S, a_dtype, m, n, lda, dv, &pa) == SK_OK) ? plan_ws_floats(pa, d, n, m, S.s) : 0;
        j->wsb_floats = (make_plan(&j->Sb, SK_F32, m, 1, 1, dv, &pb) == SK_OK) ? plan_ws_floats(pb, d, 1, m, S.s) : 0;
        j->ows = j->ws_floats ? take(j->ws_floats * 4) : kNoWs;
        j->owsb = j->wsb_floats ? take(j->wsb_floats * 4) : kNoWs;
        set_error(SK_OK, "");
    }
    j->total = off;

    RowArgs& ra = j->ra;
    ra = RowArgs{};
    ra.A = A;
    ra.lda = lda;
    ra.m = m;
    ra.rpw = rpw;
    ra.n = (int32_t)n;
    ra.vec = ((lda * esz) % 16 == 0 && (uintptr_t)A % 16 == 0) ? 1 : 0;
    ra.mask = j->geo.mask;
    ra.b = b;
    ra.x = x;
    ra.ldp = n;
    ra.pst = pst;
    j->phase = 0;
    *footprint = j->total;
    return SK_OK;
}

namespace {

hipError_t job_record(SolveJob* j, int i)
{
    const hipError_t e = hipEventRecord(j->ev[i], j->st);
    if (e == hipSuccess) j->recorded |= 1u << i;
    return e;
}

int job_fail(SolveJob* j, int rc)
{
    j->rc = rc;
    j->phase = 4;
    return rc;
}

// Copy the device state to the pinned slot and mark the point to wait for.
int job_mark(SolveJob* j)
{
    hipError_t e = hipMemcpyAsync(j->host, j->ra.st, sizeof(SolveState), hipMemcpyDeviceToHost, j->st);
    if (e == hipSuccess) e = hipEventRecord(j->ev_state, j->st);
    return e == hipSuccess ? SK_OK : hip_err(e, "reading the solver state");
}

int job_lsqr_batch(SolveJob* j)
{
    const int batch = std::min(8, j->o.max_inner - j->launched);
    for (int i = 0; i < batch; ++i) {
        hipError_t e = launch_rows(j->a_dtype, false, j->geo, j->ra, j->nwg, j->st);
        if (e != hipSuccess) return hip_err(e, "LSQR pass");
    }
    j->launched += batch;
    return job_mark(j);
}

int job_resid(SolveJob* j)
{
    j->ra.first = j->k == 0 ? 1 : 0;
    hipError_t e = launch_rows(j->a_dtype, true, j->geo, j->ra, j->nwg, j->st);
    if (e != hipSuccess) return hip_err(e, "residual pass");
    return job_mark(j);
}

}  // namespace

// Bind the job to device memory (>= its footprint, 256-byte aligned) and a
// stream, and enqueue sketch, factorisation and the first residual pass.
int job_start(SolveJob* j, void* device_base, hipStream_t st)
{
    hipError_t e;
    if (!j->host) {
        if ((e = hipHostMalloc((void**)&j->host, sizeof(SolveState), hipHostMallocDefault)) != hipSuccess) {
            j->host = nullptr;
            return set_error(SK_ENOMEM, "pinned status: %s", hipGetErrorString(e));
        }
        for (hipEvent_t& ev : j->ev)
            if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_err(e, "hipEventCreate");
        if ((e = hipEventCreateWithFlags(&j->ev_state, hipEventDisableTiming)) != hipSuccess)
            return hip_err(e, "hipEventCreate");
    }
    j->st = st;
    j->base = (char*)device_base;
    char* base = j->base;
    j->Mw = (float*)(base + j->oM);
    j->SA16 = (uint16_t*)(base + j->o16);
    j->b32 = (float*)(base + j->ob32);
    j->tau = (float*)(base + j->otau);
    j->Tq = (float*)(base + j->oTq);
    j->Z = j->qr_blocks > 1 ? (float*)(base + j->oZ) : nullptr;
    RowArgs& ra = j->ra;
    ra.u = (float*)(base + j->ou);
    ra.t = (float*)(base + j->ot);
    ra.M = (const float*)(base + j->oP);        // P, then M = P P^T in the same place
    ra.PT = (const float*)(base + j->oPT);
    ra.tv = (double*)(base + j->ov);
    ra.W = (double*)(base + j->ow);
    ra.Y = (double*)(base + j->oy);
    ra.part = (double*)(base + j->opart);
    ra.st = (SolveState*)(base + j->ost);
    ra.ticket = (uint32_t*)(base + j->otk);
    j->S.ws = j->ows != kNoWs ? (float*)(base + j->ows) : nullptr;
    j->S.ws_floats = j->ows != kNoWs ? j->ws_floats : 0;
    j->Sb.ws = j->owsb != kNoWs ? (float*)(base + j->owsb) : nullptr;
    j->Sb.ws_floats = j->owsb != kNoWs ? j->wsb_floats : 0;
    j->k = 0;
    j->launched = 0;
    j->steps = 0;
    j->rel0 = 0.0;
    j->converged = false;
    j->rc = SK_OK;
    j->recorded = 0;
    (void)hipGetLastError();                    // errors reported below are this job's own
    std::memset(j->host, 0, sizeof(SolveState));
    const int64_t m = j->S.m, d = j->S.d, n = j->n;
    int rc;

    // ---- sketch
    if ((e = job_record(j, 0)) != hipSuccess) return job_fail(j, hip_err(e, "hipEventRecord"));
    hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(64), 0, st, ra.st, j->o.tol, j->o.inner_tol, j->o.max_inner,
                       ra.ticket);
    if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "init kernel"));
    if (j->f16) {
        rc = sketch_apply(&j->S, j->A, j->a_dtype, m, n, j->lda, 0, j->SA16, j->ld16, 0, j->o.round_epoch, st);
        if (rc) return job_fail(j, rc);
        hipLaunchKernelGGL(f16_to_f32_kernel, dim3(256), dim3(256), 0, st, (const uint16_t*)j->SA16, j->ld16, j->Mw,
                           j->ldm, d, (int32_t)n);
        if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "convert kernel"));
    } else {
        rc = sketch_apply(&j->S, j->A, j->a_dtype, m, n, j->lda, 0, j->Mw, j->ldm, 0, j->o.round_epoch, st);
        if (rc) return job_fail(j, rc);
    }
    hipLaunchKernelGGL(cast_f64_f32_kernel, dim3(1024), dim3(256), 0, st, j->b, j->b32, m);
    if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "cast kernel"));
    rc = sketch_apply(&j->Sb, j->b32, SK_F32, m, 1, 1, 0, j->Mw + n, j->ldm, 0, 0, st);
    if (rc) return job_fail(j, rc);
    if ((e = job_record(j, 1)) != hipSuccess) return job_fail(j, hip_err(e, "hipEventRecord"));

    // ---- factor: QR of [SA | Sb], P = R^-1, x0 = P Q^T Sb
    if (j->qr_blocks == 1) {
        if ((e = run_qr(j->Mw, d, n + 1, j->ldm, n, j->tau, j->Tq, st)) != hipSuccess)
            return job_fail(j, hip_err(e, "QR kernels"));
    } else {
        // two-level QR: [R c] of the stacked blocks' [R_i c_i] equals that of [SA | Sb]
        const int64_t ldz = n + 1;
        for (int32_t i = 0; i < j->qr_blocks; ++i) {
            const int64_t r0 = (int64_t)i * j->qr_rows, rows = std::min<int64_t>(j->qr_rows, d - r0);
            if ((e = run_qr(j->Mw + r0 * j->ldm, rows, n + 1, j->ldm, n, j->tau, j->Tq, st)) != hipSuccess)
                return job_fail(j, hip_err(e, "QR kernels"));
            hipLaunchKernelGGL(copy_upper_kernel, dim3(256), dim3(256), 0, st, (const float*)(j->Mw + r0 * j->ldm),
                               j->ldm, j->Z + (int64_t)i * n * ldz, ldz, (int32_t)n);
            if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "stack kernel"));
        }
        if ((e = run_qr(j->Z, (int64_t)j->qr_blocks * n, n + 1, ldz, n, j->tau, j->Tq, st)) != hipSuccess)
            return job_fail(j, hip_err(e, "QR kernels"));
        hipLaunchKernelGGL(copy_upper_kernel, dim3(256), dim3(256), 0, st, (const float*)j->Z, ldz, j->Mw, j->ldm,
                           (int32_t)n);
        if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "stack kernel"));
    }
    if ((e = run_trinv(j->Mw, j->ldm, n, (float*)ra.M, (float*)ra.PT, n, &ra.st->bad, &ra.st->rfro2, st)) != hipSuccess)
        return job_fail(j, hip_err(e, "inverse kernel"));
    hipLaunchKernelGGL(gram_kernel, dim3((unsigned)((n + 15) / 16), (unsigned)((n + 15) / 16)), dim3(256), 0, st,
                       ra.PT, (int64_t)n, (int32_t)n, (float*)ra.M);
    if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "Gram kernel"));
    hipLaunchKernelGGL(x0_kernel, dim3(1), dim3(kT), 0, st, ra.PT, (int64_t)n, (int32_t)n, (const float*)j->Mw,
                       j->ldm, (int32_t)n, j->x);
    if ((e = hipGetLastError()) != hipSuccess) return job_fail(j, hip_err(e, "x0 kernel"));
    if ((e = job_record(j, 2)) != hipSuccess) return job_fail(j, hip_err(e, "hipEventRecord"));

    // ---- first residual
    if ((rc = job_resid(j))) return job_fail(j, rc);
    j->phase = 1;
    return SK_OK;
}

// Advance the job.  Returns 1 while work is in flight, SK_OK when finished
// successfully (or SK_ENOTCONV), another negative code on failure.
int job_step(SolveJob* j, bool block)
{
    for (;;) {
        if (j->phase == 4) return j->rc;
        if (j->phase == 0) return set_error(SK_EINVAL, "solve job not started");
        hipEvent_t wait = j->phase == 3 ? j->ev[3] : j->ev_state;
        hipError_t e;
        if (block) {
            e = hipEventSynchronize(wait);
        } else {
            e = hipEventQuery(wait);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();            // not an error: leave no trace for later launch checks
                return 1;
            }
        }
        if (e != hipSuccess) return job_fail(j, hip_err(e, "waiting for the solver"));
        SolveState* h = j->host;
        int rc;
        if (j->phase == 3) {
            j->phase = 4;
            if (!j->converged)
                j->rc = set_error(SK_ENOTCONV, "not converged after %d refinement steps: criterion %.3e > %.3e",
                                  j->steps, h->crit, j->o.tol);
            return j->rc;
        }
        if (h->bad) {
            return job_fail(j, set_error(SK_EINVAL, j->phase == 1 && j->k == 0
                                                        ? "SA is numerically rank deficient (zero or non-finite pivot)"
                                                        : "the solver produced a non-finite value"));
        }
        bool finish = false;
        if (j->phase == 1) {
            if (j->k == 0) j->rel0 = h->rel;
            j->steps = j->k;
            if (h->outer_done) {
                j->converged = true;
                finish = true;
            } else if (j->k == j->o.max_refine) {
                finish = true;
            } else {
                j->launched = 0;
                if ((rc = job_lsqr_batch(j))) return job_fail(j, rc);
                j->phase = 2;
            }
        } else {   // phase 2: a batch of LSQR iterations
            if (h->inner_done || j->launched >= j->o.max_inner) {
                ++j->k;
                if ((rc = job_resid(j))) return job_fail(j, rc);
                j->phase = 1;
            } else if ((rc = job_lsqr_batch(j))) {
                return job_fail(j, rc);
            }
        }
        if (finish) {
            if ((e = job_record(j, 3)) != hipSuccess) return job_fail(j, hip_err(e, "hipEventRecord"));
            j->phase = 3;
        }
        if (!block) return 1;
    }
}

void job_info(const SolveJob* j, sk_solve_info* info)
{
    std::memset(info, 0, sizeof(*info));
    if (j->phase != 4) return;
    const SolveState* h = j->host;
    info->converged = j->converged ? 1 : 0;
    info->refine_steps = j->steps;
    info->inner_iters = h->total_inner;
    info->crit = h->crit;
    info->rel_residual = h->rel;
    info->rel_residual_x0 = j->rel0;
    auto span = [&](int a, int b, double* out) {
        const uint32_t need = (1u << a) | (1u << b);
        float ms = 0;
        if ((j->recorded & need) == need && hipEventElapsedTime(&ms, j->ev[a], j->ev[b]) == hipSuccess) *out = ms;
    };
    span(0, 1, &info->ms_sketch);
    span(1, 2, &info->ms_factor);
    span(2, 3, &info->ms_refine);
    span(0, 3, &info->ms_total);
    (void)hipGetLastError();
}

// Device workspace of sketch_solve, grown on demand, and its job.
struct SolveWs {
    int device = -1;
    void* base = nullptr;
    size_t bytes = 0;
    SolveJob* job = nullptr;
};

void solve_release(sk_sketch* h)
{
    if (!h || !h->sw) return;
    SolveWs* w = h->sw;
    if (w->base) (void)hipFree(w->base);
    job_delete(w->job);
    delete w;
    h->sw = nullptr;
}

}  // namespace sk

using namespace sk;

extern "C" {

int sketch_qr_f32(float* M, int64_t rows, int64_t cols, int64_t ldm, int64_t k, float* tau, void* stream)
{
    if (!M || !tau) return set_error(SK_EINVAL, "NULL argument");
    if (rows < 1 || cols < 1 || ldm < cols || k < 0 || k > rows || k > cols)
        return set_error(SK_EINVAL, "bad shape rows=%lld cols=%lld ldm=%lld k=%lld", (long long)rows,
                         (long long)cols, (long long)ldm, (long long)k);
    if (rows > kQRRows || cols > kMaxN + 1)
        return set_error(SK_EUNSUPPORTED, "rows <= %lld and cols <= %d", (long long)kQRRows, kMaxN + 1);
    if (k == 0) return SK_OK;
    // the block reflectors' 32 x 32 factor and the update's partials,
    // allocated in stream order
    hipStream_t st = (hipStream_t)stream;
    float* T = nullptr;
    hipError_t e = hipMallocAsync((void**)&T, (size_t)kQRScratchFloats * 4, st);
    if (e != hipSuccess) return set_error(SK_ENOMEM, "QR factor buffer: %s", hipGetErrorString(e));
    e = run_qr(M, rows, cols, ldm, k, tau, T, st);
    const hipError_t ef = hipFreeAsync(T, st);
    if (e == hipSuccess) e = ef;
    return e == hipSuccess ? SK_OK : hip_err(e, "QR kernels");
}

int sketch_trinv_f32(const float* R, int64_t n, int64_t ldr, float* P, float* PT, int64_t ldp, int32_t* bad,
                     void* stream)
{
    if (!R || !P || !PT || !bad) return set_error(SK_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxN || ldr < n || ldp < n) return set_error(SK_EINVAL, "bad shape n=%lld", (long long)n);
    hipError_t e = run_trinv(R, ldr, n, P, PT, ldp, bad, nullptr, (hipStream_t)stream);
    return e == hipSuccess ? SK_OK : hip_err(e, "inverse kernel");
}

int sketch_solve(sk_handle h, const void* A, int32_t a_dtype, int64_t n, int64_t lda, const double* b, double* x,
                 const sk_solve_opts* opts, sk_solve_info* info, void* stream)
{
    if (!h) return set_error(SK_EINVAL, "handle is NULL");
    SolveJob probe;
    size_t need = 0;
    int rc = job_prepare(&probe, *h, A, a_dtype, n, lda, b, x, opts, &need);
    if (rc) return rc;
    if (!h->sw) {
        h->sw = new (std::nothrow) SolveWs;
        if (!h->sw) return set_error(SK_ENOMEM, "out of host memory");
        h->sw->job = job_new();
        if (!h->sw->job) return set_error(SK_ENOMEM, "out of host memory");
    }
    SolveWs* w = h->sw;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice");
    if (w->bytes < need || w->device != dev) {
        if (w->base) (void)hipFree(w->base);
        w->base = nullptr;
        w->bytes = 0;
        if ((e = hipMalloc(&w->base, need)) != hipSuccess)
            return set_error(SK_ENOMEM, "solve workspace of %zu bytes: %s", need, hipGetErrorString(e));
        w->bytes = need;
        w->device = dev;
    }
    SolveJob* j = w->job;
    if ((rc = job_prepare(j, *h, A, a_dtype, n, lda, b, x, opts, &need))) return rc;
    if ((rc = job_start(j, w->base, (hipStream_t)stream))) return rc;
    rc = job_step(j, true);
    if (info) job_info(j, info);
    return rc;
}

}  // extern "C"
