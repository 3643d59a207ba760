/*
 * sketch.h -- C ABI of libsketch.so, an MI355X (gfx950) library that applies
 * sparse oblivious subspace embeddings to tall matrices.
 *
 * Method: "Randomized Sketching is Robust to Low-Precision Rounding on GPUs"
 * (Jeendgar, Flint, Anzt).  Given A (m x n, m >> n) and a random S (d x m),
 * form SA (Section 1; Section 2.1).  S is a SparseStack matrix: s stacked
 * CountSketch blocks of d/s rows, one nonzero +-1/sqrt(s) per block and
 * column (Section 2.2, SparseStack definition; block ranges and the value
 * scale in Section 4.1); s = 1 is CountSketch (Section 2.2).  SA is
 * accumulated in FP32, or in FP16 with one of three rounding rules:
 * round-to-nearest, exact stochastic rounding, dithered rounding (Section
 * 2.3; Section 4.2).
 *
 * Conventions
 *  - Every function returns SK_OK (0) or a negative SK_E* code; the message
 *    of the last failure on the calling thread is in sketch_last_error().
 *  - Matrices are row-major with an explicit leading dimension in elements.
 *  - Pointers named A, SA, x, out, buckets, signs are DEVICE pointers owned by
 *    the caller; the library never frees or keeps them past the call.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    asynchronously; HIP errors of a launch are returned when detected at
 *    launch time, later asynchronous faults surface on a later call.
 *  - Argument checks run before any HIP call, so invalid calls fail the same
 *    way on a machine without a GPU.
 *  - A handle may be used by one thread at a time; distinct handles are
 *    independent.
 */
#ifndef SKETCH_H
#define SKETCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define SK_OK            0
#define SK_EINVAL       -1   /* bad argument (shape, pointer, flag, code)     */
#define SK_EUNSUPPORTED -2   /* valid but not supported (alignment, size)     */
#define SK_ENOMEM       -3   /* device allocation failed                      */
#define SK_EHIP         -4   /* a HIP runtime call failed                     */
#define SK_ENOTCONV     -5   /* sketch_solve: stopping test not reached       */
#define SK_EADMIT       -6   /* request larger than the server's memory budget */
#define SK_EBUSY        -7   /* server shutting down                          */

/* ---- element types ----------------------------------------------------- */
#define SK_F32  0
#define SK_F16  1
#define SK_BF16 2

/* ---- accumulation of SA (fixed per handle) ----------------------------- */
#define SK_ACC_F32        0  /* SA is FP32                                    */
#define SK_ACC_F16_RN     1  /* SA is FP16, round-to-nearest-even            */
#define SK_ACC_F16_SR     2  /* SA is FP16, exact stochastic rounding        */
#define SK_ACC_F16_DITHER 3  /* SA is FP16, dithered rounding                */
#define SK_ACC_BF16_RN    4  /* SA is BF16, round-to-nearest-even            */
#define SK_ACC_BF16_SR    5  /* SA is BF16, exact stochastic rounding        */
#define SK_ACC_BF16_DITHER 6 /* SA is BF16, dithered rounding (2^-7 scale)   */

/* ---- sketch_apply flags ------------------------------------------------ */
#define SK_ACCUMULATE 1u     /* SA += S*A instead of SA = S*A                 */

typedef struct sk_sketch *sk_handle;

/*
 * Work decomposition of one sketch_apply call.  Rows are cut into units of
 * `chunk_rows` consecutive rows; each unit is summed by one workgroup per
 * column tile (and per group of `block_group` SparseStack blocks) into an
 * FP32 partial (an integer fixed-point sum in LDS, decoded once) and then
 * added into SA once.  In the FP16 modes each unit's partial is scaled
 * by fl32(1/sqrt(s)), rounded to FP16 with the handle's rule, and added with
 * FP16 round-to-nearest atomics, so `chunk_rows` fixes the rounding sites:
 * site q of entry (b, c) in the unit starting at global row r0 is
 * q = r0*d*n + b*n + c.  Zero fields mean "choose automatically".
 */
typedef struct sk_schedule {
    int32_t chunk_rows;   /* rows per unit, a multiple of 64                  */
    int32_t block_group;  /* blocks per workgroup: 1, 2, 4 or 8, dividing s   */
    int32_t waves;        /* waves (64 lanes) per workgroup: 4, 8 or 16       */
    int32_t xcd_remap;    /* 1: place all tiles of a unit on one XCD; 0: off  */
    int32_t per_contribution; /* 1: the paper's kernel scheme, see below      */
    int32_t col_tile;     /* columns per workgroup tile: 32, 8, 4 or 2; with  */
                          /* 32: block_group 1, 2, 4 or 8; 8: 1, 2 or 4;      */
                          /* 4: 1 or 2; 2: 1.  Narrow tiles fit larger d/s   */
                          /* in LDS and waste no lanes when n is small        */
    int32_t global_atomics; /* 1: no LDS partials: the call's contributions   */
                          /* go by FP32 global atomics into a d x n workspace */
    int32_t gather;       /* 1: no LDS partials and no value atomics: rows    */
                          /* are listed by bucket (counting sort of the hash) */
                          /* and one wave per SA row chunk sums its listed    */
                          /* rows in FP64 into the d x n workspace.  Reads A  */
                          /* s times; the planner takes it when d/s leaves    */
                          /* only narrow tiles (or none) in LDS for rows of   */
                          /* 256 bytes or more, or when no tile fits at all   */
    int32_t reserved[1];  /* must be zero                                     */
} sk_schedule;

/*
 * per_contribution = 1 replaces the workgroup partials by one global atomic
 * per contribution, the scheme of the paper's Section 4 kernels: for every
 * row i, block j and column c the FP32 value fl32(rho_ij * fl32(1/sqrt(s)) *
 * A[i][c]) is added to SA[b_ij][c] -- in FP32 mode with an FP32 atomic
 * (Section 4.1), in the FP16 modes after rounding it to FP16 with the
 * handle's rule and with packed FP16 atomics on column pairs (Section 4.2),
 * so m*n*s values are rounded and summed in FP16 in an unspecified order.
 * SR and dither take site q = (i*s + j)*n + c of the rounding stream.  The
 * other schedule fields are ignored; single sketches only (not batches).
 * It is a reference for accuracy and atomic counts, far slower than the
 * partial-sum scheme, and the planner never picks it.
 */

/*
 * sketch_create -- describe S (d x m) once.
 *   m        >= 1, number of columns of S (rows of the full A).
 *   d        >= 1, sketch rows; d % s == 0 (Section 4.1 assumes it).
 *   s        1..16, nonzeros per column (the paper's zeta).
 *   seed     64-bit key of the row hash; S is a pure function of (m, d, s,
 *            seed) and hash version 1, never stored.
 *   rounding SK_ACC_F32 / SK_ACC_F16_RN / SK_ACC_F16_SR / SK_ACC_F16_DITHER,
 *            or SK_ACC_BF16_RN / SK_ACC_BF16_SR / SK_ACC_BF16_DITHER (BF16
 *            output, sketch_apply only).
 *   out      receives the handle.
 * Allocates no device memory.  Errors: SK_EINVAL.
 */
int sketch_create(int64_t m, int64_t d, int32_t s, uint64_t seed, int32_t rounding,
                  sk_handle *out);

/* sketch_destroy -- free the handle and its workspace (NULL is accepted). */
int sketch_destroy(sk_handle h);

/*
 * sketch_apply -- SA = S[:, row_offset : row_offset+rows] * A  (Section 4.1,
 * SparseStack accumulation; Section 4.2 for the FP16 modes).
 *   A          device, rows x n, element type a_dtype (SK_F32/F16/BF16),
 *              leading dimension lda >= n.  May be NULL when rows == 0.
 *   row_offset first global row; row_offset + rows <= m.  The hash uses
 *              global row indices, so calls on consecutive row ranges with
 *              SK_ACCUMULATE reproduce one call on the whole range.
 *   SA         device, d x n, FP32 for SK_ACC_F32 else FP16 (raw 16-bit),
 *              leading dimension ldsa >= n.  FP16 SA must be 4-byte aligned
 *              with ldsa even (packed FP16 atomics).
 *   flags      0 or SK_ACCUMULATE.
 *   round_epoch selects the rounding-noise stream of the SR / dither modes
 *              (S does not change with it).
 * FP32 mode: SA = fl32(fl32(1/sqrt(s)) * sum) with the sum accumulated in
 * FP32 in an unspecified order (exact for integer-valued A whose partial sums
 * stay below 2^24).  FP16 modes: see sk_schedule.
 * BF16 modes: BF16 keeps 8 significant bits, so summing unit partials in
 * BF16 would cost about 2^-9 per addition; instead the whole call is summed
 * in FP32 (the FP32 mode's partials, added into a d x n FP32 workspace the
 * handle allocates on first need) and each entry is rounded once to BF16
 * with the handle's rule at site q = row_offset*d*n + b*n + c (SR: exact
 * stochastic rounding between the BF16 neighbours; dither: round-to-nearest
 * of fma(u*2^-24 - 1/2, x*2^-7, x)), then stored, or added to SA with one
 * BF16 round-to-nearest addition under SK_ACCUMULATE.  BF16 SA needs 2-byte
 * alignment only.  BF16 handles are not accepted by batches, sketch_solve or
 * the request server (SK_EUNSUPPORTED).
 * Large d/s: the partials take narrower column tiles (8, 4 or 2 columns)
 * as d/s grows.  When only a tile narrower than the width calls for fits (or
 * none), the whole call is one unit summed into a d x n FP32 workspace that
 * the handle allocates on first need and keeps (with, for the gather, its
 * bucket lists: 3d + rows*s 32-bit words): by the bucket-sorted gather (rows
 * of 256 bytes or more; 64 or more when no tile fits), whose entries are
 * the FP32 rounding of their FP64 sums, or else by FP32 atomics per
 * contribution; the sum is then scaled and (16-bit modes) rounded once per
 * entry at sites q = row_offset*d*n + b*n + c.  sketch_plan reports which.
 * The call enqueues work on `stream` and returns; it does not synchronise.
 * Errors: SK_EINVAL (shapes, pointers, flags), SK_EUNSUPPORTED (alignment, a
 * forced block_group that does not fit), SK_ENOMEM, SK_EHIP.
 */
int sketch_apply(sk_handle h, const void *A, int32_t a_dtype, int64_t rows, int64_t n,
                 int64_t lda, int64_t row_offset, void *SA, int64_t ldsa, uint32_t flags,
                 uint32_t round_epoch, void *stream);

/*
 * sketch_apply_noalloc -- sketch_apply for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, semantics and results as
 * sketch_apply; it calls no hipMalloc or hipFree.  Where sketch_apply would
 * use the handle's d x n FP32 workspace (d/s beyond the LDS partials, BF16
 * output, FP32 accumulation into SA with a non-power-of-two 1/sqrt(s)), it
 * uses instead a static device scratch array of 4194304 floats (16 MiB) that
 * the library holds on each GPU it runs on until the process ends; it clears
 * what it uses with a fill kernel (the gather's counters; its other arrays
 * are written whole before they are read).  Calls that would need more than
 * 4194304 workspace floats fail with SK_EINVAL; where the planner chose the
 * bucket-sorted gather and its lists do not fit beside the d x n sum, the
 * call takes the FP32-atomic workspace path instead (a schedule that forces
 * the gather fails).  Every call on one
 * GPU shares that GPU's scratch: calls that overlap on one GPU (two streams,
 * two threads) race and give wrong results.
 */
int sketch_apply_noalloc(sk_handle h, const void *A, int32_t a_dtype, int64_t rows, int64_t n,
                         int64_t lda, int64_t row_offset, void *SA, int64_t ldsa, uint32_t flags,
                         uint32_t round_epoch, void *stream);

/*
 * sketch_set_schedule -- force a schedule for later sketch_apply calls on h
 * (NULL restores the automatic choice).  Fields are checked against the
 * handle at apply time.  Errors: SK_EINVAL (bad field values).
 */
int sketch_set_schedule(sk_handle h, const sk_schedule *sched);

/*
 * sketch_plan -- the schedule sketch_apply would use for (a_dtype, rows, n)
 * on this handle and the current device, written to *out (all fields zero
 * for the workspace path of large d/s, see sketch_apply).  Errors:
 * SK_EINVAL, SK_EUNSUPPORTED, SK_EHIP (device query).
 */
int sketch_plan(sk_handle h, int32_t a_dtype, int64_t rows, int64_t n, sk_schedule *out);

/*
 * sketch_hash -- the S entries of global rows row_begin .. row_begin+count-1
 * (Section 2.2 SparseStack definition, hash version 1): buckets[i*s + j] in
 * [j*d/s, (j+1)*d/s) and signs[i*s + j] in {-1, +1}.  Device int32 / int8
 * arrays of count*s entries.  A debugging and testing export.
 * Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_hash(sk_handle h, int64_t row_begin, int64_t count, int32_t *buckets,
                int8_t *signs, void *stream);

/*
 * sketch_quantize -- the 16-bit rounding rules of Section 4.2 applied to
 * `count` FP32 values: out[k] = Q_mode(x[k]) with rounding noise of site
 * site0 + k under (seed, epoch).  mode: SK_ACC_F16_RN / _SR / _DITHER (FP16
 * bit patterns) or SK_ACC_BF16_RN / _SR / _DITHER (BF16 bit patterns).  x
 * and out are device arrays.  A testing export of exactly the quantisers
 * the 16-bit modes of sketch_apply use.
 * Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_quantize(int32_t mode, const float *x, uint16_t *out, int64_t count, uint64_t seed,
                    uint32_t epoch, uint64_t site0, void *stream);

/* ---- batches of independent sketches -------------------------------------- */

/*
 * One problem of a batch: SA = S A with S described by (m, d, s, seed) as in
 * sketch_create and rounding rule `rounding`; A, SA as in sketch_apply (rows =
 * m, row_offset = 0, no SK_ACCUMULATE).  All problems of a batch share a_dtype
 * and the accumulation class (all SK_ACC_F32, or all FP16 rules); m, n, d, s,
 * seed, rule and epoch may differ.  SA of distinct problems must not overlap.
 */
typedef struct sk_problem {
    int64_t m, n, d;
    int32_t s, rounding;
    uint64_t seed;
    const void *A;
    int64_t lda;
    void *SA;
    int64_t ldsa;
    int32_t a_dtype;
    uint32_t round_epoch;
    int32_t reserved[4];  /* must be zero */
} sk_problem;

typedef struct sk_batch *sk_batch_handle;

/*
 * sketch_batch_create -- plan a batch once: validates every problem, picks
 * the schedule (`sched`, else the tuning table entry for this batch's
 * signature, else the default), sorts the problems largest first and uploads
 * their descriptors to the current device.  The problems' A and SA pointers
 * are recorded and must stay valid while the handle is used.  sched fields:
 * chunk_rows (rows per work item; default 16384), block_group, waves,
 * col_tile (0: 8 columns for n <= 16 and 32 otherwise, per problem; or 32 or
 * 8 for all); xcd_remap is ignored.
 * Errors: SK_EINVAL, SK_EUNSUPPORTED, SK_ENOMEM, SK_EHIP.
 */
int sketch_batch_create(const sk_problem *probs, int32_t count, const sk_schedule *sched, sk_batch_handle *out);

/*
 * sketch_batch_apply -- run the batch on `stream`: one kernel clears every
 * SA and resets the work counter, then ONE persistent launch sketches all
 * problems, each workgroup taking (problem, unit, column tile) work items
 * from a device counter (plus one scale kernel for FP32 problems whose
 * 1/sqrt(s) is not a power of two).  Asynchronous; no allocation, no host
 * synchronisation, no memset nodes, so it may be captured in a graph.  Calls
 * on one handle must not overlap (they share the work counter).
 * Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_batch_apply(sk_batch_handle b, void *stream);

/*
 * sketch_batch_graph -- the same work replayed from a HIP graph: the first
 * call captures sketch_batch_apply on a library-owned stream and
 * instantiates it; every call launches the instantiated graph on `stream`.
 * Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_batch_graph(sk_batch_handle b, void *stream);

/*
 * sketch_apply_batched -- one-shot form: create, apply, wait for the stream,
 * destroy.  Allocates and synchronises; use the handle API for repeated or
 * captured launches.  Errors: as sketch_batch_create / sketch_batch_apply.
 */
int sketch_apply_batched(const sk_problem *probs, int32_t count, const sk_schedule *sched, void *stream);

/* sketch_batch_schedule -- the schedule the batch was planned with. */
int sketch_batch_schedule(sk_batch_handle b, sk_schedule *out);

/* sketch_batch_destroy -- free descriptors and graph (NULL is accepted). */
int sketch_batch_destroy(sk_batch_handle b);

/*
 * sketch_tune_batch -- time candidate schedules (rows per work item x waves
 * per workgroup x column tile: each problem's own, or 32 columns for all) on
 * this batch with real launches (each problem's SA is
 * overwritten), keep the fastest in the process-wide tuning table under the
 * batch's signature, append it to the JSON file `cache_path` (NULL: no file)
 * and return it in *out (may be NULL).  Errors: as sketch_batch_create.
 */
int sketch_tune_batch(const sk_problem *probs, int32_t count, const char *cache_path, sk_schedule *out);

/*
 * sketch_tune_apply -- the same for single sketch_apply calls of this handle
 * on (a_dtype, rows, n): candidates over chunk_rows x waves x block_group x
 * column tile (32, 8, 4 or 2 columns), and the two workspace paths (FP32
 * global atomics; the bucket-sorted gather);
 * SA is overwritten.  The winner is used by later sketch_apply calls with the
 * same signature (handle's d, s, rounding; a_dtype; n; rows rounded to a
 * power of two) unless a schedule is forced.  Errors: as sketch_apply.
 */
int sketch_tune_apply(sk_handle h, const void *A, int32_t a_dtype, int64_t rows, int64_t n, int64_t lda,
                      void *SA, int64_t ldsa, const char *cache_path, sk_schedule *out, void *stream);

/*
 * sketch_load_tuning -- merge a JSON file written by the tuners into the
 * tuning table.  Returns the number of entries read (>= 0) or SK_EINVAL (file
 * missing or malformed).  sketch_clear_tuning empties the table.
 */
int sketch_load_tuning(const char *path);
int sketch_clear_tuning(void);

/* ---- least squares -------------------------------------------------------- */

/*
 * Options of sketch_solve.  Zero fields take the defaults in brackets.
 *   tol         stopping tolerance on the normal-equations residual
 *               ||A^T r|| / (||A||_F ||r||), r = b - A x, evaluated in FP64;
 *               the solve also stops when ||r|| <= tol ||b||        [1e-10]
 *   inner_tol   LSQR tolerance (Paige-Saunders tests on the corrected
 *               problem, relative to ||r||)                          [1e-6]
 *   max_refine  FP64 refinement steps                                [10]
 *   max_inner   LSQR iterations per refinement step                  [100]
 *   round_epoch rounding-noise stream of the SR / dither sketch of A  [0]
 */
typedef struct sk_solve_opts {
    double tol;
    double inner_tol;
    int32_t max_refine;
    int32_t max_inner;
    uint32_t round_epoch;
    int32_t reserved[3];  /* must be zero */
} sk_solve_opts;

/* Statistics of one sketch_solve call (times from HIP events, in ms). */
typedef struct sk_solve_info {
    int32_t converged;       /* 1 if the stopping test was met                */
    int32_t refine_steps;    /* FP64 residual evaluations after the start     */
    int32_t inner_iters;     /* LSQR iterations over all steps                */
    int32_t reserved0;
    double crit;             /* ||A^T r|| / (||A||_F ||r||) of the returned x */
    double rel_residual;     /* ||b - A x|| / ||b|| of the returned x         */
    double rel_residual_x0;  /* the same for the sketch-and-solve start x0    */
    double ms_sketch;        /* sketch of A and b                             */
    double ms_factor;        /* Householder QR of [SA | Sb], R^-1, M, x0      */
    double ms_refine;        /* residuals and LSQR                            */
    double ms_total;
    double reserved[4];
} sk_solve_info;

/*
 * sketch_solve -- least squares min ||A x - b||_2 for A (m x n, m = the
 * handle's m) by sketch-and-precondition with FP64 iterative refinement.
 * The paper forms SA and Sb and solves the sketched problem with an FP32
 * reduced QR and a triangular solve (Section 5.1, sketch-and-solve); it names
 * sketch-and-precondition as related and future work (Section 3.1; Section 6).
 * Here: SA = S A with the handle's accumulation mode (Section 4) and Sb in
 * FP32; R from an FP32 Householder QR of SA; P = R^-1 formed explicitly in
 * FP32; x0 = P (Q^T Sb) (the sketch-and-solve solution); then repeat:
 * r = b - A x in FP64 (A upcast exactly); stop when the criterion of
 * sk_solve_opts holds; LSQR (Paige & Saunders 1982) on min ||A P y - r/||r|| ||
 * with the products by A in FP32 over A in its storage type; x += ||r|| P y in
 * FP64.
 *   A      device, m x n, element type a_dtype (SK_F32/F16/BF16), lda >= n.
 *   n      1 .. 1024 and n <= d; d <= 16384.
 *   b      device FP64, m values.      x  device FP64, n values (output).
 *   opts   NULL for the defaults.      info  may be NULL.
 * Synchronises `stream` a few times per refinement step to read the stopping
 * tests.  Device workspace is allocated by the handle on first use (and when
 * a larger problem arrives) and kept until sketch_destroy.
 * Errors: SK_EINVAL (arguments; SA numerically rank deficient), SK_EUNSUPPORTED,
 * SK_ENOMEM, SK_EHIP, SK_ENOTCONV (x holds the last iterate and info its
 * criterion).
 */
int sketch_solve(sk_handle h, const void *A, int32_t a_dtype, int64_t n, int64_t lda, const double *b,
                 double *x, const sk_solve_opts *opts, sk_solve_info *info, void *stream);

/*
 * sketch_qr_f32 -- in-place FP32 Householder QR of the first k columns of M
 * (rows x cols, row-major, leading dimension ldm, k <= min(rows, cols)), the
 * factorisation sketch_solve applies to [SA | Sb].  The reflectors
 * H_j = I - tau_j v_j v_j^T (v_j[j] = 1, LAPACK convention) are applied to all
 * `cols` columns.  On return the upper triangle of M[0:k, 0:cols] holds R (and
 * Q^T applied to the columns beyond k), v_j below the diagonal and tau_j in
 * tau[j] (device, k floats).  rows <= 16384, cols <= 1025.  A testing export.
 * Errors: SK_EINVAL, SK_EUNSUPPORTED, SK_EHIP.
 */
int sketch_qr_f32(float *M, int64_t rows, int64_t cols, int64_t ldm, int64_t k, float *tau, void *stream);

/*
 * sketch_trinv_f32 -- P = R^-1 for the upper-triangular R in the first n rows
 * and columns of R (leading dimension ldr), by FP32 back substitution, one
 * column of P at a time.  P and PT (= P^T) are n x n with leading dimension
 * ldp; entries below (above) the diagonal are zero.  *bad (device int32) is
 * set to 1 if a diagonal entry of R is zero or a result is not finite (it is
 * not cleared).  n <= 1024.  A testing export of the preconditioner sketch_solve
 * uses.  Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_trinv_f32(const float *R, int64_t n, int64_t ldr, float *P, float *PT, int64_t ldp, int32_t *bad,
                     void *stream);

/* ---- request server ----------------------------------------------------- */

/*
 * A least-squares request: min ||A x - b|| with the sketch (m, d, s, seed,
 * rounding) as in sketch_create and options as in sketch_solve.
 *   gen = 0  A (device, m x n, a_dtype, lda) and b (device FP64) are given by
 *            the caller and must stay valid until the request completes.
 *   gen = 1  the server generates A = N(0,1) at admission (gen = 2: coherent,
 *            1e-3 N(0,1) with rows 0..n-1 = 100 I_n) in a_dtype from gen_seed,
 *            x* = N(0,1) and b = A x* + 1e-6 N(0,1) in FP64, inside its own
 *            memory (A, lda, b are ignored).  The generator is Philox4x32-10
 *            with Box-Muller; its time is reported as ms_ingest.
 *   x        device FP64, n values: receives the solution.
 */
typedef struct sk_request {
    int64_t m, n, d;
    int32_t s, rounding;
    uint64_t seed;
    int32_t a_dtype, gen;
    const void *A;
    int64_t lda;
    const double *b;
    double *x;
    uint64_t gen_seed;
    sk_solve_opts opts;
    int32_t reserved[4];  /* must be zero */
} sk_request;

/* Outcome of one request; times in seconds on the server's clock (sk_server_clock). */
typedef struct sk_result {
    int32_t status;       /* SK_OK, SK_ENOTCONV or the error of the solve       */
    int32_t reserved0;
    double t_submit, t_admit, t_done;
    double ms_ingest;     /* generation kernels (gen != 0), HIP events          */
    sk_solve_info info;
} sk_result;

typedef struct sk_server_info {
    int64_t submitted, completed, in_flight, queued;
    int64_t bytes_in_use, bytes_high_water, budget;
    int32_t slots, reserved;
} sk_server_info;

typedef struct sk_server *sk_server_handle;

/*
 * sk_server_create -- a continuous-batching least-squares server on the
 * current device.  It allocates one device pool of budget_bytes and
 * max_slots (1..64) streams, and runs one scheduler thread.  Requests wait
 * in arrival order; the head is admitted as soon as a slot is free and the
 * pool has room for its footprint (sk_server_footprint), so requests that
 * arrive while others run join them on the device; each admitted request
 * advances on its own stream, interleaved with the others, and releases its
 * memory when done.  Errors: SK_EINVAL, SK_ENOMEM, SK_EHIP.
 */
int sk_server_create(size_t budget_bytes, int32_t max_slots, sk_server_handle *out);

/* sk_server_footprint -- device bytes a request holds while admitted. */
int sk_server_footprint(const sk_request *req, size_t *bytes);

/*
 * sk_server_submit -- queue a request (copied); *ticket identifies it.
 * Errors: SK_EINVAL (validation as in sketch_solve), SK_EADMIT (footprint
 * larger than the budget: it could never run), SK_EBUSY (shutting down).
 */
int sk_server_submit(sk_server_handle srv, const sk_request *req, uint64_t *ticket);

/*
 * sk_server_poll -- *done = 1 and *out filled once the request finished
 * (the ticket is then forgotten), else *done = 0.  sk_server_wait blocks
 * until done.  Errors: SK_EINVAL (unknown ticket).
 */
int sk_server_poll(sk_server_handle srv, uint64_t ticket, int32_t *done, sk_result *out);
int sk_server_wait(sk_server_handle srv, uint64_t ticket, sk_result *out);

/* sk_server_stats -- counters and the pool's high-water mark. */
int sk_server_stats(sk_server_handle srv, sk_server_info *out);

/* sk_server_clock -- seconds since the server was created. */
double sk_server_clock(sk_server_handle srv);

/* sk_server_destroy -- finish queued and running requests, then free all. */
int sk_server_destroy(sk_server_handle srv);

/*
 * sk_server_simulate -- the server's admission policy on the host only, as a
 * discrete-event simulation (a testing export; no device is used): request k
 * arrives at arrive[k] (non-decreasing), holds footprint[k] bytes and runs
 * for service[k] seconds once admitted; returns admit[k] and done[k].
 * Errors: SK_EINVAL, SK_EADMIT (a footprint above the budget).
 */
int sk_server_simulate(size_t budget_bytes, int32_t max_slots, int32_t count, const double *arrive,
                       const uint64_t *footprint, const double *service, double *admit, double *done);

/* sketch_last_error -- message of the last failure on this thread ("" if none). */
const char *sketch_last_error(void);

/* sketch_version -- library version * 100 + hash version. */
int sketch_version(void);

/*
 * sketch_sync -- wait for the work this library enqueued on `stream` (NULL:
 * the default stream) and report an asynchronous HIP failure of that work,
 * which the enqueueing calls cannot see.  h may be NULL; a non-NULL h is
 * only checked for validity.  Returns SK_OK, or SK_EHIP with the HIP message
 * in sketch_last_error().
 */
int sketch_sync(sk_handle h, void *stream);

/*
 * sketch_stream_read -- measurement export: read `bytes` bytes of device
 * memory at p once (16-byte non-temporal loads, folded by XOR into out[0..255],
 * 256 device words the caller provides).  Its time is the streaming-read ceiling of
 * the device, against which sketch_apply's bandwidth is compared.  bytes: a
 * positive multiple of 16; p: 16-byte aligned.  Asynchronous on `stream`.
 * Errors: SK_EINVAL, SK_EHIP.
 */
int sketch_stream_read(const void *p, int64_t bytes, uint32_t *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SKETCH_H */
