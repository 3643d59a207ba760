/*
 * C FP64 oracle for the sparse-sketch library.  TEST INFRASTRUCTURE ONLY:
 * linked by the test-suite and the CPU-baseline leg of the benchmark, never by
 * the product.  Shares no code with the HIP implementation.
 *
 * Paper: "Randomized Sketching is Robust to Low-Precision Rounding on GPUs"
 * (Jeendgar, Flint, Anzt).
 *   - SparseStack S (Section 2.2, Definition "SparseStack"): s blocks of
 *     d/s rows; column i has one nonzero per block, value +-1/sqrt(s)
 *     (Section 4.1 gives the block ranges and the value scale).  s = 1 is
 *     CountSketch (Section 2.2).
 *   - SA is formed by scattering each row of A into its s target rows
 *     (Section 4.1, explicit SparseStack accumulation); here in FP64 with one
 *     private d x n partial per thread, summed at the end.
 *   - Least squares by Householder QR (the FP64 reference the sketch-based
 *     solver is compared with; Section 5.1 solves min ||Ax - b||).
 *
 * The row hash (bucket, sign) uses Philox4x32-10 (Salmon et al., SC'11) with
 * key (lo32 seed, hi32 seed) and counter (lo32 i, hi32 i, j/4, TAG_SKETCH);
 * word j%4 = w gives bucket j*W + (w*W >> 32) (W = d/s) and sign -1 iff w&1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_M0 0xD2511F53u
#define ORC_M1 0xCD9E8D57u
#define ORC_W0 0x9E3779B9u
#define ORC_W1 0xBB67AE85u
#define ORC_TAG_SKETCH 0x534B4348u

void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += ORC_W0; k1 += ORC_W1; }
        uint64_t p0 = (uint64_t)ORC_M0 * c0;
        uint64_t p1 = (uint64_t)ORC_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* buckets[i*s + j], signs[i*s + j] for global rows row_begin .. +count-1 */
int orc_hash(uint64_t seed, int64_t d, int32_t s, int64_t row_begin, int64_t count,
             int64_t *buckets, int8_t *signs)
{
    if (s < 1 || d < 1 || d % s) return -1;
    const uint64_t W = (uint64_t)(d / s);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    #pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < count; ++t) {
        uint64_t i = (uint64_t)(row_begin + t);
        uint32_t w4[4];
        for (int32_t j = 0; j < s; ++j) {
            if ((j & 3) == 0) {
                uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)(j >> 2), ORC_TAG_SKETCH};
                orc_philox(ctr, key, w4);
            }
            uint32_t w = w4[j & 3];
            buckets[t * s + j] = (int64_t)j * (int64_t)W + (int64_t)(((uint64_t)w * W) >> 32);
            signs[t * s + j] = (w & 1u) ? -1 : 1;
        }
    }
    return 0;
}

static double half_to_double(uint16_t h)
{
    int sgn = h >> 15, e = (h >> 10) & 31, f = h & 1023;
    double v;
    if (e == 0) v = ldexp((double)f, -24);
    else if (e == 31) v = f ? NAN : INFINITY;
    else v = ldexp((double)(1024 + f), e - 25);
    return sgn ? -v : v;
}

static double bf16_to_double(uint16_t h)
{
    uint32_t bits = (uint32_t)h << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

static double load_elem(const void *A, int dtype, int64_t idx)
{
    switch (dtype) {
    case 0: return (double)((const float *)A)[idx];
    case 1: return half_to_double(((const uint16_t *)A)[idx]);
    case 2: return bf16_to_double(((const uint16_t *)A)[idx]);
    default: return ((const double *)A)[idx];
    }
}

/*
 * SA (d x n, row-major, FP64) = scale * sum over rows of sign * A[row, :]
 * scattered into the hashed rows.  dtype: 0 FP32, 1 FP16, 2 BF16, 3 FP64.
 * nthreads <= 0 means all OpenMP threads.
 */
int orc_sketch_f64(const void *A, int dtype, int64_t rows, int64_t n, int64_t lda,
                   int64_t row_offset, int64_t d, int32_t s, uint64_t seed,
                   double scale, double *SA, int nthreads)
{
    if (s < 1 || d < 1 || d % s || n < 1 || lda < n || rows < 0) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    const uint64_t W = (uint64_t)(d / s);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double *part = (double *)calloc((size_t)nthreads * (size_t)(d * n), sizeof(double));
    if (!part) return -3;
    #pragma omp parallel num_threads(nthreads)
    {
        double *P = part + (size_t)omp_get_thread_num() * (size_t)(d * n);
        double *row = (double *)malloc(sizeof(double) * (size_t)n);
        #pragma omp for schedule(static)
        for (int64_t t = 0; t < rows; ++t) {
            uint64_t i = (uint64_t)(row_offset + t);
            for (int64_t c = 0; c < n; ++c) row[c] = load_elem(A, dtype, t * lda + c);
            uint32_t w4[4];
            for (int32_t j = 0; j < s; ++j) {
                if ((j & 3) == 0) {
                    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), (uint32_t)(j >> 2), ORC_TAG_SKETCH};
                    orc_philox(ctr, key, w4);
                }
                uint32_t w = w4[j & 3];
                int64_t b = (int64_t)j * (int64_t)W + (int64_t)(((uint64_t)w * W) >> 32);
                double *dst = P + b * n;
                if (w & 1u) for (int64_t c = 0; c < n; ++c) dst[c] -= row[c];
                else        for (int64_t c = 0; c < n; ++c) dst[c] += row[c];
            }
        }
        free(row);
    }
    #pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t e = 0; e < d * n; ++e) {
        double acc = 0.0;
        for (int t = 0; t < nthreads; ++t) acc += part[(size_t)t * (size_t)(d * n) + (size_t)e];
        SA[e] = scale * acc;
    }
    free(part);
    return 0;
}

/*
 * Least squares min ||A x - b|| by Householder QR in FP64 (A: m x n row-major,
 * any dtype code as above, lda stride; b: FP64).  x gets n values.
 * Returns 0, -1 on bad shape, -3 on allocation failure, -4 if R is singular.
 */
int orc_lstsq(const void *A, int dtype, int64_t m, int64_t n, int64_t lda,
              const double *b, double *x, int nthreads)
{
    if (m < n || n < 1 || lda < n) return -1;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
    /* column-major copy so each Householder step walks contiguous columns */
    double *Q = (double *)malloc(sizeof(double) * (size_t)m * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    if (!Q || !y) { free(Q); free(y); return -3; }
    #pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c) Q[(size_t)c * m + i] = load_elem(A, dtype, i * lda + c);
    memcpy(y, b, sizeof(double) * (size_t)m);
    for (int64_t k = 0; k < n; ++k) {
        double *v = Q + (size_t)k * m;
        double nrm = 0.0;
        #pragma omp parallel for reduction(+:nrm) num_threads(nthreads)
        for (int64_t i = k; i < m; ++i) nrm += v[i] * v[i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) { free(Q); free(y); return -4; }
        double alpha = (v[k] > 0) ? -nrm : nrm;       /* R[k][k] */
        double v0 = v[k] - alpha;
        /* reflector u = (v0, v[k+1..m-1]) ; H = I - 2 u u^T / (u^T u) */
        double uu = v0 * v0 + (nrm * nrm - v[k] * v[k]);
        v[k] = v0;
        #pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int64_t c = k + 1; c < n; ++c) {
            double *w = Q + (size_t)c * m;
            double dot = 0.0;
            for (int64_t i = k; i < m; ++i) dot += v[i] * w[i];
            double f = 2.0 * dot / uu;
            for (int64_t i = k; i < m; ++i) w[i] -= f * v[i];
        }
        double dot = 0.0;
        #pragma omp parallel for reduction(+:dot) num_threads(nthreads)
        for (int64_t i = k; i < m; ++i) dot += v[i] * y[i];
        double f = 2.0 * dot / uu;
        #pragma omp parallel for schedule(static) num_threads(nthreads)
        for (int64_t i = k; i < m; ++i) y[i] -= f * v[i];
        v[k] = alpha;                                  /* keep R's diagonal here */
    }
    /* back substitution R x = y[0:n]; R[k][c] (c > k) sits at Q[c*m + k] */
    for (int64_t k = n - 1; k >= 0; --k) {
        double acc = y[k];
        for (int64_t c = k + 1; c < n; ++c) acc -= Q[(size_t)c * m + k] * x[c];
        x[k] = acc / Q[(size_t)k * m + k];
    }
    free(Q); free(y);
    return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
