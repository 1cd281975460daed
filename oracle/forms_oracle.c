/*
 * forms_oracle.c -- plain, slow reference for the forms built on top of the
 * paper's RKA / RKAB iterations: FP32-accumulation iterations, FP64
 * residuals, iterative refinement (with the residual projected onto range(A)
 * for inconsistent systems) and the least-squares gradient.
 *
 * TEST INFRASTRUCTURE ONLY (see rka_oracle.h): nothing in the solver library
 * includes, links or calls this code.
 *
 * The paper (arXiv 2401.17474) defines the iterations (Eq. (7) for RKA,
 * Sec. 3.4.1 for RKAB) and notes that randomized Kaczmarz started from zero
 * on an underdetermined consistent system converges to its minimum-norm
 * solution (Sec. 2.1), and that RKA on an inconsistent system stalls at a
 * convergence horizon set by the least-squares residual (Sec. 2.3.1).  The
 * precision form, the refinement and the gradient are additions of this
 * implementation; their definitions are written out in rka_oracle.h.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "rka_oracle.h"

/* Element (i, c) of A widened exactly to binary32 (dtype 1 or 2 only). */
static float elem32(const void* A, int dtype, int64_t lda, int64_t i, int64_t c)
{
    if (dtype == 1) return ((const float*)A)[i * lda + c];
    uint32_t bits = (uint32_t)((const uint16_t*)A)[i * lda + c] << 16;
    float f;
    memcpy(&f, &bits, sizeof f);
    return f;
}

/* Element (i, c) of A widened exactly to binary64. */
static double elem64(const void* A, int dtype, int64_t lda, int64_t i, int64_t c)
{
    if (dtype == 0) return ((const double*)A)[i * lda + c];
    return (double)elem32(A, dtype, lda, i, c);
}

static int narrow_ok(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                     const double* b, const double* x, int32_t q, int32_t bs, double alpha,
                     int64_t K)
{
    if (!A || !b || !x || (dtype != 1 && dtype != 2)) return 0;
    if (m < 1 || n < 1 || lda < n || q < 1 || bs < 1 || K < 0) return 0;
    if (!(alpha > 0.0) || !isfinite(alpha)) return 0;
    return 1;
}

/* <A^(i), v> in binary32, summed left to right. */
static float dot32(const void* A, int dtype, int64_t lda, int64_t i, int64_t n, const float* v)
{
    float d = 0.0f;
    for (int64_t c = 0; c < n; ++c) {
        float p = elem32(A, dtype, lda, i, c) * v[c];
        d = d + p;
    }
    return d;
}

/* RKA, Eq. (7), with every iteration quantity in binary32: x32 = x rounded;
 * per iteration d_w = <A^(i_w), x32>, s_w = alpha32 (b32_i - d_w) / w32_i
 * (b_i and ||A^(i)||^2 rounded to binary32 once), u_c = sum_w s_w A[i_w, c]
 * in worker order, x32_c = x32_c + u_c * (1/q)32.  x = x32 widened at the end. */
int oracle_rka_f32_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         const double* b, double* x, int32_t q, double alpha, int64_t K,
                         const int32_t* idx)
{
    if (!narrow_ok(A, dtype, m, n, lda, b, x, q, 1, alpha, K) || !idx) return ORACLE_EINVAL;
    double* wn = (double*)malloc((size_t)m * sizeof(double));
    float* x32 = (float*)malloc((size_t)n * sizeof(float));
    float* s = (float*)malloc((size_t)q * sizeof(float));
    if (!wn || !x32 || !s) {
        free(wn);
        free(x32);
        free(s);
        return ORACLE_EINVAL;
    }
    oracle_row_norms(A, dtype, m, n, lda, wn);
    for (int64_t c = 0; c < n; ++c) x32[c] = (float)x[c];
    const float a32 = (float)alpha, invq = (float)(1.0 / (double)q);
    for (int64_t k = 0; k < K; ++k) {
        const int32_t* rows = idx + k * q;
        for (int32_t w = 0; w < q; ++w) {
            float d = dot32(A, dtype, lda, rows[w], n, x32);
            s[w] = a32 * ((float)b[rows[w]] - d) / (float)wn[rows[w]];
        }
        for (int64_t c = 0; c < n; ++c) {
            float u = 0.0f;
            for (int32_t w = 0; w < q; ++w) {
                float t = s[w] * elem32(A, dtype, lda, rows[w], c);
                u = u + t;
            }
            float t = u * invq;
            x32[c] = x32[c] + t;
        }
    }
    for (int64_t c = 0; c < n; ++c) x[c] = (double)x32[c];
    free(wn);
    free(x32);
    free(s);
    return ORACLE_OK;
}

/* RKAB (Sec. 3.4.1) in binary32: every worker starts from v = x32, applies
 * bs projections v_c = v_c + s A[i, c] with s = alpha32 (b32_i - <A^(i), v>)
 * / w32_i, and x32_c = (sum_w v_w,c) / q32 in worker order. */
int oracle_rkab_f32_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                          const double* b, double* x, int32_t q, int32_t bs, double alpha,
                          int64_t K, const int32_t* idx)
{
    if (!narrow_ok(A, dtype, m, n, lda, b, x, q, bs, alpha, K) || !idx) return ORACLE_EINVAL;
    double* wn = (double*)malloc((size_t)m * sizeof(double));
    float* x32 = (float*)malloc((size_t)n * sizeof(float));
    float* v = (float*)malloc((size_t)n * sizeof(float));
    float* sum = (float*)malloc((size_t)n * sizeof(float));
    if (!wn || !x32 || !v || !sum) {
        free(wn);
        free(x32);
        free(v);
        free(sum);
        return ORACLE_EINVAL;
    }
    oracle_row_norms(A, dtype, m, n, lda, wn);
    for (int64_t c = 0; c < n; ++c) x32[c] = (float)x[c];
    const float a32 = (float)alpha, q32 = (float)q;
    for (int64_t k = 0; k < K; ++k) {
        for (int64_t c = 0; c < n; ++c) sum[c] = 0.0f;
        for (int32_t w = 0; w < q; ++w) {
            for (int64_t c = 0; c < n; ++c) v[c] = x32[c];
            for (int32_t j = 0; j < bs; ++j) {
                int64_t i = idx[(k * q + w) * (int64_t)bs + j];
                float d = dot32(A, dtype, lda, i, n, v);
                float s = a32 * ((float)b[i] - d) / (float)wn[i];
                for (int64_t c = 0; c < n; ++c) {
                    float t = s * elem32(A, dtype, lda, i, c);
                    v[c] = v[c] + t;
                }
            }
            for (int64_t c = 0; c < n; ++c) sum[c] = sum[c] + v[c];
        }
        for (int64_t c = 0; c < n; ++c) x32[c] = sum[c] / q32;
    }
    for (int64_t c = 0; c < n; ++c) x[c] = (double)x32[c];
    free(wn);
    free(x32);
    free(v);
    free(sum);
    return ORACLE_OK;
}

int oracle_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At)
{
    if (!A || !At || m < 1 || n < 1 || lda < n) return ORACLE_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c) {
            if (dtype == 0)
                ((double*)At)[c * m + i] = ((const double*)A)[i * lda + c];
            else if (dtype == 1)
                ((float*)At)[c * m + i] = ((const float*)A)[i * lda + c];
            else if (dtype == 2)
                ((uint16_t*)At)[c * m + i] = ((const uint16_t*)A)[i * lda + c];
            else
                return ORACLE_EINVAL;
        }
    return ORACLE_OK;
}

/* out_i = (c ? c_i : 0) + gamma * sum_j M[i, j] v_j, in binary64, left to right. */
int oracle_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                const double* v, const double* c, double gamma, double* out)
{
    if (!M || !v || !out || rows < 1 || cols < 1 || ld < cols) return ORACLE_EINVAL;
    if (dtype != 0 && dtype != 1 && dtype != 2) return ORACLE_EINVAL;
    for (int64_t i = 0; i < rows; ++i) {
        double d = 0.0;
        for (int64_t j = 0; j < cols; ++j) {
            double p = elem64(M, dtype, ld, i, j) * v[j];
            d = d + p;
        }
        double t = gamma * d;
        out[i] = (c ? c[i] : 0.0) + t;
    }
    return ORACLE_OK;
}

/* One inner solve from zero: K iterations of RKA (bs = 1, method 0) or RKAB
 * on the system (M, rhs), rows drawn with oracle_indices on stream `dom` from
 * iteration offset `off`, in binary32 (acc32) or binary64. */
static int inner_solve(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       const double* rhs, double* out, int32_t method, int32_t q, int32_t bs,
                       int32_t acc32, double alpha, int64_t K, uint64_t seed, int64_t off,
                       int32_t dom)
{
    if (method == 0) bs = 1;
    for (int64_t c = 0; c < cols; ++c) out[c] = 0.0;
    if (K == 0) return ORACLE_OK;
    double* w = (double*)malloc((size_t)rows * sizeof(double));
    int32_t* idx = (int32_t*)malloc((size_t)K * (size_t)q * (size_t)bs * sizeof(int32_t));
    int st = ORACLE_EINVAL;
    if (w && idx) {
        oracle_row_norms(M, dtype, rows, cols, ld, w);
        st = oracle_indices(w, rows, seed, off, K, q, bs, dom, idx);
    }
    if (st == ORACLE_OK) {
        if (acc32)
            st = method == 0
                     ? oracle_rka_f32_given(M, dtype, rows, cols, ld, rhs, out, q, alpha, K, idx)
                     : oracle_rkab_f32_given(M, dtype, rows, cols, ld, rhs, out, q, bs, alpha, K,
                                             idx);
        else
            st = method == 0
                     ? oracle_rka_given(M, dtype, rows, cols, ld, rhs, out, q, alpha, K, idx)
                     : oracle_rkab_given(M, dtype, rows, cols, ld, rhs, out, q, bs, alpha, K, idx);
    }
    free(w);
    free(idx);
    return st;
}

/* Iterative refinement.  Per sweep s (0-based):
 *   r = b - A x                                   (binary64)
 *   if range_iters > 0:
 *     g = A^T r                                   (binary64)
 *     y = range_iters iterations of RKA (range_q workers, weight range_alpha)
 *         on the columns, A^T y = g, from y = 0, stream dom 1, offset
 *         s * range_iters -- the minimum-norm solution of A^T y = A^T r is the
 *         projection of r onto range(A) (Sec. 2.1: Kaczmarz from zero on a
 *         consistent underdetermined system tends to its minimum-norm
 *         solution); r = y
 *   d = inner_iters iterations of RKA / RKAB (q, bs, alpha) on A d = r from
 *       d = 0, stream dom 0, offset s * inner_iters, binary32 if acc32
 *   x = x + d                                     (binary64)
 *   measures[s] = ||x - x_ref|| / ||x_ref||, or ||b - A x|| / ||b||. */
int oracle_refine(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
                  const double* x0, double* x, int32_t method, int32_t q, int32_t bs,
                  int32_t acc32, double alpha, int64_t inner_iters, int64_t range_iters,
                  int32_t range_q, double range_alpha, int32_t sweeps, uint64_t seed,
                  const double* x_ref, double* measures)
{
    if (!A || !b || !x || m < 1 || n < 1 || lda < n || sweeps < 1 || q < 1 || inner_iters < 0 ||
        range_iters < 0 || (range_iters > 0 && range_q < 1))
        return ORACLE_EINVAL;
    if (acc32 && dtype == 0) return ORACLE_EINVAL;
    int es = dtype == 0 ? 8 : (dtype == 1 ? 4 : 2);
    double* r = (double*)malloc((size_t)m * sizeof(double));
    double* y = (double*)malloc((size_t)m * sizeof(double));
    double* g = (double*)malloc((size_t)n * sizeof(double));
    double* d = (double*)malloc((size_t)n * sizeof(double));
    void* At = range_iters > 0 ? malloc((size_t)m * (size_t)n * (size_t)es) : NULL;
    int st = ORACLE_OK;
    if (!r || !y || !g || !d || (range_iters > 0 && !At)) {
        st = ORACLE_EINVAL;
        goto done;
    }
    if (At) oracle_transpose(A, dtype, m, n, lda, At);
    for (int64_t c = 0; c < n; ++c) x[c] = x0 ? x0[c] : 0.0;
    double den = 0.0;
    if (x_ref)
        for (int64_t c = 0; c < n; ++c) den = den + x_ref[c] * x_ref[c];
    else
        for (int64_t i = 0; i < m; ++i) den = den + b[i] * b[i];
    for (int32_t s = 0; s < sweeps; ++s) {
        oracle_gemv(A, dtype, m, n, lda, x, b, -1.0, r);
        const double* rhs = r;
        if (range_iters > 0) {
            oracle_gemv(At, dtype, n, m, m, r, NULL, 1.0, g);
            st = inner_solve(At, dtype, n, m, m, g, y, 0, range_q, 1, acc32, range_alpha,
                             range_iters, seed, (int64_t)s * range_iters, 1);
            if (st != ORACLE_OK) goto done;
            rhs = y;
        }
        st = inner_solve(A, dtype, m, n, lda, rhs, d, method, q, bs, acc32, alpha, inner_iters,
                         seed, (int64_t)s * inner_iters, 0);
        if (st != ORACLE_OK) goto done;
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + d[c];
        double num = 0.0;
        if (x_ref) {
            for (int64_t c = 0; c < n; ++c) {
                double e = x[c] - x_ref[c];
                num = num + e * e;
            }
        } else {
            oracle_gemv(A, dtype, m, n, lda, x, b, -1.0, r);
            for (int64_t i = 0; i < m; ++i) num = num + r[i] * r[i];
        }
        if (measures) measures[s] = sqrt(num) / sqrt(den);
    }
done:
    free(r);
    free(y);
    free(g);
    free(d);
    free(At);
    return st;
}

/* ------------------------------------------------------------------ */
/* The Distributed Approach and partial-matrix weights (Sec. 3.3.2).    */
/* ------------------------------------------------------------------ */

/* Worker w draws only from its block of rows floor(w m / q) .. floor((w+1)
 * m / q) - 1: the running sum restarted at the block, t = u * (block total),
 * the smallest row of the block whose running sum exceeds t, else the
 * block's last row of positive weight. */
int oracle_indices_blocks(const double* w, int64_t m, uint64_t seed, int64_t iter_offset,
                          int64_t K, int32_t q, int32_t bs, int32_t dom, int32_t* idx)
{
    if (!w || !idx || m < 1 || q < 1 || q > m || bs < 1 || K < 0 || iter_offset < 0 || dom < 0 ||
        dom > 255)
        return ORACLE_EINVAL;
    double* c = (double*)malloc((size_t)m * sizeof(double));
    if (!c) return ORACLE_EINVAL;
    int st = ORACLE_OK;
    for (int32_t wk = 0; wk < q && st == ORACLE_OK; ++wk) {
        int64_t lo = (int64_t)wk * m / q, hi = ((int64_t)wk + 1) * m / q;
        st = oracle_prefix(w + lo, hi - lo, c + lo);
    }
    for (int64_t k = 0; k < K && st == ORACLE_OK; ++k)
        for (int32_t wk = 0; wk < q; ++wk) {
            int64_t lo = (int64_t)wk * m / q, hi = ((int64_t)wk + 1) * m / q;
            for (int32_t j = 0; j < bs; ++j) {
                double u = oracle_uniform(seed, (uint64_t)(k + iter_offset), (uint32_t)wk,
                                          (uint32_t)j, (uint32_t)dom);
                idx[(k * q + wk) * (int64_t)bs + j] =
                    (int32_t)(lo + oracle_pick_row(c + lo, w + lo, hi - lo, u));
            }
        }
    free(c);
    return st;
}

/* The weight of a projection onto row i drawn by worker wk: the row's own
 * weight w_i of Eq. (7) when row weights are given, else the worker's. */
static double weight_of(const double* walpha, const double* wrow, int32_t wk, int64_t i)
{
    return wrow ? wrow[i] : walpha[wk];
}

/* RKA, Eq. (7), with weights per worker (the partial-matrix alpha of
 * Sec. 3.3.2) or per row: x^(k+1) = x^(k) + (1/q) sum_w weight (b_i -
 * <A^(i), x^(k)>) / ||A^(i)||^2 A^(i)^T, every dot product against x^(k).
 * A row of zero norm contributes nothing (only the cyclic order reaches
 * one). */
static int rka_weighted_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                              const double* b, double* x, int32_t q, const double* walpha,
                              const double* wrow, int64_t K, const int32_t* idx)
{
    if (!A || !b || !x || (!walpha && !wrow) || !idx || m < 1 || n < 1 || lda < n || q < 1 ||
        K < 0)
        return ORACLE_EINVAL;
    double* wn = (double*)malloc((size_t)m * sizeof(double));
    double* s = (double*)malloc((size_t)q * sizeof(double));
    double* acc = (double*)malloc((size_t)n * sizeof(double));
    if (!wn || !s || !acc) {
        free(wn);
        free(s);
        free(acc);
        return ORACLE_EINVAL;
    }
    oracle_row_norms(A, dtype, m, n, lda, wn);
    for (int64_t k = 0; k < K; ++k) {
        const int32_t* rows = idx + k * q;
        for (int32_t wk = 0; wk < q; ++wk) {
            int64_t i = rows[wk];
            if (wn[i] == 0.0) {
                s[wk] = 0.0;
                continue;
            }
            double d = 0.0;
            for (int64_t c = 0; c < n; ++c) {
                double p = elem64(A, dtype, lda, i, c) * x[c];
                d = d + p;
            }
            s[wk] = weight_of(walpha, wrow, wk, i) * ((b[i] - d) / wn[i]);
        }
        for (int64_t c = 0; c < n; ++c) {
            double a = 0.0;
            for (int32_t wk = 0; wk < q; ++wk) {
                double t = s[wk] * elem64(A, dtype, lda, rows[wk], c);
                a = a + t;
            }
            acc[c] = a;
        }
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + acc[c] / (double)q;
    }
    free(wn);
    free(s);
    free(acc);
    return ORACLE_OK;
}

/* RKAB (Sec. 3.4.1) with weights per worker or per row; zero rows as above. */
static int rkab_weighted_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                               const double* b, double* x, int32_t q, int32_t bs,
                               const double* walpha, const double* wrow, int64_t K,
                               const int32_t* idx)
{
    if (!A || !b || !x || (!walpha && !wrow) || !idx || m < 1 || n < 1 || lda < n || q < 1 ||
        bs < 1 || K < 0)
        return ORACLE_EINVAL;
    double* wn = (double*)malloc((size_t)m * sizeof(double));
    double* v = (double*)malloc((size_t)n * sizeof(double));
    double* sum = (double*)malloc((size_t)n * sizeof(double));
    if (!wn || !v || !sum) {
        free(wn);
        free(v);
        free(sum);
        return ORACLE_EINVAL;
    }
    oracle_row_norms(A, dtype, m, n, lda, wn);
    for (int64_t k = 0; k < K; ++k) {
        for (int64_t c = 0; c < n; ++c) sum[c] = 0.0;
        for (int32_t wk = 0; wk < q; ++wk) {
            for (int64_t c = 0; c < n; ++c) v[c] = x[c];
            for (int32_t j = 0; j < bs; ++j) {
                int64_t i = idx[(k * q + wk) * (int64_t)bs + j];
                if (wn[i] == 0.0) continue;
                double d = 0.0;
                for (int64_t c = 0; c < n; ++c) {
                    double p = elem64(A, dtype, lda, i, c) * v[c];
                    d = d + p;
                }
                double s = weight_of(walpha, wrow, wk, i) * ((b[i] - d) / wn[i]);
                for (int64_t c = 0; c < n; ++c) {
                    double t = s * elem64(A, dtype, lda, i, c);
                    v[c] = v[c] + t;
                }
            }
            for (int64_t c = 0; c < n; ++c) sum[c] = sum[c] + v[c];
        }
        for (int64_t c = 0; c < n; ++c) x[c] = sum[c] / (double)q;
    }
    free(wn);
    free(v);
    free(sum);
    return ORACLE_OK;
}

int oracle_rka_walpha_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                            const double* b, double* x, int32_t q, const double* walpha,
                            int64_t K, const int32_t* idx)
{
    if (!walpha) return ORACLE_EINVAL;
    return rka_weighted_given(A, dtype, m, n, lda, b, x, q, walpha, NULL, K, idx);
}

int oracle_rkab_walpha_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                             const double* b, double* x, int32_t q, int32_t bs,
                             const double* walpha, int64_t K, const int32_t* idx)
{
    if (!walpha) return ORACLE_EINVAL;
    return rkab_weighted_given(A, dtype, m, n, lda, b, x, q, bs, walpha, NULL, K, idx);
}

int oracle_rka_wrow_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                          const double* b, double* x, int32_t q, const double* wrow, int64_t K,
                          const int32_t* idx)
{
    if (!wrow) return ORACLE_EINVAL;
    return rka_weighted_given(A, dtype, m, n, lda, b, x, q, NULL, wrow, K, idx);
}

int oracle_rkab_wrow_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                           const double* b, double* x, int32_t q, int32_t bs, const double* wrow,
                           int64_t K, const int32_t* idx)
{
    if (!wrow) return ORACLE_EINVAL;
    return rkab_weighted_given(A, dtype, m, n, lda, b, x, q, bs, NULL, wrow, K, idx);
}

/* ------------------------------------------------------------------ */
/* Cyclic Kaczmarz (Sec. 2.1).                                          */
/* ------------------------------------------------------------------ */

/* The rows in order: draw (k, w, j) of a stream of q workers with blocks of
 * bs takes row (((k + iter_offset) q + w) bs + j) mod m, so that one worker
 * with blocks of one walks the rows 0, 1, ..., m-1, 0, 1, ... */
int oracle_indices_cyclic(int64_t m, int64_t iter_offset, int64_t K, int32_t q, int32_t bs,
                          int32_t* idx)
{
    if (!idx || m < 1 || m > INT32_MAX || q < 1 || bs < 1 || K < 0 || iter_offset < 0)
        return ORACLE_EINVAL;
    for (int64_t k = 0; k < K; ++k)
        for (int32_t wk = 0; wk < q; ++wk)
            for (int32_t j = 0; j < bs; ++j) {
                int64_t pos = ((k + iter_offset) * q + wk) * (int64_t)bs + j;
                idx[(k * q + wk) * (int64_t)bs + j] = (int32_t)(pos % m);
            }
    return ORACLE_OK;
}

/* Cyclic Kaczmarz as Sec. 2.1 writes it: iteration k projects onto the
 * hyperplane of row i = k mod m with relaxation alpha_i,
 *   x <- x + alpha_i (b_i - <A^(i), x>) / ||A^(i)||^2 A^(i)^T,
 * for k = 0 .. iters-1, starting from the x passed in.  relax: m
 * relaxations, or NULL for alpha_i = 1.  A zero row leaves x unchanged. */
int oracle_ck(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
              double* x, const double* relax, int64_t iters)
{
    if (!A || !b || !x || m < 1 || n < 1 || lda < n || iters < 0) return ORACLE_EINVAL;
    for (int64_t k = 0; k < iters; ++k) {
        int64_t i = k % m;
        double nrm = 0.0, d = 0.0;
        for (int64_t c = 0; c < n; ++c) {
            double a = elem64(A, dtype, lda, i, c);
            nrm = nrm + a * a;
            d = d + a * x[c];
        }
        if (nrm == 0.0) continue;
        double s = (relax ? relax[i] : 1.0) * ((b[i] - d) / nrm);
        for (int64_t c = 0; c < n; ++c) x[c] = x[c] + s * elem64(A, dtype, lda, i, c);
    }
    return ORACLE_OK;
}
