/*
 * rka_oracle.h -- plain, slow, single-threaded FP64 reference for randomized
 * Kaczmarz with averaging (RKA) and its block variant (RKAB).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library includes, links
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no header, helper, table or
 * constant with the GPU path.
 *
 * Paper: Ferreira, Acebron, Monteiro, "Parallelization Strategies for the
 * Randomized Kaczmarz Algorithm on Large-Scale Dense Systems" (arXiv
 * 2401.17474).  Each function cites the passage it follows.
 *
 * Conventions (all arrays are host memory owned by the caller):
 *   A      m x n, row-major, leading dimension lda >= n (elements).
 *          dtype 0 = IEEE binary64, 1 = binary32, 2 = bfloat16 (the upper
 *          16 bits of a binary32, stored as uint16).  Narrow types are widened
 *          exactly to binary64 before any arithmetic.
 *   b      m doubles;  x, x0, x_ref  n doubles.
 *   Index stream layout: idx[(k*q + w)*bs + j] is the row used by worker w
 *   at projection j of (outer) iteration k.
 */
#ifndef RKA_ORACLE_H
#define RKA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_NOT_CONVERGED = 1,
    ORACLE_EINVAL = -1,
    ORACLE_EZERONORM = -2,
    ORACLE_EDIVERGED = -3
};

typedef struct {
    int64_t iterations;   /* outer iterations performed                    */
    int64_t projections;  /* row projections performed (iter * q * bs)     */
    double  rel_err;      /* last convergence measure computed (or NaN)    */
    int32_t status;
    int32_t reserved;
} oracle_info;

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform double in [0,1) for draw (k, w, j) of stream `dom`:
 * counter = (k_lo, k_hi, w, j | dom << 24), key = (seed_lo, seed_hi),
 * u = ((r0 << 32 | r1) >> 11) * 2^-53.  Requires j < 2^24, dom < 256. */
double oracle_uniform(uint64_t seed, uint64_t k, uint32_t w, uint32_t j, uint32_t dom);

/* Squared row norms w_l = sum_c A[l,c]^2 (Eq. (4) numerator), summed left to
 * right with a rounded square and a rounded add per term. */
int oracle_row_norms(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, double* w);

/* Inclusive running sum c_l = c_{l-1} + w_l, left to right.  Returns
 * ORACLE_EZERONORM when the total is zero or not finite. */
int oracle_prefix(const double* w, int64_t m, double* c);

/* Inverse-CDF pick: t = u * c[m-1]; the smallest l with c_l > t; if none,
 * the largest l with w_l > 0. */
int64_t oracle_pick_row(const double* c, const double* w, int64_t m, double u);

/* K*q*bs sampled row indices for iterations iter_offset .. iter_offset+K-1. */
int oracle_indices(const double* w, int64_t m, uint64_t seed, int64_t iter_offset,
                   int64_t K, int32_t q, int32_t bs, int32_t dom, int32_t* idx);

/* RKA with uniform weights (Eq. (7), Algorithm 1). */
int oracle_rka(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
               const double* b, const double* x0, double* x,
               int32_t q, double alpha, int64_t max_iter, double tol, uint64_t seed,
               const double* x_ref, int64_t iter_offset, int64_t check_every,
               oracle_info* info);

/* RKAB (the block-averaging equations of Section 3.4.1, Algorithm 3). */
int oracle_rkab(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                const double* b, const double* x0, double* x,
                int32_t q, int32_t block_size, double alpha, int64_t max_iter,
                double tol, uint64_t seed, const double* x_ref, int64_t iter_offset,
                int64_t check_every, oracle_info* info);

/* The same two iterations driven by a caller-supplied index stream (layout
 * above), K outer iterations, no stopping test.  Used to pin the iteration
 * arithmetic independently of the sampler. */
int oracle_rka_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                     const double* b, double* x, int32_t q, double alpha,
                     int64_t K, const int32_t* idx);
int oracle_rkab_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                      const double* b, double* x, int32_t q, int32_t bs, double alpha,
                      int64_t K, const int32_t* idx);

/* ------------------------------------------------------------------ */
/* Forms built on the iterations (forms_oracle.c).                      */
/* ------------------------------------------------------------------ */

/* The two iterations above with every iteration quantity in binary32
 * ("FP32 accumulation", the inner solves of the precision form): A widened
 * exactly to binary32 (dtype 1 or 2 only), x rounded to binary32 on entry and
 * widened on exit, b_i and ||A^(i)||^2 (binary64 norms as above) rounded to
 * binary32 once per use; dot products left to right; RKA adds the scaled rows
 * in worker order and multiplies by (1/q) rounded to binary32; RKAB divides
 * the worker sum by q. */
int oracle_rka_f32_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         const double* b, double* x, int32_t q, double alpha, int64_t K,
                         const int32_t* idx);
int oracle_rkab_f32_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                          const double* b, double* x, int32_t q, int32_t bs, double alpha,
                          int64_t K, const int32_t* idx);

/* At (n x m, leading dimension m) = A^T, element bits copied. */
int oracle_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At);

/* out_i = (c ? c_i : 0) + gamma * sum_j M[i,j] v_j, binary64, left to right. */
int oracle_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                const double* v, const double* c, double gamma, double* out);

/* Iterative refinement sweeps around inner RKA / RKAB solves (binary32 if
 * acc32), with the residual projected onto range(A) by a column solve when
 * range_iters > 0; measures[s] = the relative error (x_ref) or residual after
 * sweep s.  The steps are listed above the definition. */
int oracle_refine(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
                  const double* x0, double* x, int32_t method, int32_t q, int32_t bs,
                  int32_t acc32, double alpha, int64_t inner_iters, int64_t range_iters,
                  int32_t range_q, double range_alpha, int32_t sweeps, uint64_t seed,
                  const double* x_ref, double* measures);

/* The Distributed Approach of Sec. 3.3.2: worker w samples only its block of
 * rows floor(w m / q) .. floor((w+1) m / q) - 1 (running sum restarted at the
 * block); layout as oracle_indices. */
int oracle_indices_blocks(const double* w, int64_t m, uint64_t seed, int64_t iter_offset,
                          int64_t K, int32_t q, int32_t bs, int32_t dom, int32_t* idx);

/* RKA / RKAB on a given stream with a weight per worker (the partial-matrix
 * alpha of Sec. 3.3.2); walpha: q doubles. */
int oracle_rka_walpha_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                            const double* b, double* x, int32_t q, const double* walpha,
                            int64_t K, const int32_t* idx);
int oracle_rkab_walpha_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                             const double* b, double* x, int32_t q, int32_t bs,
                             const double* walpha, int64_t K, const int32_t* idx);

/* RKA / RKAB on a given stream with the row weights w_i of Eq. (7) in place
 * of a uniform alpha; wrow: m doubles.  In these and the per-worker forms a
 * row of zero norm is a step that leaves the iterate unchanged. */
int oracle_rka_wrow_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                          const double* b, double* x, int32_t q, const double* wrow, int64_t K,
                          const int32_t* idx);
int oracle_rkab_wrow_given(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                           const double* b, double* x, int32_t q, int32_t bs, const double* wrow,
                           int64_t K, const int32_t* idx);

/* The cyclic row order of Sec. 2.1 extended to q workers and blocks of bs:
 * draw (k, w, j) takes row (((k + iter_offset) q + w) bs + j) mod m; layout
 * as oracle_indices. */
int oracle_indices_cyclic(int64_t m, int64_t iter_offset, int64_t K, int32_t q, int32_t bs,
                          int32_t* idx);

/* Cyclic Kaczmarz (Sec. 2.1): iters projections onto rows 0, 1, ..., m-1,
 * 0, ... in turn, row i relaxed by relax[i] (NULL: 1), x updated in place. */
int oracle_ck(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
              double* x, const double* relax, int64_t iters);

#ifdef __cplusplus
}
#endif
#endif
