/*
 * rka.h -- C ABI of librka.so: randomized Kaczmarz with averaging (RKA) and
 * its block-averaging variant (RKAB) for dense overdetermined A x = b, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Paper: Ferreira, Acebron, Monteiro, "Parallelization Strategies for the
 * Randomized Kaczmarz Algorithm on Large-Scale Dense Systems", arXiv
 * 2401.17474.  The problem is the one of Sec. 1 (Eqs. (1)-(2)): A in
 * R^{m x n}, b in R^m, find x with A x = b, or the least-squares x when the
 * system is inconsistent; m >= n is the intended use (m < n is accepted).
 *
 * General conventions (apply to every entry point):
 *   - Every array argument is a DEVICE pointer into memory owned by the
 *     caller (for instance a torch tensor's storage).  The library never
 *     frees caller memory.  `info` arguments are HOST pointers.
 *   - A is row-major, m rows of n elements, consecutive rows lda >= n
 *     elements apart.  Element type is given by `dtype` (rka_dtype).  The
 *     fast vector path is used when the base address and the row pitch
 *     (lda * element size) are multiples of 16 bytes and n is a multiple of
 *     16 / element size; other layouts take a scalar path with identical
 *     results for the sampler and row norms.
 *   - b, x0, x, x_ref are FP64 vectors (b: m entries, the others n).
 *   - All work is ordered on `stream` (a hipStream_t; NULL = the null
 *     stream).  Entry points that return an rka_info wait for the stream
 *     once, at the end, to read it back; the others only enqueue work.
 *   - Scratch memory is allocated and freed on `stream` (stream-ordered
 *     allocation); no scratch outlives a call.
 *   - Two identical calls give bitwise identical outputs.  The iteration
 *     (the rows drawn, the projections, the average) depends only on the
 *     inputs and the method parameters (q, block_size, alpha, seed,
 *     iter_offset, max_iter, tol).  Its floating-point rounding also depends
 *     on the launch: the number of workgroups (by default chosen from the
 *     device's compute units and the row length, or the grid option) fixes
 *     the order in which
 *     partial sums meet, and the kernels that run several RKA iterations per
 *     exchange end a block wherever a stopping test falls (every
 *     check_every iterations) or a chunk of iterations ends, so check_every
 *     and the block length move block ends (with tol > 0 the chunks of the
 *     kernel with precomputed coefficients start at max(1024, 4 check_every)
 *     iterations and double).  Results of
 *     different launches agree to rounding (for FP64 arithmetic within
 *     1e-12 relative of the plain iteration in every case tested).
 *   - Return value: an rka_status.  Arguments are validated before any
 *     work is enqueued; a violation returns RKA_EINVAL and touches nothing.
 *     So is a shape that no kernel's register and LDS tiles hold: RKA with
 *     long rows and many workers (FP64, n of about 16000 or more with
 *     q > 88) returns RKA_EINVAL with a message naming n.
 *     No entry point throws, aborts or exits.  rka_status_string() names a
 *     status; rka_last_error() gives a thread-local message for the last
 *     failing call.
 */
#ifndef RKA_H
#define RKA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rka_dtype { RKA_F64 = 0, RKA_F32 = 1, RKA_BF16 = 2 } rka_dtype;

typedef enum rka_status {
    RKA_OK = 0,             /* converged (or ran max_iter with tol == 0)          */
    RKA_NOT_CONVERGED = 1,  /* max_iter reached with tol > 0; x is the last iterate */
    RKA_EINVAL = -1,        /* invalid argument; nothing was enqueued              */
    RKA_EZERONORM = -2,     /* ||A||_F^2 is zero or not finite                     */
    RKA_EDIVERGED = -3,     /* the stopping measure became non-finite              */
    RKA_ENOMEM = -4,        /* scratch allocation failed                           */
    RKA_EDEVICE = -5        /* a HIP call failed (no device, launch error, ...)    */
} rka_status;

typedef struct rka_info {
    int64_t iterations;   /* outer iterations performed                           */
    int64_t projections;  /* row projections performed = iterations * q * bs      */
    double rel_err;       /* last stopping measure computed (NaN if none)         */
    int32_t status;       /* same as the return value                             */
    int32_t reserved;
} rka_info;

/*
 * rka_solve -- RKA with uniform weight alpha, Eq. (7) of Sec. 3.3.1 (Eq. (5)
 * with w_i = alpha): per iteration k, q rows i are drawn independently, with
 * replacement, with probability ||A^(i)||^2 / ||A||_F^2 (Eq. (4)), and
 *     x^(k+1) = x^(k) + (alpha/q) sum_i (b_i - <A^(i), x^(k)>) / ||A^(i)||^2 A^(i)^T.
 * The draw for worker w at iteration k uses Philox4x32-10 with counter
 * (k + iter_offset, w, 0, 0) and key = seed, mapped to u in [0,1) with 53
 * bits, and picks the smallest row l whose running sum of squared row norms
 * (summed left to right) exceeds u * ||A||_F^2.
 *
 *   x0          start vector, or NULL for zero (the paper's usual start).
 *   x           output, n doubles; may alias x0.  Valid when the return
 *               value is >= 0 (RKA_NOT_CONVERGED returns the last iterate).
 *   q           workers averaged per iteration, >= 1 (Sec. 2.3.1).
 *   alpha       relaxation weight, finite and > 0.
 *   max_iter    iteration cap, >= 0.
 *   tol         relative tolerance >= 0.  tol == 0 runs exactly max_iter
 *               iterations.  Otherwise the stopping measure -- ||x - x_ref||
 *               / ||x_ref|| if x_ref is given (Sec. 3.1 stops on the error
 *               to the solution), else ||b - A x|| / ||b|| -- is taken on x^(k)
 *               for every k that is a multiple of check_every and for k =
 *               max_iter; the solve stops at the first k where it is <= tol.
 *   seed        Philox key.
 *   x_ref       reference solution (NULL: use the residual measure).
 *   iter_offset added to k in the random counter, so that a solve of K2
 *               iterations started from the result of a K1-iteration solve
 *               with iter_offset = K1 continues the same stream.
 *   check_every stopping-test interval (values < 1 mean 1).
 */
int rka_solve(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
              const double* x0, double* x, int32_t q, double alpha, int64_t max_iter, double tol,
              uint64_t seed, const double* x_ref, int64_t iter_offset, int64_t check_every,
              void* stream, rka_info* info);

/*
 * rkab_solve -- RKAB, the block-averaging variant of Sec. 3.4.1
 * (Algorithm 3): per outer iteration every worker w starts from
 * v = x^(k) and applies block_size relaxed projections
 *     v <- v + alpha (b_i - <A^(i), v>) / ||A^(i)||^2 A^(i)^T
 * with rows drawn as above using counter (k + iter_offset, w, j, 0) for the
 * j-th projection; then x^(k+1) = (1/q) sum_w v_w.  block_size = 1 is RKA.
 * Arguments as rka_solve; block_size must be in [1, 2^24).  The stopping
 * measure is taken on the averaged iterates only.
 */
int rkab_solve(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
               const double* x0, double* x, int32_t q, int32_t block_size, double alpha,
               int64_t max_iter, double tol, uint64_t seed, const double* x_ref,
               int64_t iter_offset, int64_t check_every, void* stream, rka_info* info);

/* Options of rka_solve_ex.  Zero-initialise and set what you need. */
typedef struct rka_opts {
    int64_t check_every;    /* stopping-test interval, as in rka_solve (< 1 means 1)     */
    int32_t grid;           /* workgroups of the iteration kernel; 0 = chosen by the
                               library.  Changes the summation order (results stay
                               within rounding of each other), never the method.       */
    int32_t collect_timing; /* nonzero: time every phase with HIP events recorded on
                               `stream` and fill the *_ms fields of rka_stats          */
    int32_t allreduce;      /* RKA exchange of the q partial dot products between
                               workgroups: 0 = chosen by the library, 1 = one barrier
                               and every workgroup sums all partials, 2 = two barriers
                               (sums scattered over workgroups).  The two add the
                               partials in different orders: results agree to
                               rounding, each is bitwise reproducible.                */
    int32_t accumulate;     /* 0 = FP64 arithmetic (default); 1 = FP32: the iterate, the
                               dot products, the scales and the average are binary32
                               (the inner solves of the precision form).  FP32 needs
                               RKA_F32 or RKA_BF16 storage, else RKA_EINVAL.  The
                               stopping measures stay FP64 either way.               */
    int32_t stream_id;      /* counter domain `dom` of the row stream, 0..255 (default
                               0; the column solves of the refinement use 1)          */
    int32_t sampling;       /* 0 = every worker samples all rows (default); 1 = the
                               Distributed Approach of Sec. 3.3.2: worker w samples
                               only rows floor(w m / q) .. floor((w+1) m / q) - 1, by
                               their norms within that block (q <= m); 2 = cyclic
                               order (Sec. 2.1): draw (k, w, j) takes row
                               ((k*q + w)*bs + j) mod m with k counted from
                               iter_offset, so q = 1 (RKA) is Cyclic Kaczmarz.  In
                               the cyclic order a row of zero norm is a step that
                               leaves the iterate unchanged; seed is not used.     */
    const double* worker_alpha; /* NULL (every worker uses alpha) or q doubles on the
                               device: worker w's weight (the partial-matrix alpha of
                               Sec. 3.3.2, rka_partial_alpha)                         */
    const double* row_weight; /* NULL or m doubles on the device: the row weights w_i
                               of Eq. (7) (the relaxations alpha_i of Sec. 2.1), used
                               in place of alpha for every projection onto row i.
                               Not combined with worker_alpha (RKA_EINVAL if both).
                               Values are not checked; the convergence results of
                               the paper assume 0 < w_i < 2.                          */
    int32_t steps_per_exchange; /* RKA only: iterations per exchange between
                               workgroups.  0 = chosen by the library; 1 = one (the
                               column-split kernel, or kernel 4 with p = 1 when
                               rka_block = 2); p >= 2 = blocks of up to p iterations
                               whose scales come from one exchange (rka_block says
                               how; the same iteration in exact arithmetic, rounding
                               differs).  Needs FP64 arithmetic and allreduce = 0;
                               if the block does not fit (q p <= 64 for kernel 3,
                               <= 128 for kernel 4), the column-split kernel runs.
                               Blocks end at stopping tests, so check_every = 1
                               gives p = 1.                                           */
    int32_t rkab_split;     /* RKAB only: 0 = chosen by the library; 1 = worker-split
                               (one workgroup per worker, kernel 2); 2 = column-split
                               (every workgroup holds a slice of every worker's rows
                               and of every worker's iterate; an outer iteration runs
                               as sub-blocks of c <= bs projections per worker, q c <=
                               256, one exchange each carrying the rows' dot products
                               with their worker's iterate and each worker's inner
                               products between its rows, from which every workgroup
                               forms each worker's projections in order: the same
                               iteration in exact arithmetic, kernel 3).  2 needs FP64
                               arithmetic and q <= 256, else kernel 2 runs.          */
    int32_t rka_block;      /* RKA with several iterations per exchange, and
                               column-split RKAB: 0 = chosen by the library (kernel 4
                               when it fits: for RKA blocks of several iterations
                               for q <= 64, of one iteration for 64 < q <= 256, else
                               kernel 3 for q <= 16, else the column-split kernel;
                               for column-split RKAB one outer iteration per block
                               when q bs <= 256 and bs <= 12 fit, else sub-blocks of
                               c <= 12 projections per worker (q dividing the
                               workgroup's row groups; every worker's iterate kept
                               for the slice), with M_w = (I + N_w)^-1 per worker
                               from its own rows, N_w[j][l] = alpha_j <a_j, a_l> /
                               ||a_j||^2 for l < j, else kernel 3); 1 = the inner
                               products between the
                               block's rows travel in the exchange (kernel 3); 2 = a
                               streaming pass over the chunk's rows forms, per block,
                               M = (I + N)^-1 with N_{r,c} = alpha_r <a_r, a_c> /
                               (q ||a_r||^2) for rows c of earlier iterations of the
                               block, and the exchange carries only the q p dot
                               products with x^(k): the scales are s = M c with c_r =
                               alpha_r (b_r - <a_r, x^(k)>) / ||a_r||^2 (the same
                               iteration in exact arithmetic, kernel 4; q p <= 128,
                               or p = 1 and q <= 256, else the column-split kernel
                               runs; column-split RKAB that kernel 4 does not hold
                               runs on the worker-split kernel 2, which
                               rka_stats.kernel reports).                             */
} rka_opts;

/* Launch facts and phase times of one rka_solve_ex call. */
typedef struct rka_stats {
    double norms_ms;          /* squared row norms                                     */
    double prefix_ms;         /* running sum                                           */
    double sample_ms;         /* row stream, summed over chunks                        */
    double iterate_ms;        /* persistent iteration kernel, summed over chunks       */
    double measure_ms;        /* stopping measures                                     */
    int64_t iterate_launches; /* chunks (launches of the iteration kernel)             */
    int32_t kernel;           /* 1 = column-split RKA kernel, 2 = worker-split kernel,
                                 3 = RKA with several iterations per exchange, 4 = the
                                 same with coefficients from a streaming pass           */
    int32_t grid;             /* workgroups of the iteration kernel                    */
    int32_t threads;          /* threads per workgroup of the iteration kernel         */
    int32_t bucket;           /* register-tile bucket of the kernel instance: rows per
                                 thread (kernel 1) or 16-byte vecs per thread (kernel 2) */
    int32_t variant;          /* kernel 1: 1 = one-barrier all-gather of the partials;
                                 kernel 2: 1 = worker iterate kept in LDS;
                                 kernels 3 and 4: RKA iterations per exchange (p), or
                                 RKAB projections per worker per exchange (c; c < bs:
                                 sub-blocks)                                      */
    int32_t accumulate;       /* accumulation type used: 0 = FP64, 1 = FP32             */
    double coef_ms;           /* kernel 4: the coefficient passes, summed over chunks
                                 (not in iterate_ms); 0 for the other kernels           */
} rka_stats;

/*
 * rka_solve_ex -- rka_solve (method 0) or rkab_solve (method 1) with extra
 * options and launch statistics.  opts may be NULL (defaults, check_every =
 * 1); stats may be NULL.  block_size is ignored for method 0.  Everything
 * else is as documented for rka_solve / rkab_solve.
 */
int rka_solve_ex(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
                 const double* x0, double* x, int32_t method, int32_t q, int32_t block_size,
                 double alpha, int64_t max_iter, double tol, uint64_t seed, const double* x_ref,
                 int64_t iter_offset, const rka_opts* opts, void* stream, rka_info* info,
                 rka_stats* stats);

/*
 * rka_solve_ex_noalloc -- rka_solve_ex for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same arguments, iteration and results, with
 * every scratch buffer carved from a fixed 64 MiB device array of the library
 * instead of stream-ordered allocations.  The call makes no hipMalloc /
 * hipFree or other allocating call; the caller still passes A, b, x0, x and
 * x_ref.  The array holds the squared row norms and running sum (16 m
 * bytes), the exchange slots or worker iterates of the chosen kernel, and
 * the row records of one chunk (32 bytes per projection; chunks are
 * shortened to fit, which for RKA with several iterations per exchange moves
 * block ends and so changes results at rounding level).  A problem whose
 * fixed buffers plus one iteration of records exceed 64 MiB is rejected with
 * RKA_EINVAL before anything is enqueued.  opts->collect_timing is ignored
 * (no events are created).  Every call on one device shares that device's
 * array: calls that overlap on a device (on different streams or threads)
 * race and give undefined results; calls ordered on one stream are safe
 * (each clears what it needs zeroed).  Each device that runs it holds its
 * own copy of the array; its address is looked up once per device.
 */
int rka_solve_ex_noalloc(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         const double* b, const double* x0, double* x, int32_t method, int32_t q,
                         int32_t block_size, double alpha, int64_t max_iter, double tol,
                         uint64_t seed, const double* x_ref, int64_t iter_offset,
                         const rka_opts* opts, void* stream, rka_info* info, rka_stats* stats);

/*
 * rka_row_norms -- w_l = sum_c A[l,c]^2 for every row (the numerators of
 * Eq. (4)), each summed left to right in FP64 with a rounded square and a
 * rounded add per term (narrow types widen exactly first).  w: m doubles.
 * Enqueue only.
 */
int rka_row_norms(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, double* w,
                  void* stream);

/*
 * rka_prefix -- running sum c_l = c_{l-1} + w_l, left to right, so that
 * c[m-1] = ||A||_F^2 (Eq. (4) denominator); also stores in *last_pos (device
 * int64, may be NULL) the largest l with w_l > 0.  Waits for the stream to
 * read c[m-1] back and returns RKA_EZERONORM if it is zero or not finite.
 */
int rka_prefix(const double* w, int64_t m, double* c, int64_t* last_pos, void* stream);

/*
 * rka_sample_indices -- the row stream both solvers use: for k in [0, K),
 * w in [0, q), j in [0, bs): idx[(k*q + w)*bs + j] = the row picked by the
 * draw with counter (k + iter_offset, w, j, dom) and key seed (see
 * rka_solve).  w, c as produced by rka_row_norms / rka_prefix; idx: K*q*bs
 * int32 on the device.  dom in [0, 255] selects an independent stream (0 is
 * the solvers' row stream).  Enqueue only.
 */
int rka_sample_indices(const double* w, const double* c, int64_t m, uint64_t seed,
                       int64_t iter_offset, int64_t K, int32_t q, int32_t bs, int32_t dom,
                       int32_t* idx, void* stream);

/*
 * rka_gemv -- out_i = (c ? c_i : 0) + gamma * sum_j M[i,j] v_j for i < rows,
 * in FP64 (narrow storage widens exactly).  M is rows x cols with leading
 * dimension ld; v: cols doubles; c (nullable) and out: rows doubles (out
 * may alias c).  With c = b, gamma = -1 this is the residual b - A x; on a
 * transposed copy it forms A^T r.  Each row's sum has a fixed order.
 * Enqueue only.
 */
int rka_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld, const double* v,
             const double* c, double gamma, double* out, void* stream);

/*
 * rka_gemv_t -- out_c = (c ? c_c : 0) + gamma * sum_i M[i,c] t_i for c < cols
 * (A^T t without a transposed copy), FP64: blocks of 512 rows form partial
 * column sums, added in block order (bitwise reproducible).  t: rows doubles;
 * c (nullable) and out: cols doubles (out may alias c).  rows must be below
 * 65535 * 512.  Allocates and frees its partial sums on the stream.
 */
int rka_gemv_t(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld, const double* t,
               const double* c, double gamma, double* out, void* stream);

/*
 * rka_spectral_bounds -- the extreme squared singular values sigma_min^2 and
 * sigma_max^2 of A (over its min(m, n) singular values), which alpha* of
 * Eq. (6) needs as s = sigma^2 / ||A||_F^2.  Lanczos with full
 * reorthogonalisation on the smaller of A^T A and A A^T, from a Philox start
 * vector (key seed, stream dom 2), min(steps, min(m, n)) steps, two streaming
 * passes over A per step; the extreme Ritz values by Sturm bisection.  Ritz
 * values lie inside the spectrum: *lam_min >= sigma_min^2 and
 * *lam_max <= sigma_max^2, both converging with steps (exact at steps =
 * min(m, n) in exact arithmetic).  *fro2 (nullable) = ||A||_F^2 from the
 * squared row norms.  Host outputs; waits for the stream.  m must be below
 * 65535 * 512.
 */
int rka_spectral_bounds(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, int32_t steps,
                        uint64_t seed, void* stream, double* lam_min, double* lam_max,
                        double* fro2);

/*
 * rka_partial_alpha -- the partial-matrix weights of Sec. 3.3.2: for every
 * worker w, Eq. (6) evaluated with q and the extreme squared singular values
 * of its own row block A[floor(w m / q) .. floor((w+1) m / q) - 1, :] over
 * that block's squared Frobenius norm (rka_spectral_bounds on the block, key
 * seed + w).  alpha_out: q doubles on the host.  Use them with
 * rka_opts.worker_alpha (copied to the device).  Waits for the stream.
 */
int rka_partial_alpha(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, int32_t q,
                      int32_t steps, uint64_t seed, void* stream, double* alpha_out);

/*
 * rka_transpose -- At[j, i] = A[i, j] (element bits copied), so that the
 * columns of A become contiguous rows for the column solves.  At: n rows of
 * m elements, leading dimension ldat >= m, same dtype; must not overlap A.
 * m must be below 65535 * 64.  Enqueue only.
 */
int rka_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At,
                  int64_t ldat, void* stream);

/*
 * rka_lsq_grad_A -- dA[i, j] = r_i lambda_j - z_i x_j (formed in FP64, stored
 * as out_dtype = RKA_F64 or RKA_F32, leading dimension ldd >= n): the gradient
 * of a loss L(x) through the least-squares solution x = argmin ||A x - b||
 * with respect to A, where r = b - A x, z = dL/db (the minimum-norm solution
 * of A^T z = dL/dx) and lambda solves A lambda = z.  r, z: m doubles;
 * lambda, x: n doubles.  Enqueue only.
 */
int rka_lsq_grad_A(int64_t m, int64_t n, const double* r, const double* lam, const double* z,
                   const double* x, void* dA, int out_dtype, int64_t ldd, void* stream);

/* Options of rka_refine_solve. */
typedef struct rka_refine_opts {
    int32_t method;       /* inner solver: 0 = RKA (rka_solve), 1 = RKAB (rkab_solve)    */
    int32_t q;            /* inner workers, >= 1                                         */
    int32_t block_size;   /* inner RKAB block size (method 1)                            */
    int32_t accumulate;   /* inner arithmetic: 0 = FP64, 1 = FP32 (narrow storage only)  */
    double alpha;         /* inner relaxation weight, finite and > 0                     */
    int64_t inner_iters;  /* outer iterations of every inner row solve, >= 0             */
    int64_t range_iters;  /* iterations of the column solve that projects the residual
                             onto range(A) (0: plain refinement, for consistent systems) */
    int32_t range_q;      /* workers of the column solve                                 */
    int32_t max_sweeps;   /* refinement sweeps, >= 1                                     */
    double range_alpha;   /* relaxation weight of the column solve                       */
    double tol;           /* stop after the first sweep whose measure is <= tol
                             (0: run max_sweeps)                                         */
} rka_refine_opts;

typedef struct rka_refine_info {
    int32_t sweeps;       /* sweeps performed                                            */
    int32_t status;       /* same as the return value                                    */
    double rel;           /* measure after the last sweep                                */
    int64_t projections;  /* row projections of all inner solves                         */
} rka_refine_info;

/*
 * rka_refine_solve -- mixed-precision iterative refinement around the
 * Kaczmarz solves, for the least-squares problem of Eq. (2).  Per sweep s:
 *     r = b - A x                      (FP64, rka_gemv)
 *     if range_iters > 0:              (inconsistent systems)
 *         g = A^T r                    (FP64, on the transposed copy At)
 *         y = RKA on the columns, A^T y = g from y = 0: range_iters iterations,
 *             range_q workers, weight range_alpha, row stream dom = 1 with
 *             iter_offset = s * range_iters -- converges to the projection of
 *             r onto range(A), so that the next system is consistent
 *         r = y
 *     d = RKA / RKAB on A d = r from d = 0: inner_iters iterations, dom = 0,
 *         iter_offset = s * inner_iters, accumulation as `accumulate`
 *     x = x + d                        (FP64)
 * then the measure ||x - x_ref|| / ||x_ref|| (x_ref given) or ||b - A x|| /
 * ||b|| is written to sweep_measure[s] (host array of max_sweeps doubles,
 * nullable).  With x_ref and tol > 0 the inner solve also stops early, at
 * the first multiple of 25 iterations where ||d - (x_ref - x)|| <= tol
 * ||x_ref|| (the sweep's own stopping test, measured on the correction).  Plain RKA stops at the convergence horizon set by the
 * least-squares residual (Sec. 2.3.1); the range projection removes that
 * residual from every correction, so the sweeps converge to the
 * least-squares solution itself.  With FP32 accumulation every inner solve
 * is accurate to roughly FP32 rounding and the FP64 residual recovers the
 * rest.  A, b, x, x0, x_ref as in rka_solve; At: the n x m transpose of A
 * (rka_transpose), needed only when range_iters > 0.  Waits for the stream
 * once per sweep.  Returns RKA_OK (converged, or tol == 0),
 * RKA_NOT_CONVERGED (max_sweeps reached with tol > 0), or an error.
 */
int rka_refine_solve(const void* A, const void* At, int dtype, int64_t m, int64_t n, int64_t lda,
                     int64_t ldat, const double* b, const double* x0, double* x,
                     const rka_refine_opts* opts, uint64_t seed, const double* x_ref,
                     double* sweep_measure, void* stream, rka_refine_info* info);

/* One system of a batch (rka_batch_solve).  nrhs right-hand sides share A
 * and one row stream. */
typedef struct rka_batch_system {
    const void* A;          /* m x n, leading dimension lda (dtype of the batch)       */
    int64_t m, n, lda;      /* 1 <= m < 2^31, 1 <= n <= 4096                           */
    const double* b;        /* right-hand side r at b + r * ldb (ldb >= m)             */
    int64_t ldb;
    double* x;              /* iterate r at x + r * ldx (ldx >= n): start in, result
                               out                                                    */
    int64_t ldx;
    const double* x_ref;    /* nullable: reference r at x_ref + r * ldxr for the
                               stopping test                                          */
    int64_t ldxr;
    int32_t nrhs;           /* >= 1                                                    */
    int32_t q;              /* workers; 0 = chosen by the library                      */
    int32_t block_size;     /* projections per worker and iteration; 0 = chosen       */
    int32_t tpr;            /* threads per row (16, 32, 64, 128 or 256 with
                               16 tpr >= n); 0 = chosen                               */
    int32_t rhs_per_task;   /* right-hand sides one workgroup carries (<= 8); 0 =
                               the most that fit 64 KB of LDS                         */
    int32_t reserved;
    double alpha;           /* relaxation weight, finite and > 0; 0 = chosen by the
                               tuner (1 if the batch is not tuned)                    */
    int64_t max_iter;       /* iteration cap, >= 0                                     */
} rka_batch_system;

typedef struct rka_batch_result {
    int64_t iterations;     /* iterations run (the largest over the system's tasks)   */
    double rel;             /* largest last relative error over its tasks (0 if none) */
    double alpha;           /* relaxation weight used                                  */
    int32_t status;         /* RKA_OK, RKA_NOT_CONVERGED or RKA_EDIVERGED              */
    int32_t q, block_size, tpr, rhs_per_task;  /* parameters used                      */
    int32_t reserved;
} rka_batch_result;

typedef struct rka_batch_stats {
    int32_t tasks;          /* workgroup tasks (systems x right-hand-side groups)     */
    int32_t chunks;         /* row-stream chunks                                      */
    int32_t lds_bytes;      /* dynamic LDS of the iteration launch                    */
    int32_t graph;          /* 1 if the launches ran as one captured HIP graph         */
    double setup_ms;        /* plain launches: row norms and running sums (HIP events) */
    double iterate_ms;      /* plain launches: the chunks of iterations; graph: the
                               whole graph (set-up included)                          */
} rka_batch_stats;

/*
 * rka_batch_solve -- RKAB (Sec. 3.4.1; block_size = 1 is RKA, Eq. (7)) on
 * `count` independent systems at once, every iteration in binary32 on FP32
 * or BF16 storage (dtype RKA_F32 / RKA_BF16).  System i draws its rows with
 * key seed + i and counter (k, w, j, 0) exactly as rka_solve / rkab_solve
 * do, from its own squared row norms (Eq. (4)); the nrhs right-hand sides of
 * a system share that row stream, so each sampled row is read once per
 * group of rhs_per_task right-hand sides.  Iteration k of every worker is
 *     v = x^(k);  bs times: v += alpha (b_i - <A^(i), v>) / ||A^(i)||^2 A^(i)^T
 *     x^(k+1) = (sum_w v_w) / q                (binary32, worker order)
 * With tol > 0 and x_ref given, a group stops after the first multiple of
 * check_every where ||x - x_ref|| <= tol ||x_ref|| over its right-hand sides,
 * or (status RKA_NOT_CONVERGED) once its squared error has not halved for
 * 60000 dependent projection steps (iterations x (block_size + 2)) -- the
 * rounding floor of a binary32 iteration, which rka_batch_refine_solve goes
 * below.
 * chunk_iters > 0 caps the iterations per chunk (0: as many as keep the
 * chunk's row streams within 64 Mi indices).  use_graph != 0 captures the whole launch sequence (set-up, then per chunk
 * of iterations a row-stream launch and one iteration launch for all
 * systems) in one HIP graph and launches it once; `stream` must then not be
 * the null stream.  results: host array of count entries (nullable).  Waits
 * for the stream once.  Returns RKA_OK, RKA_NOT_CONVERGED (some system did
 * not reach tol), RKA_EDIVERGED, or an error.
 */
int rka_batch_solve(const rka_batch_system* systems, int32_t count, int dtype, uint64_t seed,
                    double tol, int64_t check_every, int64_t chunk_iters, int32_t use_graph,
                    void* stream, rka_batch_result* results, rka_batch_stats* stats);

/*
 * rka_batch_sample_indices -- parity hook of the batching form: runs the set-up
 * and the row-stream launches of rka_batch_solve (same chunks of chunk_iters
 * iterations, 0 = the library's chunk length) without iterating, and copies
 * the draws: system i's max_iter * q * block_size row indices, layout
 * [(k * q + w) * block_size + j] as rka_sample_indices, at idx + sum over
 * j < i of max_iter_j * q_j * block_size_j (device int32).  Every system must
 * give q >= 1 and block_size >= 1; x is not touched.  Waits for the stream.
 */
int rka_batch_sample_indices(const rka_batch_system* systems, int32_t count, int dtype,
                             uint64_t seed, int64_t chunk_iters, int32_t* idx, void* stream);

/*
 * rka_batch_refine_solve -- the batch with FP64 iterative refinement (the
 * precision form of rka_refine_solve, for consistent systems): per sweep s,
 * r = b - A x in FP64 for every system and right-hand side, then one batch
 * solve as rka_batch_solve (binary32) of A d = r from d = 0 with keys
 * seed + s * 65536 + i, then x += d in FP64.  With x_ref and tol > 0 a task
 * stops once ||x + d - x_ref|| <= tol ||x_ref|| and the sweeps end when every
 * system has; this reaches accuracies below the binary32 rounding floor of
 * one batch solve.  results: iterations summed over sweeps, rel and status of
 * the last sweep.  Other arguments as rka_batch_solve (chunk length chosen
 * by the library).
 */
int rka_batch_refine_solve(const rka_batch_system* systems, int32_t count, int dtype,
                           uint64_t seed, double tol, int64_t check_every, int32_t sweeps,
                           int32_t use_graph, void* stream, rka_batch_result* results,
                           rka_batch_stats* stats);

/*
 * rka_batch_tune -- the batching form's autotuner.  Groups the systems by
 * size class (n rounded up to a power of two) and runs candidates on each
 * class's median system for about m/2 projections, measuring the residual
 * reduction per millisecond and per projection.  Candidates: tpr in {t0,
 * 2 t0} with t0 the smallest that covers a row and W = 256 / tpr workers per
 * workgroup; RKAB with alpha = 1, q in {1, W/4, W}, block_size in {n/8, n/2}
 * clipped to [1, 256]; and RKA (block size 1) with q = W, alpha in {W/4,
 * W/2}.  The choice per class minimises the modelled batch time to a
 * 10^-6 residual reduction: the larger of the slowest class's own time and
 * the row bytes of all tasks at 5 TB/s.  Writes q, block_size, tpr and alpha
 * into every system of a class where they are 0; x is not touched.  Meant for
 * consistent systems (the residual is the progress measure).  *trials
 * (nullable) = candidates timed.
 */
int rka_batch_tune(rka_batch_system* systems, int32_t count, int dtype, uint64_t seed,
                   void* stream, int32_t* trials);

/*
 * rka_sample_blocks -- the row stream of the Distributed Approach (Sec. 3.3.2):
 * draw (k, w, j) with counter (k + iter_offset, w, j, dom) picks, within
 * worker w's block of rows floor(w m / q) .. floor((w+1) m / q) - 1, the
 * smallest row whose running sum restarted at the block exceeds u times the
 * block's total (falling back to the block's last row of positive weight).
 * w: the m squared row norms (rka_row_norms); idx: K*q*bs int32, layout as
 * rka_sample_indices.  Waits for the stream; RKA_EZERONORM if a block has
 * zero weight.
 */
int rka_sample_blocks(const double* w, int64_t m, uint64_t seed, int64_t iter_offset, int64_t K,
                      int32_t q, int32_t bs, int32_t dom, int32_t* idx, void* stream);

/*
 * Plans: the sampling distribution of Eq. (4) as a per-matrix object.  A plan
 * holds, on the device it was made on, the squared row norms w_l of A
 * (rka_row_norms' order), their running sum c (rka_prefix's order), W =
 * ||A||_F^2 and the last row of positive weight, computed once; every solve,
 * refinement and row stream over the same A then skips that set-up (a pass
 * over A and a sequential sum over its m rows).  The plan refers to A by
 * pointer: A must stay allocated and unchanged while the plan is used.
 */
typedef struct rka_plan rka_plan;

/*
 * rka_plan_create -- make a plan for A (layout and dtype as in rka_solve):
 * allocates 16 m + 264 bytes of device memory (hipMalloc), enqueues the row
 * norms and the running sum on `stream` and waits for it to read W back.
 * *plan receives the handle (NULL on failure).  RKA_EZERONORM if W is zero
 * or not finite (nothing is kept), RKA_ENOMEM if the allocation fails.
 */
int rka_plan_create(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* stream,
                    rka_plan** plan);

/* rka_plan_destroy -- free a plan's device memory (hipFree, which waits for
 * the device); NULL is accepted.  No call may still use the plan. */
int rka_plan_destroy(rka_plan* plan);

/* rka_plan_query -- m, n, ||A||_F^2 and the last row of positive weight of a
 * plan (each output nullable; last_pos is read from the device, waiting for
 * the null stream). */
int rka_plan_query(const rka_plan* plan, int64_t* m, int64_t* n, double* fro2, int64_t* last_pos);

/* rka_plan_row_norms -- copy the plan's m squared row norms (Eq. (4)
 * numerators, as rka_row_norms computes them) to w (m doubles, device).
 * Enqueue only. */
int rka_plan_row_norms(const rka_plan* plan, double* w, void* stream);

/* rka_plan_sample_indices -- the row stream of rka_sample_indices (same
 * counters, same layout idx[(k*q + w)*bs + j]) from the plan's running sum.
 * Enqueue only. */
int rka_plan_sample_indices(const rka_plan* plan, uint64_t seed, int64_t iter_offset, int64_t K,
                            int32_t q, int32_t bs, int32_t dom, int32_t* idx, void* stream);

/*
 * rka_plan_solve -- rka_solve_ex on the plan's matrix: the same iteration,
 * options and results (bitwise: the plan's norms and running sum are the
 * ones the solve would compute), without the per-call set-up.  With
 * opts->sampling = 1 (Distributed Approach) the running sum is still
 * restarted per worker block, from the plan's norms.
 */
int rka_plan_solve(const rka_plan* plan, const double* b, const double* x0, double* x,
                   int32_t method, int32_t q, int32_t block_size, double alpha, int64_t max_iter,
                   double tol, uint64_t seed, const double* x_ref, int64_t iter_offset,
                   const rka_opts* opts, void* stream, rka_info* info, rka_stats* stats);

/*
 * rka_plan_refine_solve -- rka_refine_solve on the plans of A and of its
 * transpose At (pAt nullable when opts->range_iters == 0; else a plan of the
 * n x m transpose, same dtype).  rka_refine_solve itself builds both plans
 * once per call, in stream-ordered scratch.
 */
int rka_plan_refine_solve(const rka_plan* pA, const rka_plan* pAt, const double* b,
                          const double* x0, double* x, const rka_refine_opts* opts, uint64_t seed,
                          const double* x_ref, double* sweep_measure, void* stream,
                          rka_refine_info* info);

/*
 * rka_alpha_star -- the optimal uniform weight of Eq. (6) (Sec. 2.3.1) for q
 * workers, from s_min = sigma_min^2 / ||A||_F^2 and s_max = sigma_max^2 /
 * ||A||_F^2 (rka_spectral_bounds):
 *     alpha* = q / (1 + (q-1) s_min)                if s_max - s_min <= 1/(q-1),
 *     alpha* = 2q / (1 + (q-1) (s_min + s_max))     otherwise
 * (q = 1 takes the first case).  *alpha (host) receives it; RKA_EINVAL
 * unless q >= 1 and 0 <= s_min <= s_max <= 1.
 */
int rka_alpha_star(double s_min, double s_max, int32_t q, double* alpha);

/* Name of a status code (static string). */
const char* rka_status_string(int status);

/* Message describing the last failure on the calling thread ("" if none). */
const char* rka_last_error(void);

/* Library version, as major*10000 + minor*100 + patch. */
int rka_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RKA_H */
