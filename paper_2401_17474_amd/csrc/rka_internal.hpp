// rka_internal.hpp -- host-side launchers shared between the translation
// units of librka.so (not part of the public C ABI in include/rka.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rka {

struct DevStatus;
struct RowRec;

// Launch of a persistent kernel whose workgroups wait for one another: a
// cooperative launch, for which the runtime checks that the whole grid is
// co-resident; or, with RKA_COOPERATIVE=0 in the environment, a plain launch
// (for tools that do not handle cooperative launches -- rocprofv3 ends with a
// segmentation fault in its exit handlers after a program that made one).
// Every wait inside the kernels is bounded, so a grid that is not
// co-resident ends with RKA_EDEVICE rather than hanging.  (rka_api.hip)
hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args, unsigned lds,
                             hipStream_t s);

// --- sampler side (rka_setup.hip) ------------------------------------------
hipError_t launch_row_norms(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                            bool vec_ok, double* w, hipStream_t s);
hipError_t launch_prefix(const double* w, int64_t m, double* c, int64_t* last_pos, DevStatus* st,
                         hipStream_t s);
// the running sum restarted at each of nseg row blocks; last_pos: nseg entries
hipError_t launch_prefix_blocks(const double* w, int64_t m, int32_t nseg, double* c,
                                int64_t* last_pos, DevStatus* st, hipStream_t s);
// Row orders of the row stream (the `sampling` option of rka_solve_ex).
constexpr int32_t kSampleFull = 0;    // every worker draws from all rows
constexpr int32_t kSampleBlocks = 1;  // worker w draws from its own row block
constexpr int32_t kSampleCyclic = 2;  // rows in order: draw position mod m

// Row stream of K*q*bs draws: indices into idx and/or records (index, b_i,
// ||a_i||^2, weight) into rec (either may be NULL; b and wn are needed for
// rec).  mode kSampleBlocks: c and last_pos from launch_prefix_blocks with
// nseg = q; kSampleCyclic reads neither.  The record's weight is wrow[i] if
// wrow is given, else walpha[w] if walpha is given, else alpha.
hipError_t launch_sample(const double* c, int64_t m, const int64_t* last_pos, uint64_t seed,
                         int64_t k_base, int64_t K, int32_t q, int32_t bs, int32_t dom,
                         int32_t mode, double alpha, const double* walpha, const double* wrow,
                         int32_t* idx, RowRec* rec, const double* b, const double* wn,
                         const DevStatus* st, hipStream_t s);
hipError_t launch_check_finite(const double* v, int64_t len, DevStatus* st, hipStream_t s);

// --- iterations (rka_iter.hip) ---------------------------------------------
// Geometry of the column-split RKA kernel for one problem.
struct RkaColGeom {
  int G;       // workgroups (column slices)
  int nsv;     // vecs per slice
  int rg;      // row groups per workgroup
  int nt;      // threads per workgroup (multiple of 64)
  int rpt;     // rows per thread (template bucket)
  size_t lds;  // dynamic LDS bytes
  int gather;  // one-barrier all-gather of the partials
  int tr;      // lanes per row for the slice sums (power of two <= 64)
  int tr_g;    // lanes per row for the gathered sums (1 without all-gather)
};

struct SolveShape {
  const void* A;
  int dtype;
  int64_t m, n, lda;
  bool vec_ok;
  const double* b;
  const double* wn;
  double* x;
  const double* x_ref;
  double alpha;
  int32_t q, bs;
  int num_cu;
  int grid;       // requested workgroups of the iteration kernel (0 = automatic)
  int allreduce;  // RKA partial-dot exchange: 0 automatic, 1 all-gather, 2 two barriers
  int acc;        // accumulation type: 0 FP64, 1 FP32 (narrow storage only)
};

// Returns false when q rows of a slice do not fit the kernel's register tile.
bool rka_col_plan(const SolveShape& sh, RkaColGeom* geo);

// One chunk of iterations [k0, k0 + K) with row records rec[K*q*bs].
// check_every = 0 disables the in-kernel stopping test (x_ref mode only).
// part / scal: tagged exchange slots (16 bytes each), zeroed once per solve;
// rka_col_slots() gives how many.
hipError_t launch_rka_chunk(const SolveShape& sh, const RkaColGeom& geo, const RowRec* rec,
                            int64_t k0, int64_t K, int64_t check_every, uint64_t* part,
                            uint64_t* scal, DevStatus* st, hipStream_t s);

// Geometry of the RKA kernel with several iterations per exchange
// (rka_sstep.hip): column slices as in the column-split kernel.
struct RkaSstepGeom {
  int G, nsv, rg, nt, rpt;
  int p;       // iterations per exchange (at most; 1 for RKAB)
  int bs;      // projections per worker per iteration (1: RKA)
  int c;       // RKAB: projections per worker per exchange (sub-block)
  int nv;      // exchange values of a full block
  int tr, trp, trs, cg;  // reduction teams (see the kernel's arguments)
  int pg_in_s;           // reduce-scatter gathers into the row-slice buffer
  int pg_len;            // length of its own buffer otherwise
  size_t lds;
};
// RKA (sh.bs = 1): p_req = 0 gives the largest p the tile allows.  RKAB
// (sh.bs > 1, p_req 0 or 1): sub-blocks of the largest c <= bs projections
// per worker that fit (geo->c; c = bs is one exchange per outer iteration).
// False when the shape does not fit (the caller then runs the column-split or
// the worker-split kernel).  FP64 arithmetic only.
bool rka_sstep_plan(const SolveShape& sh, int p_req, RkaSstepGeom* geo);
// part: G x nv tagged slots, red: nv tagged slots, both zeroed once per solve.
hipError_t launch_sstep_chunk(const SolveShape& sh, const RkaSstepGeom& geo, const RowRec* rec,
                              int64_t k0, int64_t K, int64_t check_every, uint64_t* part,
                              uint64_t* red, DevStatus* st, hipStream_t s);

// Geometry of RKA in blocks of p iterations with precomputed coefficients
// (rka_blk.hip): column slices as in the column-split kernel; the
// coefficient pass runs 8 x 8 inner-product tiles of f lanes each.
// Copies of the summed values of a two-phase exchange (column kernel,
// kernels 3 and 4): the reducers write every copy and workgroup g reads copy
// g % kSumCopies, so that each copy's lines are polled by a fraction of the
// workgroups while they are written.
constexpr int kSumCopies = 8;
struct RkaBlkGeom {
  int G, nsv, rg, nt, rpt;
  int nsvp;              // lanes per row group (nsv rounded up to a power of two)
  int p;                 // iterations per exchange (at most)
  int nv;                // exchange values of a full block: p q + 1
  int ncoef;             // coefficients of a full block: q^2 p (p-1) / 2
  int tr, trp, trm;      // reduction teams (see the kernel's arguments)
  size_t lds;
  int cstride;           // doubles between blocks in the coefficient buffer
  int crs;               // coefficient pass: column stride of its staged chunk
  int clcw;              // log2 of its staged chunk's columns
  int cslots;            // its Gram tiles per wave
  int cbuf;              // its LDS-direct staging: bytes per chunk buffer
  size_t clds_dma;       // LDS bytes with LDS-direct staging (0: not possible)
  size_t clds;
  int rkab_bs;           // column-split RKAB: projections per worker (0: RKA)
  int rkab_q;            // column-split RKAB: workers
  int rkab_c;            // column-split RKAB: projections per worker per block
  int rkab_nsub;         // column-split RKAB: blocks per outer iteration
};
// p_req = 0: the largest p that fits (q p <= 128).  FP64 arithmetic, RKA only.
bool rka_blk_plan(const SolveShape& sh, int p_req, RkaBlkGeom* geo);
// Column-split RKAB in the same kernel: one outer iteration per block where
// its q bs rows fit (at most 256, bs <= kRkabBlkMaxBs), else sub-blocks of
// c <= kRkabBlkMaxBs steps per worker (q dividing the row groups); FP64
// arithmetic.
constexpr int kRkabBlkMaxBs = 12;
bool rka_blk_plan_rkab(const SolveShape& sh, RkaBlkGeom* geo);
// blocks of a chunk [k0, k0 + K) with stopping tests every check_every (0: none)
int64_t rka_blk_nblk(const RkaBlkGeom& geo, int64_t k0, int64_t K, int64_t check_every);
// The coefficient pass of a chunk (nothing for p = 1) into coef:
// rka_blk_nblk(...) x cstride doubles.
hipError_t launch_blk_coef(const SolveShape& sh, const RkaBlkGeom& geo, const RowRec* rec,
                           int64_t k0, int64_t K, int64_t check_every, double* coef,
                           const DevStatus* st, hipStream_t s);
// The chunk's iterations from those coefficients; part: G x nv, red: nv
// tagged slots (zeroed once per solve).
hipError_t launch_blk_iter(const SolveShape& sh, const RkaBlkGeom& geo, const RowRec* rec,
                           int64_t k0, int64_t K, int64_t check_every, const double* coef,
                           uint64_t* part, uint64_t* red, DevStatus* st, hipStream_t s);

struct RkabGeom {
  int G;       // workgroups (each runs workers g, g + G, ...)
  int nt;      // threads per workgroup
  int vpt;     // vecs per thread (template bucket)
  int ns;      // vecs per workgroup in the averaging phase
  bool vlds;   // worker iterate kept in LDS instead of registers
  size_t lds;  // dynamic LDS bytes
};
bool rkab_plan(const SolveShape& sh, RkabGeom* geo);
// vbuf: q x n worker iterates in the accumulation type.
hipError_t launch_rkab_chunk(const SolveShape& sh, const RkabGeom& geo, const RowRec* rec,
                             int64_t k0, int64_t K, int64_t check_every, void* vbuf,
                             double* part, unsigned* bar, DevStatus* st, hipStream_t s);

// --- stopping measures (rka_iter.hip) ---------------------------------------
hipError_t launch_status_init(DevStatus* st, double tol, hipStream_t s);
// ||ref||^2 into st->ref2 and tol^2 * ||ref||^2 into st->thresh2
hipError_t launch_ref_norm(const double* ref, int64_t len, double tol, DevStatus* st,
                           hipStream_t s);
// Measure x at iteration k and stop the solve if within tolerance (or
// non-finite).  x_ref != NULL: error measure; else residual (needs part of
// at least resid_blocks() doubles).
hipError_t launch_measure(const SolveShape& sh, int64_t k, double* part, DevStatus* st,
                          hipStream_t s);
int resid_blocks(int64_t m);

// --- dense FP64 steps (rka_dense.hip) --------------------------------------
// out_i = (c ? c_i : 0) + gamma * <M_i, v>, rows x cols, FP64 accumulation.
hipError_t launch_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       bool vec_ok, const double* v, const double* c, double gamma, double* out,
                       hipStream_t s);
hipError_t launch_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At,
                            int64_t ldat, hipStream_t s);
hipError_t launch_axpy(double* x, const double* d, int64_t n, hipStream_t s);
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s);
// zero `bytes` (a multiple of 8) at p with a kernel
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// out_c = (cin ? cin_c : 0) + gamma * sum_i M[i, c] t_i (FP64, fixed order); part holds
// gemvt_part_len(rows, cols) doubles (rka_spectral.hip)
int64_t gemvt_part_len(int64_t rows, int64_t cols);
hipError_t launch_gemvt(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                        const double* t, const double* cin, double gamma, double* out,
                        double* part, hipStream_t s);
// out[0] = sum (a - b)^2 (b may be NULL); part holds sumsq_part_len() doubles
int sumsq_part_len();
hipError_t launch_sumsq(const double* a, const double* b, int64_t len, double* part, double* out,
                        hipStream_t s);
// alpha* of Eq. (6) for q workers from s = sigma^2 / ||A||_F^2 at the extreme
// singular values (rka_spectral.hip)
double alpha_star_eq6(double s_min, double s_max, int q);
// out[i, j] = r_i lam_j - z_i x_j; out_dtype 0 = FP64, 1 = FP32
hipError_t launch_rank2(int64_t m, int64_t n, const double* r, const double* lam, const double* z,
                        const double* x, void* out, int out_dtype, int64_t ldo, hipStream_t s);

}  // namespace rka
