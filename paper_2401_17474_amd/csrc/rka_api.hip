// rka_api.hip -- the C ABI declared in include/rka.h: argument validation,
// stream-ordered scratch, and the sequence of launches of one solve:
//
//   status init -> b finite check -> row norms -> running sum (+ W check)
//   -> [reference norm, measure at k = 0]
//   -> for each chunk: row stream for the chunk -> persistent iteration
//      kernel [-> residual measure at multiples of check_every]
//   -> [final measure at k = max_iter] -> one read-back of the status.
//
// Later launches of a solve see the device status and return at once when
// an earlier one decided to stop, so the host never waits mid-solve.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>

#include "rka.h"
#include "rka_device.hpp"
#include "rka_internal.hpp"

// A plan (rka_plan_create): the squared row norms of one matrix, their
// running sum and its last row of positive weight (Eq. (4)), computed once
// and kept on the device for every solve and row stream over that matrix.
struct rka_plan {
  const void* A;
  int dtype;
  int64_t m, n, lda;
  bool vec_ok;
  int device;
  double* w;          // m squared row norms
  double* c;          // m running sums; c[m-1] = ||A||_F^2
  int64_t* last_pos;  // the largest row with w > 0
  double fro2;        // ||A||_F^2, read back at creation
  void* mem;          // one allocation holding w, c and last_pos (public plans)
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int esize(int dtype) { return dtype == RKA_F64 ? 8 : (dtype == RKA_F32 ? 4 : 2); }

bool vector_path_ok(const void* A, int dtype, int64_t n, int64_t lda) {
  const int es = esize(dtype);
  const int V = 16 / es;
  return ((uintptr_t)A % 16 == 0) && ((lda * es) % 16 == 0) && (n % V == 0);
}

int num_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

// Scratch for one call: stream-ordered allocations freed (on the stream) by
// release(), or -- arena mode -- pieces of caller-provided device memory
// (256-byte aligned) that nothing frees.
struct Scratch {
  hipStream_t s;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  void* ptrs[16];
  int n = 0;
  explicit Scratch(hipStream_t st) : s(st) {}
  Scratch(hipStream_t st, void* base, size_t bytes) : s(st), arena((char*)base), cap(bytes) {}
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
  template <typename U>
  hipError_t get(U** out, size_t count) {
    const size_t bytes = count * sizeof(U) > 0 ? count * sizeof(U) : 16;
    if (arena) {
      if (used + round(bytes) > cap) return hipErrorOutOfMemory;
      *out = (U*)(arena + used);
      used += round(bytes);
      return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess) return e;
    ptrs[n++] = p;
    *out = (U*)p;
    return hipSuccess;
  }
  void release() {
    for (int i = n - 1; i >= 0; --i) (void)hipFreeAsync(ptrs[i], s);
    n = 0;
  }
  ~Scratch() { release(); }
};

// Phase timing with HIP events recorded on the solve's stream.
enum Phase { kNorms = 0, kPrefix, kSample, kIterate, kMeasure, kCoef, kPhases };
struct PhaseTimer {
  hipStream_t s;
  bool on;
  struct Span {
    int phase;
    hipEvent_t a, b;
  };
  Span spans[4096];
  int n = 0;
  int open = -1;
  PhaseTimer(hipStream_t st, bool enabled) : s(st), on(enabled) {}
  void begin(int phase) {
    if (!on || n >= 4096) return;
    Span& sp = spans[n];
    if (hipEventCreate(&sp.a) != hipSuccess) return;
    if (hipEventCreate(&sp.b) != hipSuccess) {
      (void)hipEventDestroy(sp.a);
      return;
    }
    sp.phase = phase;
    (void)hipEventRecord(sp.a, s);
    open = n;
  }
  void end() {
    if (open < 0) return;
    (void)hipEventRecord(spans[open].b, s);
    n = open + 1;
    open = -1;
  }
  // after the stream has been synchronized
  void collect(double out[kPhases]) {
    for (int i = 0; i < kPhases; ++i) out[i] = 0.0;
    for (int i = 0; i < n; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, spans[i].a, spans[i].b) == hipSuccess)
        out[spans[i].phase] += ms;
    }
  }
  ~PhaseTimer() {
    for (int i = 0; i < n; ++i) {
      (void)hipEventDestroy(spans[i].a);
      (void)hipEventDestroy(spans[i].b);
    }
  }
};

#define HIP_TRY(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? RKA_ENOMEM : RKA_EDEVICE, "%s: %s", #call,   \
                  hipGetErrorString(e_));                                                   \
    }                                                                                       \
  } while (0)

bool bad_dtype(int d) { return d != RKA_F64 && d != RKA_F32 && d != RKA_BF16; }

int validate(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
             double* x, int32_t q, int32_t bs, double alpha, int64_t max_iter, double tol,
             int64_t iter_offset) {
  if (!A || !b || !x) return fail(RKA_EINVAL, "A, b and x must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1) return fail(RKA_EINVAL, "m and n must be >= 1 (got %lld, %lld)",
                                  (long long)m, (long long)n);
  if (m > INT32_MAX) return fail(RKA_EINVAL, "m must be < 2^31");
  if (lda < n) return fail(RKA_EINVAL, "lda (%lld) must be >= n (%lld)", (long long)lda,
                           (long long)n);
  if (q < 1) return fail(RKA_EINVAL, "q must be >= 1");
  if (bs < 1 || bs >= (1 << 24)) return fail(RKA_EINVAL, "block_size must be in [1, 2^24)");
  if (!(alpha > 0.0) || !isfinite(alpha)) return fail(RKA_EINVAL, "alpha must be finite and > 0");
  if (max_iter < 0) return fail(RKA_EINVAL, "max_iter must be >= 0");
  if (!(tol >= 0.0) || !isfinite(tol)) return fail(RKA_EINVAL, "tol must be finite and >= 0");
  if (iter_offset < 0) return fail(RKA_EINVAL, "iter_offset must be >= 0");
  return RKA_OK;
}

// Row records per chunk: at most 4 Mi entries (128 MiB).
constexpr int64_t kRecBudget = 4ll << 20;
// Kernel 4's coefficients per chunk: at most 512 MiB.
constexpr int64_t kCoefBudget = 512ll << 20;
// Kernel 4's first chunk where a stopping test may end the solve (iterations;
// the chunks after it double).
constexpr int64_t kFirstBlkChunk = 1024;
// Largest q for which the library runs several RKA iterations per exchange
// by itself (steps_per_exchange = 0): measured at 80000 x 10000 FP64, blocks
// of 64 / q iterations take 4.5 us per iteration at q = 16 (one-iteration
// kernel: 5.5 us at its best grid) and 2.7 us at q = 8 (5.2 us); at q = 32
// the block's exchange outweighs the saved round trips.
constexpr int kAutoSstepMaxQ = 16;
// RKAB with at most a quarter as many workers as CUs runs column-split
// (every workgroup holds a slice of every worker's rows) when the q bs rows
// of an outer iteration fit one exchange of the block kernel, or in
// sub-blocks when q is at most kAutoSubBlockMaxQ.  Measured at 80000 x 10000
// FP64, us per outer iteration, worker-split -> column-split: q = 16,
// bs = 10: 54 -> 22; q = 8, bs = 10: 37 -> 18; q = 32, bs = 4: 24 -> 16;
// q = 64, bs = 2: 29 -> 15; q = 4, bs = 32: 94 -> 35.
constexpr int kAutoSubBlockMaxQ = 16;
// RKA blocks with coefficients from a streaming pass (kernel 4) are the
// library's choice up to q = 256 wherever they fit: several iterations per
// block up to q = 64, one above.  Measured at 80000 x 10000 FP64, us per
// iteration with the coefficient pass included, kernel 4 against the best
// other kernel: q = 8: 1.07 (2.54, kernel 3); q = 16: 1.92 (4.4, kernel 3);
// q = 32: 3.45 (7.1, one-iteration kernel); q = 64: 6.1 (7.8); q = 96: 8.1
// (9.2); q = 128: 9.1 (10.0); q = 160: 10.7 (12.5).  With one iteration per
// block at 20000 x 1000 and 40000 x 5000, q = 96 to 256: 2% to 46% faster
// than the one-iteration kernel.
constexpr bool kAutoBlk = true;
constexpr int kAutoBlkMaxQ = 256;

int solve_impl(bool block, const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
               const double* b, const double* x0, double* x, int32_t q, int32_t bs, double alpha,
               int64_t max_iter, double tol, uint64_t seed, const double* x_ref,
               int64_t iter_offset, int64_t check_every, int grid, int allreduce, bool timing,
               int acc, int dom, int sampling, const double* walpha, const double* wrow,
               int sstep, int split, void* stream, rka_info* info, rka_stats* stats,
               const rka_plan* plan = nullptr, void* arena = nullptr, size_t arena_bytes = 0,
               int rblk = 0) {
  g_last_error.clear();
  if (stats) memset(stats, 0, sizeof *stats);
  if (info) {
    info->iterations = 0;
    info->projections = 0;
    info->rel_err = NAN;
    info->status = RKA_EINVAL;
    info->reserved = 0;
  }
  int v = validate(A, dtype, m, n, lda, b, x, q, bs, alpha, max_iter, tol, iter_offset);
  if (v != RKA_OK) return v;
  if (check_every < 1) check_every = 1;
  if (grid < 0) return fail(RKA_EINVAL, "grid must be >= 0");
  if (allreduce < 0 || allreduce > 2) return fail(RKA_EINVAL, "allreduce must be 0, 1 or 2");
  if (acc < 0 || acc > 1) return fail(RKA_EINVAL, "accumulate must be 0 (FP64) or 1 (FP32)");
  if (acc == 1 && dtype == RKA_F64)
    return fail(RKA_EINVAL, "FP32 accumulation needs RKA_F32 or RKA_BF16 storage");
  if (dom < 0 || dom > 255) return fail(RKA_EINVAL, "stream_id must be in [0, 255]");
  if (sampling < rka::kSampleFull || sampling > rka::kSampleCyclic)
    return fail(RKA_EINVAL, "sampling must be 0, 1 or 2");
  if (walpha && wrow) return fail(RKA_EINVAL, "give worker_alpha or row_weight, not both");
  if (sstep < 0 || sstep > 64) return fail(RKA_EINVAL, "steps_per_exchange must be in [0, 64]");
  if (split < 0 || split > 2) return fail(RKA_EINVAL, "rkab_split must be 0, 1 or 2");
  if (rblk < 0 || rblk > 2) return fail(RKA_EINVAL, "rka_block must be 0, 1 or 2");
  if (sampling == rka::kSampleBlocks && q > m)
    return fail(RKA_EINVAL, "the Distributed Approach needs q <= m (one row block per worker)");
  const int ncu = num_cus();
  if (ncu <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;

  rka::SolveShape sh;
  sh.A = A;
  sh.dtype = dtype;
  sh.m = m;
  sh.n = n;
  sh.lda = lda;
  sh.vec_ok = vector_path_ok(A, dtype, n, lda);
  sh.b = b;
  sh.x = x;
  sh.x_ref = (tol > 0.0) ? x_ref : nullptr;
  sh.alpha = alpha;
  sh.q = q;
  sh.bs = block ? bs : 1;
  sh.num_cu = ncu;
  sh.grid = grid > ncu ? ncu : grid;
  sh.allreduce = allreduce;
  sh.acc = acc;

  rka::RkaColGeom cgeo{};
  rka::RkabGeom bgeo{};
  rka::RkaSstepGeom sgeo{};
  rka::RkaBlkGeom kgeo{};
  bool use_blk = false;
  const int64_t in_kernel_check = (tol > 0.0 && sh.x_ref) ? check_every : 0;
  // several iterations per exchange: asked for (sstep >= 2), or chosen for
  // small q when blocks can be longer than one iteration between tests
  bool use_sstep = false;
  if (block && acc == 0 && split != 1 && (split == 2 || q * 4 <= ncu)) {
    // RKAB with every workgroup holding a slice of every worker's rows: asked
    // for, or chosen when the workers alone would leave most CUs idle and
    // the outer iteration fits one exchange or q is small.  Where one outer
    // iteration's q bs rows fit a block of kernel 4 (and rka_block is not 1),
    // the workers' inner products come from its streaming pass and the
    // exchange carries only the q bs dot products with x^(k); else kernel 3
    // carries the inner products in the exchange.
    if (rblk != 1) use_blk = rka::rka_blk_plan_rkab(sh, &kgeo);
    rka::RkaSstepGeom cand{};
    if (!use_blk && rblk != 2 && rka::rka_sstep_plan(sh, 1, &cand) &&
        (split == 2 || cand.c == bs || q <= kAutoSubBlockMaxQ)) {
      sgeo = cand;
      use_sstep = true;
    }
  } else if (!block && acc == 0 && allreduce == 0) {
    // blocks of iterations: coefficients from a streaming pass (rka_block 2),
    // or the inner products in the exchange (1)
    const bool want_blk = rblk == 2 || (rblk == 0 && kAutoBlk);
    bool multi = sstep >= 2 || (rblk == 2 && sstep == 1);  // kernel 4 also runs p = 1
    if (sstep == 0 && q <= (want_blk ? kAutoBlkMaxQ : kAutoSstepMaxQ) && in_kernel_check != 1) {
      // not where one workgroup holds the whole problem (no exchange at all)
      rka::RkaColGeom one{};
      multi = rka::rka_col_plan(sh, &one) && one.G > 1;
    }
    if (multi) {
      if (want_blk) use_blk = rka::rka_blk_plan(sh, sstep >= 1 ? sstep : 0, &kgeo);
      // kernel 3 where kernel 4 does not fit (left to the library: only
      // where kernel 3 beats the column kernel, q <= kAutoSstepMaxQ)
      if (!use_blk && rblk != 2 && (sstep >= 2 || q <= kAutoSstepMaxQ))
        use_sstep = rka::rka_sstep_plan(sh, sstep >= 2 ? sstep : 0, &sgeo);
    }
  }
  bool use_col = !block && !use_sstep && !use_blk && rka::rka_col_plan(sh, &cgeo);
  if (!use_col && !use_sstep && !use_blk) {
    // RKA whose q rows do not fit the column kernel's tile runs as RKAB with
    // one projection per worker, which is the same iteration (Sec. 3.4.2).
    if (!rka::rkab_plan(sh, &bgeo))
      return fail(RKA_EINVAL, "n = %lld is too large for the worker kernel's register and LDS tiles",
                  (long long)n);
  }

  Scratch sc = arena ? Scratch(s, arena, arena_bytes) : Scratch(s);
  rka::DevStatus* st;
  double *w, *c, *part;
  void* vbuf = nullptr;
  uint64_t *slots = nullptr, *sslots = nullptr;  // tagged exchange slots (column kernel)
  int64_t* last_pos;
  rka::RowRec* rec;
  unsigned* bar;
  const int64_t per_iter = (int64_t)q * sh.bs;
  int64_t kc_max = kRecBudget / per_iter;
  if (kc_max < 1) kc_max = 1;
  if (kc_max > max_iter) kc_max = max_iter > 0 ? max_iter : 1;
  const int G = use_blk ? kgeo.G : (use_sstep ? sgeo.G : (use_col ? cgeo.G : bgeo.G));
  size_t part_len = (size_t)G;
  if (!sh.x_ref && tol > 0.0) {
    const size_t rb = (size_t)rka::resid_blocks(m);
    if (rb > part_len) part_len = rb;
  }
  // a plan brings the norms and the running sum; the Distributed Approach
  // still restarts the running sum at every worker's block
  const bool own_norms = plan == nullptr;
  const bool own_prefix = plan == nullptr || sampling == rka::kSampleBlocks;
  const size_t n_last = sampling == rka::kSampleBlocks ? (size_t)q : 1;
  size_t nslots = 0, nsslots = 0, vb = 0;
  // coefficient blocks of a chunk of kc iterations (blk kernel): a segment
  // between stopping tests adds at most one partial block
  auto coef_blocks = [&](int64_t kc) -> int64_t {
    int64_t nb = kc / kgeo.p + 2;
    if (in_kernel_check > 0) nb += kc / in_kernel_check + 1;
    return nb * (kgeo.rkab_bs ? kgeo.rkab_nsub : 1);  // RKAB: sub-blocks per outer iteration
  };
  if (use_blk) {
    nslots = (size_t)kgeo.G * kgeo.nv;
    nsslots = (size_t)kgeo.nv * rka::kSumCopies;
    // chunks short enough that their coefficients take at most kCoefBudget
    // bytes (a chunk boundary costs two launches; a block's M is up to 57 KB)
    // (coef_blocks(kc) <= kCoefBudget / per_blk; p = 1 has no coefficients)
    if (kgeo.cstride > 0) {
      const int64_t per_blk = (int64_t)kgeo.cstride * 8;
      const double room =
          (double)(kCoefBudget / per_blk / (kgeo.rkab_bs ? kgeo.rkab_nsub : 1) - 3);
      const double per_it =
          1.0 / kgeo.p + (in_kernel_check > 0 ? 1.0 / (double)in_kernel_check : 0.0);
      int64_t kcap = (int64_t)(room / per_it);
      if (kcap < kgeo.p) kcap = kgeo.p;
      if (kc_max > kcap) kc_max = kcap;
    }
  } else if (use_sstep) {
    nslots = (size_t)sgeo.G * sgeo.nv;
    nsslots = (size_t)sgeo.nv * rka::kSumCopies;
  } else if (use_col) {
    // 16-byte slots: 2 words each
    nslots = (size_t)(cgeo.gather ? 2 : 1) * G * (q + 1);
    nsslots = ((size_t)q + 1) * rka::kSumCopies;
  } else {
    vb = (size_t)q * (size_t)n * (acc == 1 ? sizeof(float) : sizeof(double));
  }
  if (arena) {
    // the fixed buffers first, then as many iterations of row records per
    // chunk as the rest holds (at most the stream-ordered path's chunk)
    auto R = [](size_t b) { return Scratch::round(b > 0 ? b : 16); };
    size_t fixed = R(sizeof(rka::DevStatus)) + R(part_len * 8) +
                   R(rka::kGridBarCounters * sizeof(unsigned));
    if (own_norms) fixed += R((size_t)m * 8);
    if (own_prefix) fixed += R((size_t)m * 8) + R(n_last * 8);
    if (nslots) fixed += R(32 * nslots) + R(32 * nsslots);
    if (vb) fixed += R(vb);
    size_t per_rec_iter = sizeof(rka::RowRec) * (size_t)per_iter;
    if (use_blk) {
      // coefficients: (kc / p + 2 [+ kc / C + 1]) blocks of cstride doubles
      const size_t cb = (size_t)kgeo.cstride * 8;
      fixed += 256 + cb * (in_kernel_check > 0 ? 3 : 2);
      per_rec_iter += (cb + kgeo.p - 1) / kgeo.p;
      if (in_kernel_check > 0) per_rec_iter += (cb + in_kernel_check - 1) / in_kernel_check;
    }
    const int64_t fit =
        arena_bytes > fixed + 256 ? (int64_t)((arena_bytes - fixed - 256) / per_rec_iter) : 0;
    if (fit < 1)
      return fail(RKA_EINVAL,
                  "the problem needs %zu bytes of scratch for its fixed buffers plus %zu per "
                  "iteration of row records; the allocation-free scratch holds %zu",
                  fixed, per_rec_iter, arena_bytes);
    if (kc_max > fit) kc_max = fit;
  }
  HIP_TRY(sc.get(&st, 1));
  if (own_norms)
    HIP_TRY(sc.get(&w, (size_t)m));
  else
    w = plan->w;
  if (own_prefix) {
    HIP_TRY(sc.get(&c, (size_t)m));
    HIP_TRY(sc.get(&last_pos, n_last));
  } else {
    c = plan->c;
    last_pos = plan->last_pos;
  }
  HIP_TRY(sc.get(&rec, (size_t)(kc_max * per_iter)));
  HIP_TRY(sc.get(&part, part_len));
  HIP_TRY(sc.get(&bar, rka::kGridBarCounters));
  if (nslots) {
    HIP_TRY(sc.get(&slots, 2 * nslots));
    HIP_TRY(sc.get(&sslots, 2 * nsslots));
  }
  if (vb) HIP_TRY(sc.get((char**)&vbuf, vb));
  double* coef = nullptr;
  if (use_blk) HIP_TRY(sc.get(&coef, (size_t)coef_blocks(kc_max) * kgeo.cstride));
  sh.wn = w;

  PhaseTimer tm(s, timing && stats);
  if (nslots) {  // tag 0 never matches: slots start empty for the whole solve
    HIP_TRY(rka::launch_zero(slots, 16 * nslots, s));
    HIP_TRY(rka::launch_zero(sslots, 16 * nsslots, s));
  }
  HIP_TRY(rka::launch_status_init(st, tol, s));
  HIP_TRY(rka::launch_check_finite(b, m, st, s));
  if (own_norms) {
    tm.begin(kNorms);
    HIP_TRY(rka::launch_row_norms(A, dtype, m, n, lda, sh.vec_ok, w, s));
    tm.end();
  }
  if (own_prefix) {
    tm.begin(kPrefix);
    if (sampling == rka::kSampleBlocks)
      HIP_TRY(rka::launch_prefix_blocks(w, m, q, c, last_pos, st, s));
    else
      HIP_TRY(rka::launch_prefix(w, m, c, last_pos, st, s));
    tm.end();
  }
  if (x0) {
    if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    HIP_TRY(rka::launch_zero(x, (size_t)n * sizeof(double), s));
  }
  const bool resid_mode = tol > 0.0 && !sh.x_ref;
  if (tol > 0.0) {
    HIP_TRY(rka::launch_ref_norm(sh.x_ref ? sh.x_ref : b, sh.x_ref ? n : m, tol, st, s));
    tm.begin(kMeasure);
    HIP_TRY(rka::launch_measure(sh, 0, part, st, s));
    tm.end();
  }
  int64_t launches = 0;
  // Kernel 4 forms a chunk's coefficients before its iterations, so where a
  // stopping test may end the solve early its chunks start short and double
  // (at most one chunk's coefficient pass beyond the stop, twice the work
  // up to it); the passes of the chunks after a stop return at once.
  int64_t kc_grow = kc_max;
  if (use_blk && tol > 0.0) {
    kc_grow = std::max<int64_t>(kFirstBlkChunk, 4 * check_every);
    if (kc_grow > kc_max) kc_grow = kc_max;
  }
  for (int64_t k = 0; k < max_iter;) {
    int64_t kc = max_iter - k < kc_grow ? max_iter - k : kc_grow;
    if (kc_grow < kc_max) kc_grow = std::min<int64_t>(2 * kc_grow, kc_max);
    if (resid_mode) {
      const int64_t to_check = check_every - (k % check_every);
      if (to_check < kc) kc = to_check;
    }
    tm.begin(kSample);
    HIP_TRY(rka::launch_sample(c, m, last_pos, seed, k + iter_offset, kc, q, sh.bs, dom, sampling,
                               alpha, walpha, wrow, nullptr, rec, b, w, st, s));
    tm.end();
    if (use_blk) {
      tm.begin(kCoef);
      HIP_TRY(rka::launch_blk_coef(sh, kgeo, rec, k, kc, in_kernel_check, coef, st, s));
      tm.end();
    }
    tm.begin(kIterate);
    if (use_blk)
      HIP_TRY(rka::launch_blk_iter(sh, kgeo, rec, k, kc, in_kernel_check, coef, slots, sslots, st,
                                   s));
    else if (use_sstep)
      HIP_TRY(rka::launch_sstep_chunk(sh, sgeo, rec, k, kc, in_kernel_check, slots, sslots, st, s));
    else if (use_col)
      HIP_TRY(rka::launch_rka_chunk(sh, cgeo, rec, k, kc, in_kernel_check, slots, sslots, st, s));
    else
      HIP_TRY(rka::launch_rkab_chunk(sh, bgeo, rec, k, kc, in_kernel_check, vbuf, part, bar, st, s));
    tm.end();
    ++launches;
    k += kc;
    if (resid_mode && k % check_every == 0 && k < max_iter) {
      tm.begin(kMeasure);
      HIP_TRY(rka::launch_measure(sh, k, part, st, s));
      tm.end();
    }
  }
  if (tol > 0.0 && max_iter > 0) {
    tm.begin(kMeasure);
    HIP_TRY(rka::launch_measure(sh, max_iter, part, st, s));
    tm.end();
  }

  rka::DevStatus hst;
  HIP_TRY(hipMemcpyAsync(&hst, st, sizeof hst, hipMemcpyDeviceToHost, s));
  sc.release();
  HIP_TRY(hipStreamSynchronize(s));

  if (stats) {
    double ph[kPhases];
    tm.collect(ph);
    stats->norms_ms = ph[kNorms];
    stats->prefix_ms = ph[kPrefix];
    stats->sample_ms = ph[kSample];
    stats->iterate_ms = ph[kIterate];
    stats->measure_ms = ph[kMeasure];
    stats->coef_ms = ph[kCoef];
    stats->iterate_launches = launches;
    if (use_blk) {
      stats->kernel = 4;
      stats->grid = kgeo.G;
      stats->threads = kgeo.nt;
      stats->bucket = kgeo.rpt;
      stats->variant = kgeo.rkab_bs ? kgeo.rkab_c : kgeo.p;
    } else if (use_sstep) {
      stats->kernel = 3;
      stats->grid = sgeo.G;
      stats->threads = sgeo.nt;
      stats->bucket = sgeo.rpt;
      stats->variant = block ? sgeo.c : sgeo.p;
    } else {
      stats->kernel = use_col ? 1 : 2;
      stats->grid = use_col ? cgeo.G : bgeo.G;
      stats->threads = use_col ? cgeo.nt : bgeo.nt;
      stats->bucket = use_col ? cgeo.rpt : bgeo.vpt;
      stats->variant = use_col ? cgeo.gather : (bgeo.vlds ? 1 : 0);
    }
    stats->accumulate = acc;
  }
  int status = hst.status;
  if (status == RKA_EZERONORM) fail(status, "||A||_F^2 is zero or not finite");
  if (status == RKA_EINVAL) fail(status, "b has a non-finite entry");
  if (status == RKA_EDIVERGED) fail(status, "the stopping measure became non-finite");
  if (status == RKA_EDEVICE) fail(status, "a grid-wide wait inside a kernel gave up");
  if (info) {
    info->iterations = hst.iterations;
    info->projections = hst.iterations * per_iter;
    info->rel_err = isnan(hst.rel2) ? NAN : sqrt(hst.rel2);
    info->status = status;
  }
  return status;
}

}  // namespace

namespace rka {
hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args, unsigned lds,
                             hipStream_t s) {
  static const bool cooperative = [] {
    const char* v = getenv("RKA_COOPERATIVE");
    return !(v && v[0] == '0');
  }();
  if (cooperative) return hipLaunchCooperativeKernel(fn, grid, block, args, lds, s);
  return hipLaunchKernel(fn, grid, block, args, lds, s);
}
}  // namespace rka

namespace rka {
// error reporting and device query for the other translation units' entry points
int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
int api_num_cus() {
  g_last_error.clear();
  return num_cus();
}
}  // namespace rka

// Scratch of the allocation-free entry point: a fixed array that every
// device loading the library holds until the process ends.  Host code never
// uses the array's name as an address (on the host it is a stand-in symbol):
// each device's address comes from hipGetSymbolAddress, taken once per device
// with that device current.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch`, or an rka_status on failure.
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return fail(RKA_EDEVICE, "no HIP device available");
  if (dev >= kMaxDevices) return fail(RKA_EDEVICE, "device %d beyond the %d supported", dev,
                                      kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(RKA_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RKA_OK;
}
}  // namespace

extern "C" {

int rka_solve(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
              const double* x0, double* x, int32_t q, double alpha, int64_t max_iter, double tol,
              uint64_t seed, const double* x_ref, int64_t iter_offset, int64_t check_every,
              void* stream, rka_info* info) {
  return solve_impl(false, A, dtype, m, n, lda, b, x0, x, q, 1, alpha, max_iter, tol, seed, x_ref,
                    iter_offset, check_every, 0, 0, false, 0, 0, 0, nullptr, nullptr, 0, 0, stream,
                    info, nullptr);
}

// rka_solve_ex and its variants: unpack the options and solve, with the
// norms and running sum of `plan` when given, and scratch carved from
// `arena` when given.
static int solve_ex_impl(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         const double* b, const double* x0, double* x, int32_t method, int32_t q,
                         int32_t block_size, double alpha, int64_t max_iter, double tol,
                         uint64_t seed, const double* x_ref, int64_t iter_offset,
                         const rka_opts* opts, void* stream, rka_info* info, rka_stats* stats,
                         const rka_plan* plan, void* arena, size_t arena_bytes) {
  if (method != 0 && method != 1) {
    g_last_error.clear();
    if (info) info->status = RKA_EINVAL;
    return fail(RKA_EINVAL, "method must be 0 (RKA) or 1 (RKAB)");
  }
  const int64_t ce = opts ? opts->check_every : 1;
  const int grid = opts ? opts->grid : 0;
  const int allreduce = opts ? opts->allreduce : 0;
  const bool timing = opts ? opts->collect_timing != 0 : false;
  const int acc = opts ? opts->accumulate : 0;
  const int dom = opts ? opts->stream_id : 0;
  const int sampling = opts ? opts->sampling : 0;
  const double* walpha = opts ? opts->worker_alpha : nullptr;
  const double* wrow = opts ? opts->row_weight : nullptr;
  const int sstep = opts ? opts->steps_per_exchange : 0;
  const int split = opts ? opts->rkab_split : 0;
  const int rblk = opts ? opts->rka_block : 0;
  return solve_impl(method == 1, A, dtype, m, n, lda, b, x0, x, q, method == 1 ? block_size : 1,
                    alpha, max_iter, tol, seed, x_ref, iter_offset, ce, grid, allreduce, timing,
                    acc, dom, sampling, walpha, wrow, sstep, split, stream, info, stats, plan,
                    arena, arena_bytes, rblk);
}

int rka_solve_ex(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
                 const double* x0, double* x, int32_t method, int32_t q, int32_t block_size,
                 double alpha, int64_t max_iter, double tol, uint64_t seed, const double* x_ref,
                 int64_t iter_offset, const rka_opts* opts, void* stream, rka_info* info,
                 rka_stats* stats) {
  return solve_ex_impl(A, dtype, m, n, lda, b, x0, x, method, q, block_size, alpha, max_iter, tol,
                       seed, x_ref, iter_offset, opts, stream, info, stats, nullptr, nullptr, 0);
}

int rka_solve_ex_noalloc(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         const double* b, const double* x0, double* x, int32_t method, int32_t q,
                         int32_t block_size, double alpha, int64_t max_iter, double tol,
                         uint64_t seed, const double* x_ref, int64_t iter_offset,
                         const rka_opts* opts, void* stream, rka_info* info, rka_stats* stats) {
  g_last_error.clear();
  if (info) info->status = RKA_EINVAL;
  void* arena = nullptr;
  const int v = noalloc_scratch(&arena);
  if (v != RKA_OK) {
    if (info) info->status = v;
    return v;
  }
  rka_opts o{};
  if (opts) o = *opts;
  o.collect_timing = 0;  // timing would create HIP events
  return solve_ex_impl(A, dtype, m, n, lda, b, x0, x, method, q, block_size, alpha, max_iter, tol,
                       seed, x_ref, iter_offset, &o, stream, info, stats, nullptr, arena,
                       kNoAllocScratchBytes);
}

// A plan is usable on the device it was made on only.
static int check_plan(const rka_plan* plan) {
  if (!plan) return fail(RKA_EINVAL, "plan must be non-null");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RKA_EDEVICE, "no HIP device available");
  if (dev != plan->device)
    return fail(RKA_EINVAL, "the plan was made on device %d, the current device is %d",
                plan->device, dev);
  return RKA_OK;
}

int rka_plan_create(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* stream,
                    rka_plan** out) {
  g_last_error.clear();
  if (!out) return fail(RKA_EINVAL, "out must be non-null");
  *out = nullptr;
  if (!A) return fail(RKA_EINVAL, "A must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1 || lda < n) return fail(RKA_EINVAL, "need m, n >= 1 and lda >= n");
  if (m > INT32_MAX) return fail(RKA_EINVAL, "m must be < 2^31");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  rka_plan* p = new (std::nothrow) rka_plan{};
  if (!p) return fail(RKA_ENOMEM, "host allocation of the plan failed");
  p->A = A;
  p->dtype = dtype;
  p->m = m;
  p->n = n;
  p->lda = lda;
  p->vec_ok = vector_path_ok(A, dtype, n, lda);
  (void)hipGetDevice(&p->device);
  const size_t wbytes = Scratch::round((size_t)m * 8);
  hipError_t e = hipMalloc(&p->mem, 2 * wbytes + 256);
  if (e != hipSuccess) {
    delete p;
    return fail(e == hipErrorOutOfMemory ? RKA_ENOMEM : RKA_EDEVICE, "hipMalloc: %s",
                hipGetErrorString(e));
  }
  p->w = (double*)p->mem;
  p->c = (double*)((char*)p->mem + wbytes);
  p->last_pos = (int64_t*)((char*)p->mem + 2 * wbytes);
  e = rka::launch_row_norms(A, dtype, m, n, lda, p->vec_ok, p->w, s);
  if (e == hipSuccess) e = rka::launch_prefix(p->w, m, p->c, p->last_pos, nullptr, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&p->fro2, p->c + (m - 1), sizeof(double),
                                          hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(p->mem);
    delete p;
    return fail(RKA_EDEVICE, "plan set-up: %s", hipGetErrorString(e));
  }
  if (!(p->fro2 > 0.0) || !isfinite(p->fro2)) {
    (void)hipFree(p->mem);
    delete p;
    return fail(RKA_EZERONORM, "||A||_F^2 is zero or not finite");
  }
  *out = p;
  return RKA_OK;
}

int rka_plan_destroy(rka_plan* plan) {
  g_last_error.clear();
  if (!plan) return RKA_OK;
  hipError_t e = plan->mem ? hipFree(plan->mem) : hipSuccess;
  delete plan;
  if (e != hipSuccess) return fail(RKA_EDEVICE, "hipFree: %s", hipGetErrorString(e));
  return RKA_OK;
}

int rka_plan_query(const rka_plan* plan, int64_t* m, int64_t* n, double* fro2,
                   int64_t* last_pos) {
  g_last_error.clear();
  if (!plan) return fail(RKA_EINVAL, "plan must be non-null");
  if (m) *m = plan->m;
  if (n) *n = plan->n;
  if (fro2) *fro2 = plan->fro2;
  if (last_pos) {
    if (hipMemcpy(last_pos, plan->last_pos, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(RKA_EDEVICE, "reading the plan's last positive row failed");
  }
  return RKA_OK;
}

int rka_plan_row_norms(const rka_plan* plan, double* w, void* stream) {
  g_last_error.clear();
  int v = check_plan(plan);
  if (v != RKA_OK) return v;
  if (!w) return fail(RKA_EINVAL, "w must be non-null");
  HIP_TRY(hipMemcpyAsync(w, plan->w, (size_t)plan->m * sizeof(double), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return RKA_OK;
}

int rka_plan_sample_indices(const rka_plan* plan, uint64_t seed, int64_t iter_offset, int64_t K,
                            int32_t q, int32_t bs, int32_t dom, int32_t* idx, void* stream) {
  g_last_error.clear();
  int v = check_plan(plan);
  if (v != RKA_OK) return v;
  if (!idx) return fail(RKA_EINVAL, "idx must be non-null");
  if (K < 0 || q < 1 || bs < 1 || bs >= (1 << 24) || iter_offset < 0 || dom < 0 || dom > 255)
    return fail(RKA_EINVAL, "need K >= 0, q >= 1, 1 <= bs < 2^24, iter_offset >= 0, 0 <= dom < 256");
  HIP_TRY(rka::launch_sample(plan->c, plan->m, plan->last_pos, seed, iter_offset, K, q, bs, dom,
                             rka::kSampleFull, 1.0, nullptr, nullptr, idx, nullptr, nullptr,
                             nullptr, nullptr, (hipStream_t)stream));
  return RKA_OK;
}

int rka_plan_solve(const rka_plan* plan, const double* b, const double* x0, double* x,
                   int32_t method, int32_t q, int32_t block_size, double alpha, int64_t max_iter,
                   double tol, uint64_t seed, const double* x_ref, int64_t iter_offset,
                   const rka_opts* opts, void* stream, rka_info* info, rka_stats* stats) {
  g_last_error.clear();
  if (info) info->status = RKA_EINVAL;
  int v = check_plan(plan);
  if (v != RKA_OK) return v;
  return solve_ex_impl(plan->A, plan->dtype, plan->m, plan->n, plan->lda, b, x0, x, method, q,
                       block_size, alpha, max_iter, tol, seed, x_ref, iter_offset, opts, stream,
                       info, stats, plan, nullptr, 0);
}

int rka_alpha_star(double s_min, double s_max, int32_t q, double* alpha) {
  g_last_error.clear();
  if (!alpha) return fail(RKA_EINVAL, "alpha must be non-null");
  *alpha = NAN;
  if (q < 1) return fail(RKA_EINVAL, "q must be >= 1");
  if (!(s_min >= 0.0) || !(s_max >= s_min) || !(s_max <= 1.0))
    return fail(RKA_EINVAL, "need 0 <= s_min <= s_max <= 1 (squared singular values over "
                            "||A||_F^2)");
  *alpha = rka::alpha_star_eq6(s_min, s_max, q);
  return RKA_OK;
}

int rkab_solve(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, const double* b,
               const double* x0, double* x, int32_t q, int32_t block_size, double alpha,
               int64_t max_iter, double tol, uint64_t seed, const double* x_ref,
               int64_t iter_offset, int64_t check_every, void* stream, rka_info* info) {
  return solve_impl(true, A, dtype, m, n, lda, b, x0, x, q, block_size, alpha, max_iter, tol, seed,
                    x_ref, iter_offset, check_every, 0, 0, false, 0, 0, 0, nullptr, nullptr, 0, 0,
                    stream, info, nullptr);
}

int rka_row_norms(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, double* w,
                  void* stream) {
  g_last_error.clear();
  if (!A || !w) return fail(RKA_EINVAL, "A and w must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1 || lda < n) return fail(RKA_EINVAL, "need m, n >= 1 and lda >= n");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  HIP_TRY(rka::launch_row_norms(A, dtype, m, n, lda, vector_path_ok(A, dtype, n, lda), w,
                                (hipStream_t)stream));
  return RKA_OK;
}

int rka_prefix(const double* w, int64_t m, double* c, int64_t* last_pos, void* stream) {
  g_last_error.clear();
  if (!w || !c) return fail(RKA_EINVAL, "w and c must be non-null");
  if (m < 1 || m > INT32_MAX) return fail(RKA_EINVAL, "m must be in [1, 2^31)");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(rka::launch_prefix(w, m, c, last_pos, nullptr, s));
  double W = 0.0;
  HIP_TRY(hipMemcpyAsync(&W, c + (m - 1), sizeof W, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(W > 0.0) || !isfinite(W)) return fail(RKA_EZERONORM, "||A||_F^2 is zero or not finite");
  return RKA_OK;
}

int rka_sample_indices(const double* w, const double* c, int64_t m, uint64_t seed,
                       int64_t iter_offset, int64_t K, int32_t q, int32_t bs, int32_t dom,
                       int32_t* idx, void* stream) {
  g_last_error.clear();
  if (!w || !c || !idx) return fail(RKA_EINVAL, "w, c and idx must be non-null");
  if (m < 1 || m > INT32_MAX) return fail(RKA_EINVAL, "m must be in [1, 2^31)");
  if (K < 0 || q < 1 || bs < 1 || bs >= (1 << 24) || iter_offset < 0 || dom < 0 || dom > 255)
    return fail(RKA_EINVAL, "need K >= 0, q >= 1, 1 <= bs < 2^24, iter_offset >= 0, 0 <= dom < 256");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  // The fallback row (largest l with w_l > 0) comes from a pass over w.
  int64_t* last_pos = nullptr;
  double* cscratch = nullptr;
  HIP_TRY(hipMallocAsync((void**)&last_pos, sizeof(int64_t), s));
  hipError_t e = hipMallocAsync((void**)&cscratch, (size_t)m * sizeof(double), s);
  if (e == hipSuccess) e = rka::launch_prefix(w, m, cscratch, last_pos, nullptr, s);
  if (e == hipSuccess)
    e = rka::launch_sample(c, m, last_pos, seed, iter_offset, K, q, bs, dom, rka::kSampleFull, 1.0,
                           nullptr, nullptr, idx, nullptr, nullptr, nullptr, nullptr, s);
  if (cscratch) (void)hipFreeAsync(cscratch, s);
  (void)hipFreeAsync(last_pos, s);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? RKA_ENOMEM : RKA_EDEVICE, "sampling: %s",
                hipGetErrorString(e));
  return RKA_OK;
}

int rka_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld, const double* v,
             const double* c, double gamma, double* out, void* stream) {
  g_last_error.clear();
  if (!M || !v || !out) return fail(RKA_EINVAL, "M, v and out must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (rows < 1 || cols < 1 || ld < cols) return fail(RKA_EINVAL, "need rows, cols >= 1, ld >= cols");
  if (!isfinite(gamma)) return fail(RKA_EINVAL, "gamma must be finite");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  HIP_TRY(rka::launch_gemv(M, dtype, rows, cols, ld, vector_path_ok(M, dtype, cols, ld), v, c, gamma,
                           out, (hipStream_t)stream));
  return RKA_OK;
}

int rka_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At,
                  int64_t ldat, void* stream) {
  g_last_error.clear();
  if (!A || !At) return fail(RKA_EINVAL, "A and At must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1 || lda < n || ldat < m)
    return fail(RKA_EINVAL, "need m, n >= 1, lda >= n, ldat >= m");
  if ((m + 63) / 64 > 65535) return fail(RKA_EINVAL, "m must be < 65535 * 64");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  HIP_TRY(rka::launch_transpose(A, dtype, m, n, lda, At, ldat, (hipStream_t)stream));
  return RKA_OK;
}

int rka_lsq_grad_A(int64_t m, int64_t n, const double* r, const double* lam, const double* z,
                   const double* x, void* dA, int out_dtype, int64_t ldd, void* stream) {
  g_last_error.clear();
  if (!r || !lam || !z || !x || !dA) return fail(RKA_EINVAL, "every array must be non-null");
  if (m < 1 || n < 1 || ldd < n) return fail(RKA_EINVAL, "need m, n >= 1 and ldd >= n");
  if (out_dtype != RKA_F64 && out_dtype != RKA_F32)
    return fail(RKA_EINVAL, "out_dtype must be RKA_F64 or RKA_F32");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  HIP_TRY(rka::launch_rank2(m, n, r, lam, z, x, dA, out_dtype, ldd, (hipStream_t)stream));
  return RKA_OK;
}

// stopping-test interval of the inner solves when a reference is given
constexpr int64_t kInnerCheck = 25;

// The norms, running sum and last positive row of a matrix in stream-ordered
// scratch (an internal plan for the length of one call).
static int scratch_plan(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, Scratch& sc,
                        hipStream_t s, rka_plan* p) {
  *p = rka_plan{};
  p->A = A;
  p->dtype = dtype;
  p->m = m;
  p->n = n;
  p->lda = lda;
  p->vec_ok = vector_path_ok(A, dtype, n, lda);
  (void)hipGetDevice(&p->device);
  HIP_TRY(sc.get(&p->w, (size_t)m));
  HIP_TRY(sc.get(&p->c, (size_t)m));
  HIP_TRY(sc.get(&p->last_pos, 1));
  HIP_TRY(rka::launch_row_norms(A, dtype, m, n, lda, p->vec_ok, p->w, s));
  HIP_TRY(rka::launch_prefix(p->w, m, p->c, p->last_pos, nullptr, s));
  HIP_TRY(hipMemcpyAsync(&p->fro2, p->c + (m - 1), sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(p->fro2 > 0.0) || !isfinite(p->fro2))
    return fail(RKA_EZERONORM, "||A||_F^2 is zero or not finite");
  return RKA_OK;
}

static int refine_impl(const void* A, const void* At, int dtype, int64_t m, int64_t n,
                       int64_t lda, int64_t ldat, const rka_plan* pA, const rka_plan* pAt,
                       const double* b, const double* x0, double* x, const rka_refine_opts* o,
                       uint64_t seed, const double* x_ref, double* sweep_measure, void* stream,
                       rka_refine_info* info) {
  if (info) {
    info->sweeps = 0;
    info->status = RKA_EINVAL;
    info->rel = NAN;
    info->projections = 0;
  }
  if (!o) return fail(RKA_EINVAL, "opts must be non-null");
  if (!A || !b || !x) return fail(RKA_EINVAL, "A, b and x must be non-null");
  if (bad_dtype(dtype)) return fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1 || lda < n) return fail(RKA_EINVAL, "need m, n >= 1 and lda >= n");
  if (m > INT32_MAX || n > INT32_MAX) return fail(RKA_EINVAL, "m and n must be < 2^31");
  if (o->method != 0 && o->method != 1) return fail(RKA_EINVAL, "method must be 0 or 1");
  if (o->q < 1 || o->inner_iters < 0 || o->max_sweeps < 1)
    return fail(RKA_EINVAL, "need q >= 1, inner_iters >= 0, max_sweeps >= 1");
  if (o->method == 1 && (o->block_size < 1 || o->block_size >= (1 << 24)))
    return fail(RKA_EINVAL, "block_size must be in [1, 2^24)");
  if (!(o->alpha > 0.0) || !isfinite(o->alpha)) return fail(RKA_EINVAL, "alpha must be finite and > 0");
  if (!(o->tol >= 0.0) || !isfinite(o->tol)) return fail(RKA_EINVAL, "tol must be finite and >= 0");
  if (o->accumulate < 0 || o->accumulate > 1 || (o->accumulate == 1 && dtype == RKA_F64))
    return fail(RKA_EINVAL, "accumulate must be 0, or 1 with RKA_F32 / RKA_BF16 storage");
  const bool range = o->range_iters > 0;
  if (o->range_iters < 0) return fail(RKA_EINVAL, "range_iters must be >= 0");
  if (range) {
    if (!At || ldat < m) return fail(RKA_EINVAL, "the range projection needs At (n x m, ldat >= m)");
    if (o->range_q < 1 || !(o->range_alpha > 0.0) || !isfinite(o->range_alpha))
      return fail(RKA_EINVAL, "need range_q >= 1 and a finite range_alpha > 0");
  }
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  const bool vec_a = vector_path_ok(A, dtype, n, lda);
  const bool vec_t = range && vector_path_ok(At, dtype, m, ldat);

  Scratch sc(s);
  double *r, *d, *part, *acc2, *y = nullptr, *g = nullptr, *dref = nullptr;
  HIP_TRY(sc.get(&r, (size_t)m));
  HIP_TRY(sc.get(&d, (size_t)n));
  const bool early = x_ref && o->tol > 0.0;
  if (early) HIP_TRY(sc.get(&dref, (size_t)n));
  HIP_TRY(sc.get(&part, (size_t)rka::sumsq_part_len()));
  HIP_TRY(sc.get(&acc2, 2));
  if (range) {
    HIP_TRY(sc.get(&y, (size_t)m));
    HIP_TRY(sc.get(&g, (size_t)n));
  }
  // norms and running sums once per call, not once per sweep
  rka_plan own_a, own_t;
  if (!pA) {
    const int v = scratch_plan(A, dtype, m, n, lda, sc, s, &own_a);
    if (v != RKA_OK) return v;
    pA = &own_a;
  }
  if (range && !pAt) {
    const int v = scratch_plan(At, dtype, n, m, ldat, sc, s, &own_t);
    if (v != RKA_OK) return v;
    pAt = &own_t;
  }
  if (x0) {
    if (x0 != x) HIP_TRY(hipMemcpyAsync(x, x0, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    HIP_TRY(rka::launch_zero(x, (size_t)n * sizeof(double), s));
  }
  // denominator of the sweep measure
  HIP_TRY(rka::launch_sumsq(x_ref ? x_ref : b, nullptr, x_ref ? n : m, part, acc2 + 1, s));
  double ref2 = 0.0;
  HIP_TRY(hipMemcpyAsync(&ref2, acc2 + 1, sizeof ref2, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(ref2 > 0.0)) ref2 = 1.0;

  int status = o->tol > 0.0 ? RKA_NOT_CONVERGED : RKA_OK;
  int64_t projections = 0;
  double rel = NAN;
  int sweeps = 0;
  for (int sw = 0; sw < o->max_sweeps; ++sw) {
    // r = b - A x in FP64
    HIP_TRY(rka::launch_gemv(A, dtype, m, n, lda, vec_a, x, b, -1.0, r, s));
    const double* rhs = r;
    rka_info ii;
    if (range) {
      // y = the projection of r onto range(A): the minimum-norm solution of
      // A^T y = A^T r, by Kaczmarz on the columns of A from y = 0
      HIP_TRY(rka::launch_gemv(At, dtype, n, m, ldat, vec_t, r, nullptr, 1.0, g, s));
      const int st = solve_impl(false, At, dtype, n, m, ldat, g, nullptr, y, o->range_q, 1,
                                o->range_alpha, o->range_iters, 0.0, seed, nullptr,
                                (int64_t)sw * o->range_iters, 1, 0, 0, false, o->accumulate, 1, 0,
                                nullptr, nullptr, 0, 0, stream, &ii, nullptr, pAt);
      if (st < 0) return st;
      projections += ii.projections;
      rhs = y;
    }
    // d ~ argmin ||A d - rhs||, by the inner RKA / RKAB solve from d = 0.
    // With a reference the exact correction is x_ref - x, and
    // ||(x + d) - x_ref|| = ||d - (x_ref - x)||: the inner solve stops as
    // soon as the sweep would meet tol (tested every kInnerCheck iterations).
    double tol_d = 0.0;
    if (early) {
      HIP_TRY(rka::launch_sub(dref, x_ref, x, n, s));
      HIP_TRY(rka::launch_sumsq(dref, nullptr, n, part, acc2, s));
      double dr2 = 0.0;
      HIP_TRY(hipMemcpyAsync(&dr2, acc2, sizeof dr2, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (dr2 > 0.0 && isfinite(dr2)) tol_d = o->tol * sqrt(ref2 / dr2);
    }
    const int st = solve_impl(o->method == 1, A, dtype, m, n, lda, rhs, nullptr, d, o->q,
                              o->method == 1 ? o->block_size : 1, o->alpha, o->inner_iters, tol_d,
                              seed, tol_d > 0.0 ? dref : nullptr, (int64_t)sw * o->inner_iters,
                              kInnerCheck, 0, 0, false, o->accumulate, 0, 0, nullptr, nullptr, 0,
                              0, stream, &ii, nullptr, pA);
    if (st < 0) return st;
    projections += ii.projections;
    HIP_TRY(rka::launch_axpy(x, d, n, s));
    // sweep measure: ||x - x_ref|| / ||x_ref||, else ||b - A x|| / ||b||
    if (x_ref) {
      HIP_TRY(rka::launch_sumsq(x, x_ref, n, part, acc2, s));
    } else {
      HIP_TRY(rka::launch_gemv(A, dtype, m, n, lda, vec_a, x, b, -1.0, r, s));
      HIP_TRY(rka::launch_sumsq(r, nullptr, m, part, acc2, s));
    }
    double e2 = 0.0;
    HIP_TRY(hipMemcpyAsync(&e2, acc2, sizeof e2, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    rel = sqrt(e2 / ref2);
    if (sweep_measure) sweep_measure[sw] = rel;
    sweeps = sw + 1;
    if (!isfinite(rel)) {
      status = RKA_EDIVERGED;
      fail(status, "the sweep measure became non-finite");
      break;
    }
    if (o->tol > 0.0 && rel <= o->tol) {
      status = RKA_OK;
      break;
    }
  }
  sc.release();
  HIP_TRY(hipStreamSynchronize(s));
  if (info) {
    info->sweeps = sweeps;
    info->status = status;
    info->rel = rel;
    info->projections = projections;
  }
  return status;
}

int rka_refine_solve(const void* A, const void* At, int dtype, int64_t m, int64_t n, int64_t lda,
                     int64_t ldat, const double* b, const double* x0, double* x,
                     const rka_refine_opts* o, uint64_t seed, const double* x_ref,
                     double* sweep_measure, void* stream, rka_refine_info* info) {
  g_last_error.clear();
  return refine_impl(A, At, dtype, m, n, lda, ldat, nullptr, nullptr, b, x0, x, o, seed, x_ref,
                     sweep_measure, stream, info);
}

int rka_plan_refine_solve(const rka_plan* pA, const rka_plan* pAt, const double* b,
                          const double* x0, double* x, const rka_refine_opts* o, uint64_t seed,
                          const double* x_ref, double* sweep_measure, void* stream,
                          rka_refine_info* info) {
  g_last_error.clear();
  if (info) info->status = RKA_EINVAL;
  int v = check_plan(pA);
  if (v != RKA_OK) return v;
  if (pAt) {
    v = check_plan(pAt);
    if (v != RKA_OK) return v;
    if (pAt->m != pA->n || pAt->n != pA->m || pAt->dtype != pA->dtype)
      return fail(RKA_EINVAL, "pAt must be a plan of the n x m transpose of A, same dtype");
  }
  return refine_impl(pA->A, pAt ? pAt->A : nullptr, pA->dtype, pA->m, pA->n, pA->lda,
                     pAt ? pAt->lda : 0, pA, pAt, b, x0, x, o, seed, x_ref, sweep_measure, stream,
                     info);
}

int rka_sample_blocks(const double* w, int64_t m, uint64_t seed, int64_t iter_offset, int64_t K,
                      int32_t q, int32_t bs, int32_t dom, int32_t* idx, void* stream) {
  g_last_error.clear();
  if (!w || !idx) return fail(RKA_EINVAL, "w and idx must be non-null");
  if (m < 1 || m > INT32_MAX) return fail(RKA_EINVAL, "m must be in [1, 2^31)");
  if (K < 0 || q < 1 || q > m || bs < 1 || bs >= (1 << 24) || iter_offset < 0 || dom < 0 ||
      dom > 255)
    return fail(RKA_EINVAL,
                "need K >= 0, 1 <= q <= m, 1 <= bs < 2^24, iter_offset >= 0, 0 <= dom < 256");
  if (num_cus() <= 0) return fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  Scratch sc(s);
  double* c;
  int64_t* last;
  rka::DevStatus* st;
  HIP_TRY(sc.get(&c, (size_t)m));
  HIP_TRY(sc.get(&last, (size_t)q));
  HIP_TRY(sc.get(&st, 1));
  HIP_TRY(rka::launch_status_init(st, 0.0, s));
  HIP_TRY(rka::launch_prefix_blocks(w, m, q, c, last, st, s));
  HIP_TRY(rka::launch_sample(c, m, last, seed, iter_offset, K, q, bs, dom, rka::kSampleBlocks, 1.0,
                             nullptr, nullptr, idx, nullptr, nullptr, nullptr, st, s));
  rka::DevStatus hst;
  HIP_TRY(hipMemcpyAsync(&hst, st, sizeof hst, hipMemcpyDeviceToHost, s));
  sc.release();
  HIP_TRY(hipStreamSynchronize(s));
  if (hst.status == RKA_EZERONORM) return fail(RKA_EZERONORM, "a worker's row block has zero weight");
  return RKA_OK;
}

const char* rka_status_string(int status) {
  switch (status) {
    case RKA_OK: return "RKA_OK";
    case RKA_NOT_CONVERGED: return "RKA_NOT_CONVERGED";
    case RKA_EINVAL: return "RKA_EINVAL";
    case RKA_EZERONORM: return "RKA_EZERONORM";
    case RKA_EDIVERGED: return "RKA_EDIVERGED";
    case RKA_ENOMEM: return "RKA_ENOMEM";
    case RKA_EDEVICE: return "RKA_EDEVICE";
    default: return "RKA_UNKNOWN";
  }
}

const char* rka_last_error(void) { return g_last_error.c_str(); }

int rka_version(void) { return 100; }

}  // extern "C"
