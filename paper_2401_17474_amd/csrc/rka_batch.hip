// rka_batch.hip -- many independent systems (and right-hand sides) in one
// launch: the batching form.
//
// A *task* is one system with a group of R of its right-hand sides (R = 1
// for an ordinary system; a matrix shared by many right-hand sides becomes
// several tasks that share its row stream).  One workgroup runs one task, so
// tasks of uneven sizes balance through the hardware dispatcher (tasks are
// ordered largest first).  Inside a workgroup, sub-teams of `tpr` threads
// (threads per row) are the RKAB workers of Sec. 3.4.1: each keeps its
// iterate v for the R right-hand sides in LDS and applies block_size
// projections, a sampled row being read once from memory and applied to all
// R iterates; the q worker iterates are then summed in worker order and
// divided by q.  Arithmetic is binary32 on FP32 or BF16 storage.  A chunk of
// iterations is a batched row-stream launch followed by the batched
// iteration launch; the chunks of a solve can be captured in one HIP graph.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "rka.h"
#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

constexpr int kBT = 256;     // threads per batch workgroup
constexpr int kEptMax = 16;  // row elements per thread (tpr * 16 >= n)
constexpr int kRmax = 8;     // right-hand sides per task
// dependent projection steps (block size + 2 for the average) per chunk
constexpr double kChunkSteps = 4096.0;
// a task whose squared error has not halved for this many dependent
// projection steps (iterations x (block size + 2)) has reached the rounding
// floor of its binary32 iteration and stops (done = 4)
constexpr int64_t kStallSteps = 60000;

struct BatchSys {
  const double* c;         // running sum of the squared row norms
  const int64_t* last_pos; // largest row with a positive weight
  int64_t m;
  uint64_t seed;
  int64_t kc;              // iterations of this system per chunk
  int64_t max_iter;
  int32_t q, bs;
  int32_t* idx;            // row stream of the current chunk, kc x q x bs
  const int32_t* alive;    // nonzero while a task of the system still runs
};

struct BatchTask {
  const void* A;
  int64_t m, n, lda;
  const double* b;   // right-hand side r at b + r * ldb
  int64_t ldb;
  double* x;         // iterate r at x + r * ldx (start in, result out)
  int64_t ldx;
  const double* xr;  // stopping reference r at xr + r * ldxr (nullable)
  int64_t ldxr;
  const double* w;   // squared row norms
  const int32_t* idx;
  int32_t* done;     // per task
  int32_t* alive;    // per system: cleared by the sampler bookkeeping below
  int64_t* iters;    // per task
  double* rel;       // per task: last relative error (NaN if never measured)
  double* best;      // per task: smallest squared error seen at a halving
  int64_t* best_k;   // per task: iteration of that halving
  int64_t max_iter;  // iteration cap of the system
  int64_t kc;        // iterations per chunk (shared with its system's sampler)
  double ref2;       // > 0: denominator of the stopping test (else ||xr||^2)
  float alpha;
  int32_t R, q, bs, tpr;
  int32_t bf16;      // storage: 0 FP32, 1 BF16
};

__device__ __forceinline__ float load_elem(const void* A, int bf16, int64_t off) {
  if (bf16) return __uint_as_float((uint32_t)((const uint16_t*)A)[off] << 16);
  return ((const float*)A)[off];
}

// Row stream of chunk `chunk` for every system still running (one thread per
// draw): system s covers iterations [chunk kc_s, (chunk + 1) kc_s).
__global__ __launch_bounds__(256) void batch_sample_kernel(const BatchSys* __restrict__ sys,
                                                           int64_t chunk) {
  const BatchSys S = sys[blockIdx.y];
  if (S.alive && *S.alive == 0) return;
  const int64_t k0 = chunk * S.kc;
  if (k0 >= S.max_iter) return;
  const int64_t K = S.max_iter - k0 < S.kc ? S.max_iter - k0 : S.kc;
  const double W = S.c[S.m - 1];
  const int64_t last = *S.last_pos;
  const int64_t total = K * (int64_t)S.q * S.bs;
  for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < total;
       L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = L % S.bs;
    const int64_t wk = (L / S.bs) % S.q;
    const int64_t kl = L / ((int64_t)S.bs * S.q);
    const double u = draw_uniform(S.seed, (uint64_t)(k0 + kl), (uint32_t)wk, (uint32_t)j, 0u);
    S.idx[L] = (int32_t)pick_row(S.c, S.m, W, u, last);
  }
}

__global__ void batch_fill64_kernel(double* p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void batch_fill_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// One task per workgroup; chunk `chunk` covers its iterations
// [chunk kc, (chunk + 1) kc).  check_every > 0 with a reference: stop once
// ||x - xr|| <= tol ||xr|| (all R right-hand sides together), tested after
// every check_every-th iteration.
__global__ __launch_bounds__(kBT) void batch_iter_kernel(const BatchTask* __restrict__ tasks,
                                                         int64_t chunk, int64_t check_every,
                                                         double tol2) {
  const BatchTask T = tasks[blockIdx.x];
  const int64_t max_iter = T.max_iter;
  if (T.done[blockIdx.x]) return;
  const int64_t k0 = chunk * T.kc, K = T.kc;
  if (k0 >= max_iter) return;
  extern __shared__ float L[];
  __shared__ float red[kBT / kWave][kRmax];
  __shared__ double dred[kBT / kWave];
  const int n = (int)T.n, R = T.R, q = T.q, bs = T.bs, tpr = T.tpr;
  const int W = kBT / tpr;
  const int t = threadIdx.x, team = t / tpr, lane = t % tpr;
  const int nw_team = tpr > kWave ? tpr / kWave : 1;
  const int Rn = R * n;
  float* X = L;
  float* S = X + Rn;
  float* Vt = S + Rn + (size_t)team * Rn;

  for (int e = t; e < Rn; e += kBT) X[e] = (float)T.x[(e / n) * T.ldx + (e % n)];
  double ref2 = 0.0;
  const bool checking = T.xr && check_every > 0;
  if (checking) {
    double s = 0.0;
    for (int e = t; e < Rn; e += kBT) {
      const double v = T.xr[(e / n) * T.ldxr + (e % n)];
      s = fma(v, v, s);
    }
    ref2 = T.ref2 > 0.0 ? T.ref2 : block_sum(s, dred);
  }
  __syncthreads();

  const float alpha = T.alpha;
  auto load_row = [&](float (&a)[kEptMax], int64_t row) {
#pragma unroll
    for (int u = 0; u < kEptMax; ++u) {
      const int c = lane + u * tpr;
      const int cc = c < n ? c : n - 1;  // unconditional load, masked below
      a[u] = load_elem(T.A, T.bf16, row * T.lda + cc);
    }
  };

  int64_t kl = 0;
  bool stopped = false;
  for (; kl < K && k0 + kl < max_iter; ++kl) {
    for (int e = t; e < Rn; e += kBT) S[e] = 0.0f;
    for (int w0 = 0; w0 < q; w0 += W) {
      const int w = w0 + team < q ? w0 + team : q - 1;
      const int32_t* ix = T.idx + ((int64_t)kl * q + w) * bs;
      for (int e = lane; e < Rn; e += tpr) Vt[e] = X[e];
      // two rows in flight: the current one and the next
      float a[kEptMax], an[kEptMax];
      int64_t i0 = ix[0];
      int64_t i1 = ix[bs > 1 ? 1 : 0];
      load_row(a, i0);
      float bb[kRmax], wi = (float)T.w[i0];
#pragma unroll
      for (int r = 0; r < kRmax; ++r) bb[r] = (float)T.b[(r < R ? r : 0) * T.ldb + i0];
      for (int j = 0; j < bs; ++j) {
        const int64_t i2 = ix[j + 2 < bs ? j + 2 : bs - 1];
        load_row(an, i1);
        float bbn[kRmax];
        const float win = (float)T.w[i1];
#pragma unroll
        for (int r = 0; r < kRmax; ++r) bbn[r] = (float)T.b[(r < R ? r : 0) * T.ldb + i1];
        // dot products with the R iterates
        float d[kRmax];
#pragma unroll
        for (int r = 0; r < kRmax; ++r) {
          float s = 0.0f;
          if (r < R) {
#pragma unroll
            for (int u = 0; u < kEptMax; ++u) {
              const int c = lane + u * tpr;
              if (c < n) s = fmaf(a[u], Vt[r * n + c], s);
            }
          }
          d[r] = s;
        }
#pragma unroll
        for (int r = 0; r < kRmax; ++r) {
          const int top = tpr < kWave ? tpr : kWave;
          for (int off = top / 2; off > 0; off >>= 1) d[r] += __shfl_xor(d[r], off, kWave);
        }
        if (tpr > kWave) {  // several waves per team: combine in wave order
          if ((t & (kWave - 1)) == 0) {
#pragma unroll
            for (int r = 0; r < kRmax; ++r) red[t / kWave][r] = d[r];
          }
          __syncthreads();
#pragma unroll
          for (int r = 0; r < kRmax; ++r) {
            float s = 0.0f;
            for (int v = 0; v < nw_team; ++v) s += red[team * nw_team + v][r];
            d[r] = s;
          }
          __syncthreads();
        }
        // v += alpha (b_i - <a_i, v>) / ||a_i||^2 a_i   for every right-hand side
#pragma unroll
        for (int r = 0; r < kRmax; ++r) {
          if (r < R) {
            const float s = alpha * (bb[r] - d[r]) / wi;
#pragma unroll
            for (int u = 0; u < kEptMax; ++u) {
              const int c = lane + u * tpr;
              if (c < n) Vt[r * n + c] = fmaf(s, a[u], Vt[r * n + c]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kEptMax; ++u) a[u] = an[u];
#pragma unroll
        for (int r = 0; r < kRmax; ++r) bb[r] = bbn[r];
        wi = win;
        i0 = i1;
        i1 = i2;
      }
      __syncthreads();
      // sum of the worker iterates in worker order
      const int nact = q - w0 < W ? q - w0 : W;
      for (int e = t; e < Rn; e += kBT) {
        float s = S[e];
        for (int tt = 0; tt < nact; ++tt) s = s + S[Rn + (size_t)tt * Rn + e];
        S[e] = s;
      }
      __syncthreads();
    }
    const float qf = (float)q;
    for (int e = t; e < Rn; e += kBT) X[e] = S[e] / qf;
    __syncthreads();
    const int64_t k = k0 + kl + 1;  // iterations done
    if (checking && (k % check_every) == 0) {
      double s = 0.0;
      for (int e = t; e < Rn; e += kBT) {
        const double dd = (double)X[e] - T.xr[(e / n) * T.ldxr + (e % n)];
        s = fma(dd, dd, s);
      }
      const double e2 = block_sum(s, dred);
      if (t == 0) T.rel[blockIdx.x] = sqrt(e2 / ref2);
      const double best = T.best[blockIdx.x];
      const bool halved = e2 <= 0.5 * best;
      const bool stalled = !halved && (k - T.best_k[blockIdx.x]) * (bs + 2) >= kStallSteps;
      __syncthreads();  // every thread has read best before it changes
      if (halved && t == 0) {
        T.best[blockIdx.x] = e2;
        T.best_k[blockIdx.x] = k;
      }
      if (e2 <= tol2 * ref2 || !isfinite(e2) || stalled) {
        if (t == 0) {
          T.iters[blockIdx.x] = k;
          T.done[blockIdx.x] = !isfinite(e2) ? 2 : (e2 <= tol2 * ref2 ? 1 : 4);
        }
        stopped = true;
        break;
      }
    }
  }
  for (int e = t; e < Rn; e += kBT) T.x[(e / n) * T.ldx + (e % n)] = (double)X[e];
  if (!stopped && t == 0) {
    T.iters[blockIdx.x] = k0 + kl;
    if (k0 + kl >= max_iter) T.done[blockIdx.x] = 3;  // ran out of iterations
  }
}

// Per system: clear `alive` once all its tasks are done (so later chunks skip
// its sampling).  One thread per system.
__global__ void batch_alive_kernel(const int32_t* __restrict__ done, const int32_t* task_sys,
                                   int ntasks, int32_t* alive, int nsys) {
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsys; s += gridDim.x * blockDim.x) {
    int any = 0;
    for (int t = 0; t < ntasks; ++t)
      if (task_sys[t] == s && done[t] == 0) any = 1;
    alive[s] = any;
  }
}

size_t batch_lds_bytes(int64_t n, int R, int tpr) {
  return (size_t)(2 + kBT / tpr) * (size_t)R * (size_t)n * sizeof(float);
}

}  // namespace rka

// ===========================================================================
// Host side: planning, the autotuner and the C ABI.
// ===========================================================================
namespace {

using rka::BatchSys;
using rka::BatchTask;

constexpr size_t kBatchLdsMax = 64 * 1024;

bool pow2_tpr(int t) { return t == 16 || t == 32 || t == 64 || t == 128 || t == 256; }

int min_tpr(int64_t n) {
  int t = 16;
  while ((int64_t)t * rka::kEptMax < n) t *= 2;
  return t;
}

// Largest right-hand-side group (<= kRmax) whose task fits the LDS budget.
int pick_R(int64_t n, int tpr, int nrhs) {
  int R = nrhs < rka::kRmax ? nrhs : rka::kRmax;
  while (R > 1 && rka::batch_lds_bytes(n, R, tpr) > kBatchLdsMax) --R;
  return R;
}

// Heuristic parameters (used where the caller gives 0 and no tuning table
// applies): threads per row just enough for the row (16 elements a thread),
// q = the workers that run at once, block size ~ n/4 in [4, 64] (the paper
// recommends blocks of the order of n, Sec. 3.4.3; shorter blocks average
// more often).
void heuristic(int64_t n, int* q, int* bs, int* tpr) {
  if (*tpr == 0) *tpr = min_tpr(n);
  if (*q == 0) *q = rka::kBT / *tpr;
  if (*bs == 0) {
    int64_t b = n / 4;
    if (b < 4) b = 4;
    if (b > 64) b = 64;
    *bs = (int)b;
  }
}

}  // namespace

namespace rka {
int api_fail(int code, const char* fmt, ...);
int api_num_cus();
}

#define BHIP(call)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return rka::api_fail(e_ == hipErrorOutOfMemory ? RKA_ENOMEM : RKA_EDEVICE, "%s: %s",   \
                           #call, hipGetErrorString(e_));                                    \
  } while (0)

namespace {

struct DevBuf {
  std::vector<void*> p;
  hipStream_t s;
  explicit DevBuf(hipStream_t st) : s(st) {}
  template <typename U>
  hipError_t get(U** out, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, count * sizeof(U) > 0 ? count * sizeof(U) : 16, s);
    if (e != hipSuccess) return e;
    p.push_back(q);
    *out = (U*)q;
    return hipSuccess;
  }
  ~DevBuf() {
    for (size_t i = p.size(); i-- > 0;) (void)hipFreeAsync(p[i], s);
  }
};

int validate_sys(const rka_batch_system& S, int i, int dtype) {
  if (!S.A || !S.b || !S.x) return rka::api_fail(RKA_EINVAL, "system %d: A, b and x must be non-null", i);
  if (S.m < 1 || S.n < 1 || S.lda < S.n || S.m > INT32_MAX)
    return rka::api_fail(RKA_EINVAL, "system %d: need 1 <= m < 2^31, n >= 1, lda >= n", i);
  if (S.n > (int64_t)256 * rka::kEptMax)
    return rka::api_fail(RKA_EINVAL, "system %d: n must be <= %d", i, 256 * rka::kEptMax);
  if (S.nrhs < 1 || S.ldb < S.m || S.ldx < S.n || (S.x_ref && S.ldxr < S.n))
    return rka::api_fail(RKA_EINVAL, "system %d: need nrhs >= 1, ldb >= m, ldx >= n, ldxr >= n", i);
  if (S.q < 0 || S.block_size < 0 || S.block_size >= (1 << 24) || S.max_iter < 0)
    return rka::api_fail(RKA_EINVAL, "system %d: bad q, block_size or max_iter", i);
  if (S.tpr != 0 && (!pow2_tpr(S.tpr) || (int64_t)S.tpr * rka::kEptMax < S.n))
    return rka::api_fail(RKA_EINVAL, "system %d: tpr must be 16..256 (power of 2) with tpr*16 >= n", i);
  if (S.rhs_per_task < 0 || S.rhs_per_task > rka::kRmax)
    return rka::api_fail(RKA_EINVAL, "system %d: rhs_per_task must be in [0, %d]", i, rka::kRmax);
  if (!(S.alpha >= 0.0) || !isfinite(S.alpha))
    return rka::api_fail(RKA_EINVAL, "system %d: alpha must be finite and >= 0 (0: chosen)", i);
  (void)dtype;
  return RKA_OK;
}

}  // namespace

// The batch solve; ref2_rhs (nullable): per system and right-hand side (in
// system order), the squared norm that stands for ||x_ref||^2 in the
// stopping test (the refinement measures corrections against x_ref - x).
// dump (nullable): run the set-up and the row streams only, copying every
// chunk's draws of system i to dump + sum_{j<i} max_iter_j q_j bs_j (the
// parity hook rka_batch_sample_indices); no iteration runs.
static int batch_core(const rka_batch_system* systems, int32_t count, int dtype, uint64_t seed,
                      double tol, int64_t check_every, int64_t chunk_iters, int32_t use_graph,
                      void* stream, rka_batch_result* results, rka_batch_stats* stats,
                      const double* ref2_rhs, int32_t* dump = nullptr) {
  if (stats) memset(stats, 0, sizeof *stats);
  if (dump) use_graph = 0;
  if (!systems || count < 1 || count > 65535)
    return rka::api_fail(RKA_EINVAL, "need 1 to 65535 systems");
  if (dtype != RKA_F32 && dtype != RKA_BF16)
    return rka::api_fail(RKA_EINVAL, "batched solves take RKA_F32 or RKA_BF16 storage");
  if (!(tol >= 0.0) || !isfinite(tol)) return rka::api_fail(RKA_EINVAL, "tol must be finite and >= 0");
  if (chunk_iters < 0) return rka::api_fail(RKA_EINVAL, "chunk_iters must be >= 0");
  for (int i = 0; i < count; ++i) {
    int v = validate_sys(systems[i], i, dtype);
    if (v != RKA_OK) return v;
  }
  if (rka::api_num_cus() <= 0) return rka::api_fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  if (check_every < 1) check_every = 1;

  // parameters and tasks
  std::vector<int> q(count), bs(count), tpr(count), R(count);
  int64_t max_iter = 0;
  for (int i = 0; i < count; ++i) {
    const rka_batch_system& S = systems[i];
    q[i] = S.q;
    bs[i] = S.block_size;
    tpr[i] = S.tpr;
    heuristic(S.n, &q[i], &bs[i], &tpr[i]);
    if (q[i] > 65535) return rka::api_fail(RKA_EINVAL, "system %d: q too large", i);
    R[i] = S.rhs_per_task > 0 ? S.rhs_per_task : pick_R(S.n, tpr[i], S.nrhs);
    if (R[i] > S.nrhs) R[i] = S.nrhs;
    if (rka::batch_lds_bytes(S.n, R[i], tpr[i]) > 160 * 1024 - 4096)
      return rka::api_fail(RKA_EINVAL, "system %d: a task of %d right-hand sides does not fit LDS", i, R[i]);
    if (S.max_iter > max_iter) max_iter = S.max_iter;
  }

  DevBuf buf(s);
  std::vector<BatchSys> hsys(count);
  std::vector<BatchTask> htask;
  std::vector<int32_t> task_sys;
  std::vector<int64_t> task_work;
  int64_t idx_total = 0;
  // Chunks are balanced in time, not in iterations: an iteration of system s
  // is a chain of bs_s dependent projections plus the average, so system s
  // advances kc_s ~ kChunkSteps / (bs_s + 2) iterations per chunk and no task
  // holds a chunk open for the others.  The chunk's row streams stay within
  // 64 Mi indices (the budget is scaled down if needed).
  std::vector<int64_t> kc(count);
  {
    double steps = rka::kChunkSteps;
    double idx_need = 0.0;
    for (int i = 0; i < count; ++i)
      idx_need += steps / (bs[i] + 2.0) * (double)q[i] * bs[i];
    if (idx_need > (double)(64ll << 20)) steps *= (double)(64ll << 20) / idx_need;
    for (int i = 0; i < count; ++i) {
      int64_t k = (int64_t)(steps / (bs[i] + 2.0));
      if (k < 1) k = 1;
      if (chunk_iters > 0 && k > chunk_iters) k = chunk_iters;
      const int64_t cap = systems[i].max_iter > 0 ? systems[i].max_iter : 1;
      kc[i] = k < cap ? k : cap;
    }
  }
  int64_t nchunks = 0;
  for (int i = 0; i < count; ++i)
    nchunks = std::max(nchunks, (systems[i].max_iter + kc[i] - 1) / kc[i]);
  double* wbuf;
  double* cbuf;
  int64_t* lastbuf;
  int64_t mtot = 0;
  for (int i = 0; i < count; ++i) mtot += systems[i].m;
  BHIP(buf.get(&wbuf, (size_t)mtot));
  BHIP(buf.get(&cbuf, (size_t)mtot));
  BHIP(buf.get(&lastbuf, (size_t)count));
  for (int i = 0; i < count; ++i) idx_total += kc[i] * q[i] * bs[i];
  int32_t* idxbuf;
  BHIP(buf.get(&idxbuf, (size_t)idx_total));
  int64_t moff = 0, ioff = 0, roff = 0;
  for (int i = 0; i < count; ++i) {
    const rka_batch_system& S = systems[i];
    BatchSys& Y = hsys[i];
    Y.c = cbuf + moff;
    Y.last_pos = lastbuf + i;
    Y.m = S.m;
    Y.seed = seed + (uint64_t)i;
    Y.kc = kc[i];
    Y.max_iter = S.max_iter;
    Y.q = q[i];
    Y.bs = bs[i];
    Y.idx = idxbuf + ioff;
    Y.alive = nullptr;
    for (int r0 = 0; r0 < S.nrhs; r0 += R[i]) {
      BatchTask T;
      T.A = S.A;
      T.m = S.m;
      T.n = S.n;
      T.lda = S.lda;
      T.b = S.b + (int64_t)r0 * S.ldb;
      T.ldb = S.ldb;
      T.x = S.x + (int64_t)r0 * S.ldx;
      T.ldx = S.ldx;
      T.xr = S.x_ref ? S.x_ref + (int64_t)r0 * S.ldxr : nullptr;
      T.ldxr = S.ldxr;
      T.w = wbuf + moff;
      T.idx = Y.idx;
      T.alpha = (float)(S.alpha > 0.0 ? S.alpha : 1.0);
      T.R = S.nrhs - r0 < R[i] ? S.nrhs - r0 : R[i];
      T.q = q[i];
      T.bs = bs[i];
      T.tpr = tpr[i];
      T.bf16 = dtype == RKA_BF16;
      T.max_iter = S.max_iter;
      T.kc = kc[i];
      T.ref2 = 0.0;
      if (ref2_rhs)
        for (int r = 0; r < T.R; ++r) T.ref2 += ref2_rhs[roff + r0 + r];
      htask.push_back(T);
      task_sys.push_back(i);
      task_work.push_back((int64_t)T.R * S.n * q[i] * bs[i] * (S.max_iter > 0 ? S.max_iter : 1));
    }
    moff += S.m;
    ioff += kc[i] * q[i] * bs[i];
    roff += S.nrhs;
  }
  const int ntask = (int)htask.size();
  // largest tasks first, so that the long ones start at once
  std::vector<int> order(ntask);
  for (int t = 0; t < ntask; ++t) order[t] = t;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return task_work[a] > task_work[b]; });
  std::vector<BatchTask> sorted(ntask);
  std::vector<int32_t> sorted_sys(ntask);
  for (int t = 0; t < ntask; ++t) {
    sorted[t] = htask[order[t]];
    sorted_sys[t] = task_sys[order[t]];
  }
  int32_t *done, *alive, *tsys;
  int64_t *iters, *best_k;
  double *rel, *best;
  BatchTask* dtask;
  BatchSys* dsys;
  BHIP(buf.get(&done, (size_t)ntask));
  BHIP(buf.get(&alive, (size_t)count));
  BHIP(buf.get(&tsys, (size_t)ntask));
  BHIP(buf.get(&iters, (size_t)ntask));
  BHIP(buf.get(&rel, (size_t)ntask));
  BHIP(buf.get(&best, (size_t)ntask));
  BHIP(buf.get(&best_k, (size_t)ntask));
  BHIP(buf.get(&dtask, (size_t)ntask));
  BHIP(buf.get(&dsys, (size_t)count));
  for (int t = 0; t < ntask; ++t) {
    sorted[t].done = done;
    sorted[t].alive = alive;
    sorted[t].iters = iters;
    sorted[t].rel = rel;
    sorted[t].best = best;
    sorted[t].best_k = best_k;
  }
  for (int i = 0; i < count; ++i) hsys[i].alive = alive + i;
  BHIP(hipMemcpyAsync(dtask, sorted.data(), ntask * sizeof(BatchTask), hipMemcpyHostToDevice, s));
  BHIP(hipMemcpyAsync(dsys, hsys.data(), count * sizeof(BatchSys), hipMemcpyHostToDevice, s));
  BHIP(hipMemcpyAsync(tsys, sorted_sys.data(), ntask * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // NaN pattern for rel (never measured)
  {
    std::vector<double> nanv(ntask, NAN);
    BHIP(hipMemcpyAsync(rel, nanv.data(), ntask * sizeof(double), hipMemcpyHostToDevice, s));
    BHIP(hipStreamSynchronize(s));  // the host vectors go out of scope
  }
  size_t lds = 0;
  int64_t draws_max = 0;
  for (int t = 0; t < ntask; ++t)
    lds = std::max(lds, rka::batch_lds_bytes(sorted[t].n, sorted[t].R, sorted[t].tpr));
  for (int i = 0; i < count; ++i) draws_max = std::max(draws_max, kc[i] * q[i] * bs[i]);
  if (lds > 64 * 1024)
    BHIP(hipFuncSetAttribute((const void*)rka::batch_iter_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));

  // The whole solve as one launch sequence (captured in a graph if asked):
  // per system norms and running sum, flag set-up, then per chunk the row
  // streams of every running system, the iteration launch and the
  // bookkeeping of which systems still run.
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (auto& e : ev) BHIP(hipEventCreate(&e));
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() {
      for (int i = 0; i < 3; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
    }
  } ev_free{ev};
  if (use_graph)
    BHIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  else
    BHIP(hipEventRecord(ev[0], s));
  {
    int64_t off = 0;
    for (int i = 0; i < count; ++i) {
      const rka_batch_system& S = systems[i];
      const bool vec_ok = ((uintptr_t)S.A % 16 == 0) &&
                          ((S.lda * (dtype == RKA_F32 ? 4 : 2)) % 16 == 0) &&
                          (S.n % (dtype == RKA_F32 ? 4 : 8) == 0);
      hipError_t e = rka::launch_row_norms(S.A, dtype, S.m, S.n, S.lda, vec_ok, wbuf + off, s);
      if (e == hipSuccess) e = rka::launch_prefix(wbuf + off, S.m, cbuf + off, lastbuf + i, nullptr, s);
      if (e != hipSuccess) {
        if (use_graph) {
          hipGraph_t g2;
          (void)hipStreamEndCapture(s, &g2);
          if (g2) (void)hipGraphDestroy(g2);
        }
        return rka::api_fail(RKA_EDEVICE, "batch set-up: %s", hipGetErrorString(e));
      }
      off += S.m;
    }
    hipLaunchKernelGGL(rka::batch_fill_kernel, dim3(1), dim3(256), 0, s, done, (int64_t)ntask, 0);
    hipLaunchKernelGGL(rka::batch_fill_kernel, dim3(1), dim3(256), 0, s, (int32_t*)iters,
                       (int64_t)ntask * 2, 0);
    hipLaunchKernelGGL(rka::batch_fill_kernel, dim3(1), dim3(256), 0, s, (int32_t*)best_k,
                       (int64_t)ntask * 2, 0);
    hipLaunchKernelGGL(rka::batch_fill64_kernel, dim3(1), dim3(256), 0, s, best, (int64_t)ntask,
                       (double)INFINITY);
    hipLaunchKernelGGL(rka::batch_fill_kernel, dim3(1), dim3(256), 0, s, alive, (int64_t)count, 1);
    if (!use_graph) (void)hipEventRecord(ev[1], s);
    int nb = (int)((draws_max + 255) / 256);
    if (nb > 1024) nb = 1024;
    for (int64_t c = 0; c < nchunks; ++c) {
      hipLaunchKernelGGL(rka::batch_sample_kernel, dim3(nb, count), dim3(256), 0, s, dsys, c);
      if (dump) {
        int64_t doff = 0;
        for (int i = 0; i < count; ++i) {
          const int64_t per = (int64_t)q[i] * bs[i], k0 = c * kc[i], mi = systems[i].max_iter;
          if (k0 < mi) {
            const int64_t K = mi - k0 < kc[i] ? mi - k0 : kc[i];
            (void)hipMemcpyAsync(dump + doff + k0 * per, hsys[i].idx, (size_t)(K * per) * 4,
                                 hipMemcpyDeviceToDevice, s);
          }
          doff += mi * per;
        }
        continue;
      }
      hipLaunchKernelGGL(rka::batch_iter_kernel, dim3(ntask), dim3(rka::kBT), (unsigned)lds, s,
                         dtask, c, tol > 0.0 ? check_every : 0, tol * tol);
      hipLaunchKernelGGL(rka::batch_alive_kernel, dim3((count + 255) / 256), dim3(256), 0, s,
                         done, tsys, ntask, alive, count);
    }
  }
  hipError_t le = hipGetLastError();
  if (use_graph) {
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (e == hipSuccess && le == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    if (e == hipSuccess && le == hipSuccess) e = hipEventRecord(ev[0], s);
    if (e == hipSuccess && le == hipSuccess) e = hipGraphLaunch(gexec, s);
    if (e != hipSuccess) le = e;
  }
  if (le == hipSuccess) le = hipEventRecord(ev[2], s);
  if (le != hipSuccess) {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    return rka::api_fail(RKA_EDEVICE, "batch launch: %s", hipGetErrorString(le));
  }
  std::vector<int32_t> hdone(ntask);
  std::vector<int64_t> hiters(ntask);
  std::vector<double> hrel(ntask);
  BHIP(hipMemcpyAsync(hdone.data(), done, ntask * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(hiters.data(), iters, ntask * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BHIP(hipMemcpyAsync(hrel.data(), rel, ntask * sizeof(double), hipMemcpyDeviceToHost, s));
  BHIP(hipStreamSynchronize(s));
  if (gexec) (void)hipGraphExecDestroy(gexec);
  if (graph) (void)hipGraphDestroy(graph);
  int status = RKA_OK;
  if (results) {
    for (int i = 0; i < count; ++i) {
      results[i].iterations = 0;
      results[i].status = RKA_OK;
      results[i].rel = 0.0;
      results[i].q = q[i];
      results[i].block_size = bs[i];
      results[i].tpr = tpr[i];
      results[i].rhs_per_task = R[i];
      results[i].alpha = systems[i].alpha > 0.0 ? systems[i].alpha : 1.0;
    }
  }
  for (int t = 0; t < ntask; ++t) {
    const int i = sorted_sys[t];
    int st = RKA_OK;
    if (hdone[t] == 2) st = RKA_EDIVERGED;
    else if (tol > 0.0 && hdone[t] != 1) st = RKA_NOT_CONVERGED;
    if (results) {
      rka_batch_result& Rr = results[i];
      Rr.iterations = std::max(Rr.iterations, hiters[t]);
      if (st < 0 || (st > Rr.status && Rr.status >= 0)) Rr.status = st;
      if (!isnan(hrel[t])) Rr.rel = std::max(Rr.rel, hrel[t]);
    }
    if (st < 0) status = st;
    else if (st > 0 && status == RKA_OK) status = st;
  }
  if (stats) {
    float ms = 0.f;
    if (use_graph) {
      if (hipEventElapsedTime(&ms, ev[0], ev[2]) == hipSuccess) stats->iterate_ms = ms;
    } else {
      if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) stats->setup_ms = ms;
      if (hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess) stats->iterate_ms = ms;
    }
    stats->tasks = ntask;
    stats->chunks = (int32_t)nchunks;
    stats->lds_bytes = (int32_t)lds;
    stats->graph = use_graph ? 1 : 0;
  }
  return status;
}

extern "C" int rka_batch_solve(const rka_batch_system* systems, int32_t count, int dtype,
                               uint64_t seed, double tol, int64_t check_every, int64_t chunk_iters,
                               int32_t use_graph, void* stream, rka_batch_result* results,
                               rka_batch_stats* stats) {
  return batch_core(systems, count, dtype, seed, tol, check_every, chunk_iters, use_graph, stream,
                    results, stats, nullptr);
}

extern "C" int rka_batch_sample_indices(const rka_batch_system* systems, int32_t count,
                                        int dtype, uint64_t seed, int64_t chunk_iters,
                                        int32_t* idx, void* stream) {
  if (!idx) return rka::api_fail(RKA_EINVAL, "idx must be non-null");
  if (systems)
    for (int i = 0; i < count; ++i)
      if (systems[i].q < 1 || systems[i].block_size < 1)
        return rka::api_fail(RKA_EINVAL, "system %d: give q and block_size (>= 1)", i);
  const int rc = batch_core(systems, count, dtype, seed, 0.0, 1, chunk_iters, 0, stream, nullptr,
                            nullptr, nullptr, idx);
  if (rc < 0) return rc;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return rka::api_fail(RKA_EDEVICE, "batch row stream copy failed");
  return RKA_OK;
}

// Refinement of a batch: every sweep solves, for all systems at once and in
// binary32, for the corrections d with A d = b - A x (FP64 residuals), then
// x += d in FP64 -- the batch form of rka_refine_solve.  Sweep s draws its
// rows with keys seed + s * 65536 + i.
extern "C" int rka_batch_refine_solve(const rka_batch_system* systems, int32_t count, int dtype,
                                      uint64_t seed, double tol, int64_t check_every,
                                      int32_t sweeps, int32_t use_graph, void* stream,
                                      rka_batch_result* results, rka_batch_stats* stats) {
  if (stats) memset(stats, 0, sizeof *stats);
  if (!systems || count < 1 || count > 65535)
    return rka::api_fail(RKA_EINVAL, "need 1 to 65535 systems");
  if (sweeps < 1) return rka::api_fail(RKA_EINVAL, "sweeps must be >= 1");
  if (dtype != RKA_F32 && dtype != RKA_BF16)
    return rka::api_fail(RKA_EINVAL, "batched solves take RKA_F32 or RKA_BF16 storage");
  if (!(tol >= 0.0) || !isfinite(tol)) return rka::api_fail(RKA_EINVAL, "tol must be finite and >= 0");
  for (int i = 0; i < count; ++i) {
    int v = validate_sys(systems[i], i, dtype);
    if (v != RKA_OK) return v;
  }
  if (rka::api_num_cus() <= 0) return rka::api_fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  const int es = dtype == RKA_F32 ? 4 : 2;
  // scratch: per system and right-hand side a residual (m), a correction (n)
  // and, with a reference, its target x_ref - x (n)
  int64_t nr = 0, rtot = 0, ntot = 0;
  for (int i = 0; i < count; ++i) {
    nr += systems[i].nrhs;
    rtot += systems[i].nrhs * systems[i].m;
    ntot += systems[i].nrhs * systems[i].n;
  }
  bool have_ref = true;
  for (int i = 0; i < count; ++i) have_ref = have_ref && systems[i].x_ref;
  DevBuf buf(s);
  double *rbuf, *dbuf, *drbuf = nullptr, *part, *n2;
  BHIP(buf.get(&rbuf, (size_t)rtot));
  BHIP(buf.get(&dbuf, (size_t)ntot));
  BHIP(buf.get(&part, (size_t)rka::sumsq_part_len()));
  BHIP(buf.get(&n2, (size_t)nr));
  if (have_ref) BHIP(buf.get(&drbuf, (size_t)ntot));
  std::vector<double> ref2(nr, 0.0);
  if (have_ref) {
    int64_t k = 0;
    for (int i = 0; i < count; ++i)
      for (int r = 0; r < systems[i].nrhs; ++r, ++k)
        BHIP(rka::launch_sumsq(systems[i].x_ref + r * systems[i].ldxr, nullptr, systems[i].n,
                               part, n2 + k, s));
    BHIP(hipMemcpyAsync(ref2.data(), n2, nr * sizeof(double), hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
  }
  std::vector<rka_batch_system> sub(systems, systems + count);
  std::vector<rka_batch_result> res(count), acc(count);
  for (int i = 0; i < count; ++i) {
    acc[i] = rka_batch_result{};
    acc[i].status = RKA_OK;
  }
  int status = RKA_OK;
  for (int sw = 0; sw < sweeps; ++sw) {
    int64_t ro = 0, no = 0;
    for (int i = 0; i < count; ++i) {
      const rka_batch_system& S = systems[i];
      const bool vec = ((uintptr_t)S.A % 16 == 0) && ((S.lda * es) % 16 == 0) &&
                       (S.n % (16 / es) == 0);
      for (int r = 0; r < S.nrhs; ++r) {
        BHIP(rka::launch_gemv(S.A, dtype, S.m, S.n, S.lda, vec, S.x + r * S.ldx, S.b + r * S.ldb,
                              -1.0, rbuf + ro + r * S.m, s));
        if (have_ref)
          BHIP(rka::launch_sub(drbuf + no + r * S.n, S.x_ref + r * S.ldxr, S.x + r * S.ldx, S.n,
                               s));
      }
      BHIP(hipMemsetAsync(dbuf + no, 0, (size_t)S.nrhs * S.n * sizeof(double), s));
      sub[i].b = rbuf + ro;
      sub[i].ldb = S.m;
      sub[i].x = dbuf + no;
      sub[i].ldx = S.n;
      sub[i].x_ref = have_ref ? drbuf + no : nullptr;
      sub[i].ldxr = S.n;
      ro += S.nrhs * S.m;
      no += S.nrhs * S.n;
    }
    rka_batch_stats st;
    const int rc = batch_core(sub.data(), count, dtype, seed + (uint64_t)sw * 65536u, tol,
                              check_every, 0, use_graph, stream, res.data(), &st,
                              have_ref ? ref2.data() : nullptr);
    if (rc < 0 && rc != RKA_EDIVERGED) return rc;
    no = 0;
    bool all_ok = true;
    for (int i = 0; i < count; ++i) {
      const rka_batch_system& S = systems[i];
      for (int r = 0; r < S.nrhs; ++r)
        BHIP(rka::launch_axpy(S.x + r * S.ldx, dbuf + no + r * S.n, S.n, s));
      no += S.nrhs * S.n;
      acc[i].iterations += res[i].iterations;
      acc[i].rel = res[i].rel;
      acc[i].status = res[i].status;
      acc[i].q = res[i].q;
      acc[i].block_size = res[i].block_size;
      acc[i].tpr = res[i].tpr;
      acc[i].rhs_per_task = res[i].rhs_per_task;
      acc[i].alpha = res[i].alpha;
      all_ok = all_ok && res[i].status == RKA_OK;
    }
    if (stats) {
      stats->tasks = st.tasks;
      stats->chunks += st.chunks;
      stats->lds_bytes = st.lds_bytes;
      stats->graph = st.graph;
      stats->setup_ms += st.setup_ms;
      stats->iterate_ms += st.iterate_ms;
    }
    status = rc;
    if (tol > 0.0 && all_ok) break;
  }
  BHIP(hipStreamSynchronize(s));
  if (results)
    for (int i = 0; i < count; ++i) results[i] = acc[i];
  return status;
}

// ---------------------------------------------------------------------------
// Autotuner.  Systems are grouped by size class (n rounded up to a power of
// two).  On each class's median system, every candidate (tpr, q, block_size)
// runs from x = 0 for about m/2 projections; from the residual reduction rho
// and the HIP-event time t of the iterations it gets the progress per
// millisecond, r_t = ln(1/rho) / t, and per projection, r_p = ln(1/rho) / P.
// The batch then runs all tasks at once, so its time to a 10^-6 residual
// reduction (E = ln 10^6) is modelled as
//     max( max_c E / r_t(c) ,  sum_c tasks_c * (E / r_p(c)) * bytes_c / BW )
// -- the slowest task's own chain against the row bytes of all tasks through
// HBM (BW = 5 TB/s, the rate the row gathers reach on this device).  The
// tuner starts from the fastest candidate of every class and, while the
// bandwidth term dominates, moves one class at a time to the candidate that
// lowers the modelled time most.  Candidates: tpr in {t0, 2 t0} (t0 the
// smallest that covers a row) with W = 256 / tpr the workers a workgroup
// runs at once; RKAB with alpha = 1, q in {1, W/4, W} and block_size in
// {n/8, n/2} clipped to [1, 256]; RKA (block size 1) with q = W and alpha in
// {W/4, W/2} -- a weight above 1 is what makes averaging pay (Eq. (6)), and
// these stay well inside the range where it contracts when sigma_max^2 /
// ||A||_F^2 is small next to 1/q.  Only parameters the caller left at 0 are
// written; x is not touched.  The progress measure is the residual, so the tuner is meant for
// consistent systems (inconsistent ones stall at the least-squares residual,
// Sec. 2.3.1).
// ---------------------------------------------------------------------------
namespace {
struct Cand {
  int tpr, q, bs;
  double alpha;
  double rt, rp;  // e-folds per ms, per projection
};
}  // namespace

extern "C" int rka_batch_tune(rka_batch_system* systems, int32_t count, int dtype, uint64_t seed,
                              void* stream, int32_t* trials) {
  if (trials) *trials = 0;
  if (!systems || count < 1 || count > 65535)
    return rka::api_fail(RKA_EINVAL, "need 1 to 65535 systems");
  if (dtype != RKA_F32 && dtype != RKA_BF16)
    return rka::api_fail(RKA_EINVAL, "batched solves take RKA_F32 or RKA_BF16 storage");
  for (int i = 0; i < count; ++i) {
    int v = validate_sys(systems[i], i, dtype);
    if (v != RKA_OK) return v;
  }
  if (rka::api_num_cus() <= 0) return rka::api_fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  const int esz = dtype == RKA_F32 ? 4 : 2;
  std::vector<std::vector<int>> cls(16);
  for (int i = 0; i < count; ++i) {
    int c = 0;
    while ((int64_t)1 << c < systems[i].n) ++c;
    cls[c].push_back(i);
  }
  int64_t mmax = 0, nmax = 0;
  for (int i = 0; i < count; ++i) {
    mmax = std::max(mmax, systems[i].m);
    nmax = std::max(nmax, systems[i].n);
  }
  DevBuf buf(s);
  double *x, *r, *part, *acc;
  BHIP(buf.get(&x, (size_t)nmax));
  BHIP(buf.get(&r, (size_t)mmax));
  BHIP(buf.get(&part, (size_t)rka::sumsq_part_len()));
  BHIP(buf.get(&acc, 2));
  int ntrials = 0;
  struct Class {
    std::vector<int> members;
    std::vector<Cand> cands;
    double tasks = 0, bytes = 0;  // tasks of the class, row bytes per projection
    int pick = -1;
  };
  std::vector<Class> classes;
  for (auto& members : cls) {
    if (members.empty()) continue;
    std::vector<int> byw(members);
    std::sort(byw.begin(), byw.end(), [&](int a, int b) {
      return systems[a].m * systems[a].n < systems[b].m * systems[b].n;
    });
    const rka_batch_system& Rp = systems[byw[byw.size() / 2]];
    const int64_t n = Rp.n;
    Class C;
    C.members = members;
    for (int i : members) C.tasks += systems[i].nrhs;
    C.bytes = (double)n * esz + 16.0;
    BHIP(rka::launch_sumsq(Rp.b, nullptr, Rp.m, part, acc + 1, s));
    double b2 = 0.0;
    BHIP(hipMemcpyAsync(&b2, acc + 1, sizeof b2, hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    if (!(b2 > 0.0)) continue;
    const int t0 = min_tpr(n);
    // (tpr, q, block_size, alpha) candidates: RKAB with alpha = 1, and RKA
    // (block size 1) with alpha = q/4 and q/2 (inside the range where Eq. (6)'s
    // weight contracts for these spectra, sigma_max^2 / ||A||_F^2 << 1 / q)
    std::vector<Cand> trial;
    for (int tpr = t0; tpr <= 256 && tpr <= 2 * t0; tpr *= 2) {
      const int W = rka::kBT / tpr;
      const int qs[3] = {1, W / 4 > 1 ? W / 4 : 1, W};
      for (int qi = 0; qi < 3; ++qi) {
        if (qi > 0 && qs[qi] == qs[qi - 1]) continue;
        const int64_t bss[2] = {std::min<int64_t>(256, std::max<int64_t>(1, n / 8)),
                                std::min<int64_t>(256, std::max<int64_t>(1, n / 2))};
        for (int bi = 0; bi < 2; ++bi) {
          if (bi > 0 && bss[bi] == bss[0]) continue;
          trial.push_back({tpr, qs[qi], (int)bss[bi], 1.0, 0.0, 0.0});
        }
      }
      if (W >= 4) {
        trial.push_back({tpr, W, 1, W / 4.0, 0.0, 0.0});
        trial.push_back({tpr, W, 1, W / 2.0, 0.0, 0.0});
      }
    }
    for (const Cand& cd : trial) {
      const int q = cd.q, bs = cd.bs, tpr = cd.tpr;
      const int64_t K = std::max<int64_t>(1, Rp.m / 2 / ((int64_t)q * bs));
      rka_batch_system T = Rp;
      T.nrhs = 1;
      T.x = x;
      T.ldx = n;
      T.x_ref = nullptr;
      T.q = q;
      T.block_size = bs;
      T.tpr = tpr;
      T.alpha = cd.alpha;
      T.rhs_per_task = 1;
      T.max_iter = K;
      BHIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(double), s));
      rka_batch_stats st;
      int rc = rka_batch_solve(&T, 1, dtype, seed, 0.0, 1, 0, 0, stream, nullptr, &st);
      if (rc < 0) return rc;
      BHIP(rka::launch_gemv(Rp.A, dtype, Rp.m, n, Rp.lda, false, x, Rp.b, -1.0, r, s));
      BHIP(rka::launch_sumsq(r, nullptr, Rp.m, part, acc, s));
      double r2 = 0.0;
      BHIP(hipMemcpyAsync(&r2, acc, sizeof r2, hipMemcpyDeviceToHost, s));
      BHIP(hipStreamSynchronize(s));
      ++ntrials;
      double rho = sqrt(r2 / b2);
      if (!(rho > 1e-30)) rho = 1e-30;
      if (!isfinite(rho) || rho >= 1.0) continue;
      const double ms = st.iterate_ms > 1e-3 ? st.iterate_ms : 1e-3;
      const double ef = -log(rho);
      Cand c = cd;
      c.rt = ef / ms;
      c.rp = ef / (double)(K * q * bs);
      C.cands.push_back(c);
    }
    if (C.cands.empty()) continue;
    int best = 0;
    for (int k = 1; k < (int)C.cands.size(); ++k)
      if (C.cands[k].rt > C.cands[best].rt) best = k;
    C.pick = best;
    classes.push_back(C);
  }
  // batch model: max(latency of the slowest class, row bytes of all tasks / BW)
  const double E = log(1e6), BW = 5e12 / 1e3;  // bytes per ms
  auto model = [&](const std::vector<Class>& cs, double* lat, double* bw) {
    *lat = 0.0;
    *bw = 0.0;
    for (const Class& C : cs) {
      const Cand& k = C.cands[C.pick];
      *lat = std::max(*lat, E / k.rt);
      *bw += C.tasks * (E / k.rp) * C.bytes / BW;
    }
    return std::max(*lat, *bw);
  };
  double lat, bw;
  double cur = model(classes, &lat, &bw);
  for (int guard = 0; guard < 64 && bw > lat; ++guard) {
    int bc = -1, bk = -1;
    double bt = cur;
    for (int c = 0; c < (int)classes.size(); ++c) {
      const int keep = classes[c].pick;
      for (int k = 0; k < (int)classes[c].cands.size(); ++k) {
        if (k == keep) continue;
        classes[c].pick = k;
        double l2, b2;
        const double t = model(classes, &l2, &b2);
        if (t < bt) {
          bt = t;
          bc = c;
          bk = k;
        }
      }
      classes[c].pick = keep;
    }
    if (bc < 0) break;
    classes[bc].pick = bk;
    cur = model(classes, &lat, &bw);
  }
  for (const Class& C : classes) {
    const Cand& k = C.cands[C.pick];
    for (int i : C.members) {
      if (systems[i].tpr == 0) systems[i].tpr = k.tpr;
      if (systems[i].q == 0) systems[i].q = k.q;
      if (systems[i].block_size == 0) systems[i].block_size = k.bs;
      if (systems[i].alpha == 0.0) systems[i].alpha = k.alpha;
      if ((int64_t)systems[i].tpr * rka::kEptMax < systems[i].n) systems[i].tpr = min_tpr(systems[i].n);
    }
  }
  if (trials) *trials = ntrials;
  return RKA_OK;
}
