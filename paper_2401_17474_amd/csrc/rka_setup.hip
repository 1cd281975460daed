// rka_setup.hip -- the sampler side of the hot path on gfx950:
//   * squared row norms (numerators of Eq. (4), arXiv 2401.17474 Sec. 2.2),
//   * their running sum (the inverse-CDF table; its last entry is ||A||_F^2),
//   * the Philox4x32-10 row stream, drawn in bulk ahead of the iterations
//     (rows do not depend on x, so they are sampled before they are needed).
//
// This translation unit is compiled with -ffp-contract=off and uses explicit
// round-to-nearest intrinsics: every square and every add is one rounded IEEE
// operation in the order stated, so norms, table and indices match a plain
// left-to-right evaluation bit for bit.
#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// ---------------------------------------------------------------------------
// Row norms.  One thread owns one row and sums it strictly left to right.
// Rows are staged through LDS in tiles of kTileVecs vecs so that HBM reads
// stay coalesced (8 lanes cover 128 contiguous bytes of one row); the next
// tile is already in flight in registers while the current one is summed.
// ---------------------------------------------------------------------------
constexpr int kNormRows = 256;   // rows per workgroup = threads per workgroup
constexpr int kTileVecs = 8;     // vecs per row per tile
constexpr int kLoadsPerThread = kNormRows * kTileVecs / kNormRows;

template <typename T, int V>
__global__ __launch_bounds__(kNormRows) void row_norms_kernel(const T* __restrict__ A, int64_t m,
                                                              int64_t nvec, int64_t lda,
                                                              double* __restrict__ w) {
  using raw_t = typename Vec<T, V>::raw_t;
  // padded by one vec per row to keep the per-thread row walk conflict-free
  __shared__ raw_t tile[kNormRows][kTileVecs + 1];
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * kNormRows;

  raw_t next[kLoadsPerThread];
  auto issue = [&](int64_t v0) {
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
      const int lin = i * kNormRows + t;
      const int r = lin / kTileVecs, vc = lin % kTileVecs;
      const int64_t row = row0 + r, vec = v0 + vc;
      if (row < m && vec < nvec) next[i] = load_raw<T, V>(A + row * lda + vec * V);
    }
  };

  double s = 0.0;
  issue(0);
  for (int64_t v0 = 0; v0 < nvec; v0 += kTileVecs) {
#pragma unroll
    for (int i = 0; i < kLoadsPerThread; ++i) {
      const int lin = i * kNormRows + t;
      tile[lin / kTileVecs][lin % kTileVecs] = next[i];
    }
    __syncthreads();
    if (v0 + kTileVecs < nvec) issue(v0 + kTileVecs);
    const int nv = (int)((nvec - v0) < kTileVecs ? (nvec - v0) : kTileVecs);
    for (int vc = 0; vc < nv; ++vc) {
      const raw_t r = tile[t][vc];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double a = raw_elem<T, V>(r, e);
        s = __dadd_rn(s, __dmul_rn(a, a));
      }
    }
    __syncthreads();
  }
  if (row0 + t < m) w[row0 + t] = s;
}

// ---------------------------------------------------------------------------
// Running sum c_l = c_{l-1} + w_l.  The rounding of each add depends on the
// previous partial, so the chain is evaluated by one lane; the other lanes
// stream the next block of w into LDS while it runs.  Also records the last
// row with positive weight and validates the total.  With nseg > 1 workgroup
// g restarts the sum at row floor(g m / nseg) (the block sampled by worker g
// in the Distributed Approach of Sec. 3.3.2) and records its block's last
// positive row in last_pos[g].
// ---------------------------------------------------------------------------
constexpr int kPrefixThreads = 256;
constexpr int kPrefixBlock = 1024;

__global__ __launch_bounds__(kPrefixThreads) void prefix_kernel(const double* __restrict__ w_all,
                                                                int64_t m_all, int32_t nseg,
                                                                double* __restrict__ c_all,
                                                                int64_t* __restrict__ last_pos,
                                                                DevStatus* st) {
  const int64_t lo = (int64_t)blockIdx.x * m_all / nseg;
  const int64_t m = ((int64_t)blockIdx.x + 1) * m_all / nseg - lo;
  const double* __restrict__ w = w_all + lo;
  double* __restrict__ c = c_all + lo;
  __shared__ double in[2][kPrefixBlock];
  __shared__ double out[kPrefixBlock];
  __shared__ double carry_s;
  __shared__ long long last_s;
  const int t = threadIdx.x;
  if (t == 0) {
    carry_s = 0.0;
    last_s = -1;
  }
  for (int i = t; i < kPrefixBlock; i += kPrefixThreads) in[0][i] = (i < m) ? w[i] : 0.0;
  __syncthreads();
  int slot = 0;
  for (int64_t base = 0; base < m; base += kPrefixBlock) {
    const int cnt = (int)((m - base) < kPrefixBlock ? (m - base) : kPrefixBlock);
    if (t == 0) {
      // The sequential chain, on one lane of wave 0, branch-free: weights are
      // read from LDS a batch at a time, the block is zero-padded past m
      // (adding +0.0 leaves a non-negative running sum unchanged) and the last
      // positive row is tracked with a select.
      double run = carry_s;
      int lastv = -1;
      constexpr int kBatch = 32;
      for (int i0 = 0; i0 < cnt; i0 += kBatch) {
        double wv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) wv[u] = in[slot][i0 + u];  // in-bounds: block of 1024
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          run = __dadd_rn(run, wv[u]);
          out[i0 + u] = run;
          lastv = wv[u] > 0.0 ? i0 + u : lastv;
        }
      }
      carry_s = run;
      if (lastv >= 0) last_s = base + lastv;
    } else if (t >= kWave) {
      // waves 1.. stream the next block of w into the other buffer
      const int64_t nb = base + kPrefixBlock;
      for (int i = t - kWave; i < kPrefixBlock; i += kPrefixThreads - kWave)
        in[slot ^ 1][i] = (nb + i < m) ? w[nb + i] : 0.0;
    }
    __syncthreads();
    for (int i = t; i < cnt; i += kPrefixThreads) c[base + i] = out[i];
    __syncthreads();
    slot ^= 1;
  }
  if (t == 0) {
    const int64_t lastg = last_s >= 0 ? lo + last_s : -1;
    if (last_pos) last_pos[blockIdx.x] = lastg;
    if (st) {
      if (nseg == 1) st->last_pos = lastg;
      const double W = carry_s;
      if (!(W > 0.0) || !isfinite(W)) {
        st->status = -2;  // RKA_EZERONORM (of the matrix, or of one worker's block)
        st->done = 1;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Row stream: idx[(kl*q + w)*bs + j] for kl < K.  Inverse-CDF pick: the
// smallest l with c_l > u * c[m-1]; none (only possible for u = 1) falls back
// to the last row with positive weight.
// ---------------------------------------------------------------------------
//
// blocks != 0: worker w draws from its own rows [floor(w m / q), floor((w+1)
// m / q)) with the running sum restarted at the block (Distributed Approach,
// Sec. 3.3.2).  walpha (nullable): the relaxation weight of each worker (the
// partial-matrix alpha of Sec. 3.3.2), else alpha for all.
__global__ __launch_bounds__(256) void sample_kernel(const double* __restrict__ c, int64_t m,
                                                     const int64_t* __restrict__ last_pos,
                                                     uint64_t seed, int64_t k_base, int64_t K,
                                                     int32_t q, int32_t bs, uint32_t dom,
                                                     int32_t mode, double alpha,
                                                     const double* __restrict__ walpha,
                                                     const double* __restrict__ wrow,
                                                     int32_t* __restrict__ idx,
                                                     RowRec* __restrict__ rec,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ wn,
                                                     const DevStatus* st) {
  if (st && st->done) return;
  const int64_t total = K * (int64_t)q * bs;
  for (int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; L < total;
       L += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = L % bs;
    const int64_t wk = (L / bs) % q;
    const int64_t kl = L / ((int64_t)bs * q);
    int64_t i;
    if (mode == kSampleCyclic) {
      // position of the draw in the whole stream, rows taken in order
      const uint64_t pos = ((uint64_t)(k_base + kl) * (uint64_t)q + (uint64_t)wk) * (uint64_t)bs +
                           (uint64_t)j;
      i = (int64_t)(pos % (uint64_t)m);
    } else {
      const double u =
          draw_uniform(seed, (uint64_t)(k_base + kl), (uint32_t)wk, (uint32_t)j, dom);
      if (mode == kSampleBlocks) {
        const int64_t lo = wk * m / q, hi = (wk + 1) * m / q;
        i = lo + pick_row(c + lo, hi - lo, c[hi - 1], u, last_pos[wk] - lo);
      } else {
        i = pick_row(c, m, c[m - 1], u, *last_pos);
      }
    }
    if (idx) idx[L] = (int32_t)i;
    if (rec) {
      RowRec r;
      r.b = b[i];
      r.wn = wn[i];
      r.row = i;
      r.alpha = wrow ? wrow[i] : (walpha ? walpha[wk] : alpha);
      // Only the cyclic order reaches a zero row: its step leaves x as it is
      // (weight 0 over a unit norm keeps the scale finite and zero).
      if (r.wn == 0.0) {
        r.alpha = 0.0;
        r.wn = 1.0;
      }
      rec[L] = r;
    }
  }
}

// b must be finite (the right-hand side is data, checked on the device).
__global__ void check_finite_kernel(const double* __restrict__ v, int64_t len, DevStatus* st) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (!isfinite(v[i])) {
      __hip_atomic_store(&st->status, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <typename T, int V>
static hipError_t launch_norms_t(const void* A, int64_t m, int64_t n, int64_t lda, double* w,
                                 hipStream_t s) {
  const int64_t blocks = (m + kNormRows - 1) / kNormRows;
  hipLaunchKernelGGL((row_norms_kernel<T, V>), dim3((unsigned)blocks), dim3(kNormRows), 0, s,
                     (const T*)A, m, n / V, lda, w);
  return hipGetLastError();
}

hipError_t launch_row_norms(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                            bool vec_ok, double* w, hipStream_t s) {
  switch (dtype) {
    case 0:
      return vec_ok ? launch_norms_t<double, 2>(A, m, n, lda, w, s)
                    : launch_norms_t<double, 1>(A, m, n, lda, w, s);
    case 1:
      return vec_ok ? launch_norms_t<float, 4>(A, m, n, lda, w, s)
                    : launch_norms_t<float, 1>(A, m, n, lda, w, s);
    default:
      return vec_ok ? launch_norms_t<bf16_t, 8>(A, m, n, lda, w, s)
                    : launch_norms_t<bf16_t, 1>(A, m, n, lda, w, s);
  }
}

hipError_t launch_prefix(const double* w, int64_t m, double* c, int64_t* last_pos, DevStatus* st,
                         hipStream_t s) {
  hipLaunchKernelGGL(prefix_kernel, dim3(1), dim3(kPrefixThreads), 0, s, w, m, 1, c, last_pos, st);
  return hipGetLastError();
}

hipError_t launch_prefix_blocks(const double* w, int64_t m, int32_t nseg, double* c,
                                int64_t* last_pos, DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(prefix_kernel, dim3((unsigned)nseg), dim3(kPrefixThreads), 0, s, w, m, nseg,
                     c, last_pos, st);
  return hipGetLastError();
}

hipError_t launch_sample(const double* c, int64_t m, const int64_t* last_pos, uint64_t seed,
                         int64_t k_base, int64_t K, int32_t q, int32_t bs, int32_t dom,
                         int32_t mode, double alpha, const double* walpha, const double* wrow,
                         int32_t* idx, RowRec* rec, const double* b, const double* wn,
                         const DevStatus* st, hipStream_t s) {
  const int64_t total = K * (int64_t)q * bs;
  if (total <= 0) return hipSuccess;
  int64_t nb = (total + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(sample_kernel, dim3((unsigned)nb), dim3(256), 0, s, c, m, last_pos, seed,
                     k_base, K, q, bs, (uint32_t)dom, mode, alpha, walpha, wrow, idx, rec, b, wn, st);
  return hipGetLastError();
}

hipError_t launch_check_finite(const double* v, int64_t len, DevStatus* st, hipStream_t s) {
  int64_t blocks = (len + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v, len, st);
  return hipGetLastError();
}

}  // namespace rka
