// rka_rkab.hip -- RKAB (arXiv 2401.17474, Sec. 3.4.1, Algorithm 3) on gfx950:
// the worker-split persistent kernel.
//
// A worker's block of projections is a dependent chain (each projection
// reads the iterate the previous one produced), so a worker lives in one
// workgroup with its private iterate v in registers.  Rows are streamed
// from HBM through a three-deep register ring, so that two rows are always
// in flight while the third is projected.  The only grid-wide step per outer
// iteration is the average of the q iterates: every worker publishes v
// (agent-coherent stores), and after a grid barrier workgroup g averages a
// fixed slice of the columns over the workers in fixed order -- the layout
// of the per-thread iterate matrix of Sec. 3.3.1, one row per worker.
#include <math.h>

#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// Phase timing of workgroups 0 and G/2 (printed at the end of a launch), for
// builds with RKA_RKAB_PROF defined only.
#ifdef RKA_RKAB_PROF
#define RPROF_DECL                             \
  uint64_t rp_t[8] = {0, 0, 0, 0, 0, 0, 0, 0}; \
  uint64_t rp_last = __builtin_readcyclecounter();
#define RPROF(i)                                          \
  do {                                                    \
    const uint64_t rp_now = __builtin_readcyclecounter(); \
    rp_t[i] += rp_now - rp_last;                          \
    rp_last = rp_now;                                     \
  } while (0)
#else
#define RPROF_DECL
#define RPROF(i) \
  do {           \
  } while (0)
#endif

// ===========================================================================
// RKAB, worker-split persistent kernel.
// ===========================================================================
struct RkabArgs {
  const void* A;
  int64_t lda, nvec;
  const RowRec* rec;  // K x q x bs row records of the chunk
  double* x;
  const double* x_ref;
  double alpha;
  int32_t q, bs, G, ns;
  int64_t k0, K, check_every;
  void* vbuf;    // q x (nvec * V): the workers' iterates (accumulation type)
  int32_t avg_one_rsrc;  // the average's offsets fit 31 bits (one buffer resource)
  double* part;  // G
  unsigned* bar;
  DevStatus* st;
};

constexpr int kRkabThreads = 512;
constexpr int kStage = 256;  // row records staged in LDS per window slot

// W consecutive elements of C at byte offset `off` of a device-coherent
// buffer: one 16-byte access when W sizeof(C) = 16, else one element.  An
// offset at or past the buffer's end reads 0 and touches no memory (the
// range check applies to the lane's offset, so it is passed whole there).
template <typename C, int W>
__device__ __forceinline__ void load_units(__amdgpu_buffer_rsrc_t r, int off, C (&v)[W]) {
  if constexpr (W * sizeof(C) == 16) {
    const u32x4_t w = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kCoherentSC1);
    if constexpr (sizeof(C) == 8) {
      v[0] = __builtin_bit_cast(double, ((uint64_t)w[1] << 32) | w[0]);
      v[1] = __builtin_bit_cast(double, ((uint64_t)w[3] << 32) | w[2]);
    } else {
      // each element through a scalar: this compiler's bit cast of a vector
      // element expression reads element 0 whatever the index
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t e = w[k];
        v[k] = __builtin_bit_cast(float, e);
      }
    }
  } else if constexpr (sizeof(C) == 8) {
    v[0] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kCoherentSC1));
  } else {
    v[0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kCoherentSC1));
  }
}

// VLDS = false: the worker's iterate v lives in registers (short rows);
// VLDS = true: v lives in LDS (VPT * NT * V doubles of dynamic shared memory),
// leaving the registers to the row ring (long rows).  Each thread only ever
// touches its own vecs of v, so v needs no extra synchronisation.
//
// The worker's row records (index, b_i, ||a_i||^2) are staged in LDS in a
// sliding window of two kStage-entry slots, so that inside the projection
// loop the only global loads are the row data themselves and a projection
// never waits for anything but its own row.
//
// C is the accumulation type: double, or float for narrow storage (the inner
// solves of the precision form), in which case v, the dot products, the
// scales and the average are FP32.
template <typename T, typename C, int V, int VPT, bool VLDS>
__global__ __launch_bounds__(kRkabThreads) void rkab_kernel(RkabArgs p) {
  using raw_t = typename Vec<T, V>::raw_t;
  constexpr int NT = kRkabThreads;
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, g = blockIdx.x;
  const int64_t nvec = p.nvec, n = nvec * V;
  __shared__ double RED[NT / kWave];
  __shared__ C REDC[NT / kWave];
  __shared__ double Lb[2 * kStage], Lw[2 * kStage], La[2 * kStage];
  __shared__ int32_t Lr[2 * kStage];
  constexpr int kAW = 16 / (int)sizeof(C);  // elements of C in 16 bytes
  __shared__ C AV[kAW * NT];                 // partial sums of the average
  extern __shared__ double vlds_raw[];
  C* vlds = (C*)vlds_raw;
  C* vbuf = (C*)p.vbuf;

  C vreg[VLDS ? 1 : VPT][V];
  auto vat = [&](int i, int e) -> C& {
    if constexpr (VLDS)
      return vlds[(t + (int64_t)NT * i) * V + e];
    else
      return vreg[i][e];
  };
  // three row buffers used as a ring: two rows are in flight while the
  // third is projected, so a workgroup keeps ~2 rows of HBM reads queued
  raw_t B0[VPT], B1[VPT], B2[VPT];

  const RowRec* wrec = nullptr;  // this worker's records
  auto stage = [&](int blk, int bs) {
    const int j0 = blk * kStage;
    const int cnt = (bs - j0) < kStage ? (bs - j0) : kStage;
    const int base = (blk & 1) * kStage;
    for (int u = t; u < cnt; u += NT) {
      const RowRec r = wrec[j0 + u];
      Lb[base + u] = r.b;
      Lw[base + u] = r.wn;
      La[base + u] = r.alpha;
      Lr[base + u] = (int32_t)r.row;
    }
  };
  auto slot = [&](int j) { return ((j / kStage) & 1) * kStage + (j % kStage); };

  // Loads are unconditional (lanes past the row end re-read its last vec) and
  // lanes past the end are masked through the scale instead: a branch around
  // a load would make the compiler drain every in-flight load at the join.
  auto load_row = [&](raw_t (&dst)[VPT], int j) {
    const int64_t row = Lr[slot(j)];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int64_t c = t + (int64_t)NT * i;
      const int64_t cc = c < nvec ? c : nvec - 1;
      dst[i] = load_raw<T, V>(A + row * p.lda + cc * V);
    }
  };
  // v += alpha (b_i - <a_i, v>) / ||a_i||^2 a_i   (v is 0 on masked lanes)
  auto project = [&](const raw_t (&src)[VPT], int j) {
    C d = 0;
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
#pragma unroll
      for (int e = 0; e < V; ++e) d = fma(raw_elem_c<C, T, V>(src[i], e), vat(i, e), d);
    }
    const C D = block_sum(d, REDC);
    const int sl = slot(j);
    const C s = (C)La[sl] * ((C)Lb[sl] - D) / (C)Lw[sl];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const C si = (t + (int64_t)NT * i < nvec) ? s : (C)0;
#pragma unroll
      for (int e = 0; e < V; ++e) vat(i, e) = fma(si, raw_elem_c<C, T, V>(src[i], e), vat(i, e));
    }
  };

  const CoherentBuf xb(p.x, n);
  unsigned epoch = 0;  // grid barriers passed
  bool stopped = false;
  int64_t kl = 0;
  const int bs = p.bs;
  // Priming a worker: stage its first record blocks in LDS, then request its
  // first two rows.  The next worker of a workgroup (in this iteration or the
  // next) is primed before the current one publishes v and before the grid
  // barrier, so its rows stream in while the barrier and the average run.
  auto stage_first = [&](int64_t kp, int wp) {
    wrec = p.rec + (kp * p.q + wp) * (int64_t)bs;
    stage(0, bs);
    if (bs > kStage) stage(1, bs);
    __syncthreads();
  };
  auto issue_first = [&]() {
    load_row(B0, 0);
    load_row(B1, bs > 1 ? 1 : 0);  // unconditional (see load_row)
  };
  stage_first(0, g);
  issue_first();
  RPROF_DECL
  for (; kl < p.K; ++kl) {
    const int64_t k = p.k0 + kl;
    for (int w = g; w < p.q; w += p.G) {
      // v = x^(k) (coherent: x was written by other workgroups; 0 past the end)
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int64_t c = t + (int64_t)NT * i;
#pragma unroll
        for (int e = 0; e < V; ++e) vat(i, e) = (C)xb.load(c * V + e);
      }
      RPROF(0);
      int next_blk = 2;
      // block b goes into the slot of block b-2 once rows of block b-1 are
      // being projected; the ring looks at most four rows ahead
      auto restage = [&](int jj) {
        if (next_blk * kStage < bs && jj >= (next_blk - 1) * kStage) {
          __syncthreads();
          stage(next_blk, bs);
          __syncthreads();
          ++next_blk;
        }
      };
      int jj = 0;
      for (; jj + 5 <= bs; jj += 3) {
        restage(jj);
        load_row(B2, jj + 2);
        project(B0, jj);
        load_row(B0, jj + 3);
        project(B1, jj + 1);
        load_row(B1, jj + 4);
        project(B2, jj + 2);
      }
      restage(jj);
      // at most four rows remain: row jj is in B0, row jj+1 (if any) in B1
      if (jj + 2 < bs) load_row(B2, jj + 2);
      project(B0, jj);
      if (jj + 3 < bs) load_row(B0, jj + 3);
      if (jj + 1 < bs) project(B1, jj + 1);
      if (jj + 2 < bs) project(B2, jj + 2);
      if (jj + 3 < bs) project(B0, jj + 3);
      RPROF(1);
      const bool same_iter = w + p.G < p.q;
      __syncthreads();  // every thread is done with the staged records
      if (same_iter)
        stage_first(kl, w + p.G);
      else if (kl + 1 < p.K)
        stage_first(kl + 1, g);
      const CoherentOf<C> vw(vbuf + (size_t)w * n, n);  // stores past the end are dropped
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int64_t c = t + (int64_t)NT * i;
#pragma unroll
        for (int e = 0; e < V; ++e) vw.store(c * V + e, vat(i, e));
      }
      if (same_iter) issue_first();
      RPROF(2);
    }
    // grid barrier: v's published.  The workgroup arrives, then requests the
    // next iteration's first rows (to stream in during the wait and the
    // average), then waits: issuing two rows stalls on the CU's
    // outstanding-load limit, and before the arrival that stall delayed
    // every workgroup's arrival.
    wait_memory();
    RPROF(3);
    if (p.G > 1) grid_arrive(p.bar, epoch, (unsigned)p.G);
    if (kl + 1 < p.K) issue_first();
    bool ok = true;
    if (p.G > 1)
      ok = grid_wait(p.bar, epoch, (unsigned)p.G);
    else
      __syncthreads();
    RPROF(4);
    if (!ok) {
      if (t == 0) note_timeout(p.st);
      stopped = true;
      break;
    }
    // x^(k+1) = (1/q) sum_w v_w over this workgroup's column slice.  Each
    // element's sum over the workers is split over tpu threads (strided
    // worker subsets, each in increasing order) and the tpu partial sums are
    // then added in order: a fixed order for a given launch geometry.
    const bool check = p.check_every > 0 && ((k + 1) % p.check_every) == 0;
    const int64_t e0 = (int64_t)g * p.ns * V;
    const int64_t e1 = ((int64_t)(g + 1) * p.ns * V < n) ? (int64_t)(g + 1) * p.ns * V : n;
    const int E = e1 > e0 ? (int)(e1 - e0) : 0;
    constexpr int W = (V % kAW == 0) ? kAW : 1;  // elements per load of the split average
    // loads of a thread in flight (fewer for narrow storage, whose row
    // buffers leave fewer registers free)
    constexpr int kAvgDepth = V <= 2 ? 8 : 4;
    const int U = E / W;
    double err = 0.0;
    if (!p.avg_one_rsrc || U == 0 || U > NT) {
      // a thread per element, the workers in order
      for (int64_t ci = e0 + t; ci < e1; ci += NT) {
        C acc = 0;
        int w = 0;
        for (; w + 8 <= p.q; w += 8) {
          C vv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) vv[u] = CoherentOf<C>(vbuf + (size_t)(w + u) * n, n).load(ci);
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += vv[u];
        }
        for (; w < p.q; ++w) acc += CoherentOf<C>(vbuf + (size_t)w * n, n).load(ci);
        const C xn = acc / (C)p.q;
        xb.store(ci, (double)xn);
        if (check) {
          const double dd = (double)xn - p.x_ref[ci];
          err = fma(dd, dd, err);
        }
      }
    } else {
      // thread (lu, sub) sums unit lu of the slice (W consecutive elements,
      // one 16-byte access on the vector path) over the workers sub,
      // sub + tpu, ...; consecutive threads take consecutive units of the
      // same workers.  Every load goes through one buffer resource based at
      // the slice, uniform over the workgroup (a resource per worker would
      // differ between the lanes of a wave, and the compiler would then
      // serialise each load over the lanes' resources); offsets past the
      // last worker read 0 without touching memory.  kAvgDepth loads are in
      // flight before the first addition.
      int tpu = NT / U;
      if (tpu > p.q) tpu = p.q;
      const bool act = t < U * tpu;
      const int lu = act ? t % U : 0, sub = act ? t / U : 0;
      const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
          vbuf + e0, (short)0, (int)(((int64_t)p.q * n - e0) * (int64_t)sizeof(C)),
          kRawBufferWord3);
      // worker w's unit lu is at byte (w n + lu W) sizeof(C); a batch's loads
      // are tpu n sizeof(C) bytes apart, and those of workers past the last
      // fall beyond the resource
      const int wstride = (int)((int64_t)tpu * n * (int64_t)sizeof(C));
      C acc[W];
#pragma unroll
      for (int e = 0; e < W; ++e) acc[e] = 0;
      if (act) {
        for (int w0 = sub; w0 < p.q; w0 += kAvgDepth * tpu) {
          const int voff = (int)(((int64_t)w0 * n + lu * W) * (int64_t)sizeof(C));
          C vv[kAvgDepth][W];
#pragma unroll
          for (int u = 0; u < kAvgDepth; ++u) load_units<C, W>(r, voff + u * wstride, vv[u]);
          // a worker past the last adds +0, which leaves a sum started at +0
          // unchanged
#pragma unroll
          for (int u = 0; u < kAvgDepth; ++u) {
#pragma unroll
            for (int e = 0; e < W; ++e) acc[e] += vv[u][e];
          }
        }
#pragma unroll
        for (int e = 0; e < W; ++e) AV[(lu * W + e) * tpu + sub] = acc[e];
      }
      __syncthreads();
      for (int le = t; le < E; le += NT) {
        C sum = 0;
        for (int u = 0; u < tpu; ++u) sum += AV[le * tpu + u];
        const C xn = sum / (C)p.q;
        xb.store(e0 + le, (double)xn);
        if (check) {
          const double dd = (double)xn - p.x_ref[e0 + le];
          err = fma(dd, dd, err);
        }
      }
    }
    if (check) {
      const double s = block_sum(err, RED);
      if (t == 0) store_agent(&p.part[g], s);
    }
    RPROF(5);
    const bool synced = sync_grid(p.bar, epoch, (unsigned)p.G);
    RPROF(6);
    if (!synced) {
      if (t == 0) note_timeout(p.st);
      stopped = true;
      break;
    }
    if (check) {
      double e2 = 0.0;
      for (int gg = 0; gg < p.G; ++gg) e2 += load_agent(&p.part[gg]);
      const bool conv = e2 <= p.st->thresh2;
      const bool div = !isfinite(e2);
      if (conv || div) {
        if (g == 0 && t == 0) {
          p.st->iterations = k + 1;
          p.st->rel2 = e2 / p.st->ref2;
          p.st->status = conv ? 0 : -3;
          p.st->done = 1;
        }
        stopped = true;
        break;
      }
    }
  }
#ifdef RKA_RKAB_PROF
  if (t == 0 && (g == 0 || g == p.G / 2))
    printf("rkab-prof g=%d iters=%lld x_load=%llu projections=%llu publish=%llu drain=%llu "
           "barrier1=%llu average=%llu barrier2=%llu\n",
           g, (long long)kl, (unsigned long long)rp_t[0], (unsigned long long)rp_t[1],
           (unsigned long long)rp_t[2], (unsigned long long)rp_t[3], (unsigned long long)rp_t[4],
           (unsigned long long)rp_t[5], (unsigned long long)rp_t[6]);
#endif
  if (!stopped && g == 0 && t == 0) p.st->iterations = p.k0 + p.K;
}

// Register-tile buckets: 16-byte vecs per thread.  A bucket is offered for a
// storage type only if its kernel compiles without spilling on gfx950.
static int vpt_bucket(int64_t need) {
  static const int b[] = {1, 2, 3, 4, 6, 8, 10, 12, 16, 20};
  for (int v : b)
    if (need <= v) return v;
  return 0;
}

// largest spill-free bucket with v in registers / with v in LDS, per storage
// type and accumulation type
static int vpt_limit_reg(int dtype, int V, int acc) {
  if (V == 1) return dtype == 0 ? 12 : 16;
  if (acc == 1) return dtype == 2 ? 4 : 6;
  return dtype == 2 ? 3 : 6;
}
static int vpt_limit_lds(int dtype, int V, int acc) {
  if (V == 1) return 16;
  if (acc == 1) return dtype == 2 ? 4 : 8;
  return dtype == 0 ? 10 : (dtype == 1 ? 6 : 3);
}
constexpr size_t kMaxLds = 136 * 1024;  // 160 KiB minus the static LDS above (~23 KiB)

bool rkab_plan(const SolveShape& sh, RkabGeom* geo) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  const int64_t nvec = sh.n / V;
  const int vpt = vpt_bucket((nvec + kRkabThreads - 1) / kRkabThreads);
  if (vpt == 0) return false;
  bool vlds = vpt > vpt_limit_reg(sh.dtype, V, sh.acc);
  size_t lds = 0;
  if (vlds) {
    if (vpt > vpt_limit_lds(sh.dtype, V, sh.acc)) return false;
    lds = (size_t)vpt * kRkabThreads * V * (sh.acc == 1 ? sizeof(float) : sizeof(double));
    if (lds > kMaxLds) return false;
  }
  const int target = sh.grid > 0 ? sh.grid : sh.num_cu;
  const int G = sh.q < target ? sh.q : target;
  geo->G = G;
  geo->nt = kRkabThreads;
  geo->vpt = vpt;
  geo->vlds = vlds;
  geo->lds = lds;
  geo->ns = (int)((nvec + G - 1) / G);
  return true;
}

template <typename T, typename C, int V, bool VLDS>
static const void* rkab_fn(int vpt) {
  switch (vpt) {
    case 1: return (const void*)rkab_kernel<T, C, V, 1, VLDS>;
    case 2: return (const void*)rkab_kernel<T, C, V, 2, VLDS>;
    case 3: return (const void*)rkab_kernel<T, C, V, 3, VLDS>;
    case 4: return (const void*)rkab_kernel<T, C, V, 4, VLDS>;
    case 6: return (const void*)rkab_kernel<T, C, V, 6, VLDS>;
    case 8: return (const void*)rkab_kernel<T, C, V, 8, VLDS>;
    case 10: return (const void*)rkab_kernel<T, C, V, 10, VLDS>;
    case 12: return (const void*)rkab_kernel<T, C, V, 12, VLDS>;
    case 16: return (const void*)rkab_kernel<T, C, V, 16, VLDS>;
    default: return (const void*)rkab_kernel<T, C, V, 20, VLDS>;
  }
}

template <typename T, typename C, int V>
static hipError_t launch_rkab_t(const RkabGeom& geo, RkabArgs& a, hipStream_t s) {
  void* args[] = {&a};
  const void* fn =
      geo.vlds ? rkab_fn<T, C, V, true>(geo.vpt) : rkab_fn<T, C, V, false>(geo.vpt);
  if (geo.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.lds);
    if (e != hipSuccess) return e;
  }
  return launch_persistent(fn, dim3(geo.G), dim3(geo.nt), args, (unsigned)geo.lds, s);
}

hipError_t launch_rkab_chunk(const SolveShape& sh, const RkabGeom& geo, const RowRec* rec,
                             int64_t k0, int64_t K, int64_t check_every, void* vbuf,
                             double* part, unsigned* bar, DevStatus* st, hipStream_t s) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  RkabArgs a;
  a.A = sh.A;
  a.lda = sh.lda;
  a.nvec = sh.n / V;
  a.rec = rec;
  a.x = sh.x;
  a.x_ref = sh.x_ref;
  a.alpha = sh.alpha;
  a.q = sh.q;
  a.bs = sh.bs;
  a.G = geo.G;
  a.ns = geo.ns;
  a.k0 = k0;
  a.K = K;
  a.check_every = check_every;
  a.vbuf = vbuf;
  {
    const int64_t csz = sh.acc == 1 ? (int64_t)sizeof(float) : (int64_t)sizeof(double);
    // every offset of the average (workers below q + 8 tpu, tpu <= q) within
    // 31 bits
    a.avg_one_rsrc = (int64_t)9 * sh.q * a.nvec * V * csz < (1ll << 31) ? 1 : 0;
  }
  a.part = part;
  a.bar = bar;
  a.st = st;
  if (geo.G > 1) {
    hipError_t e = launch_zero(bar, kGridBarCounters * sizeof(unsigned), s);
    if (e != hipSuccess) return e;
  }
  if (sh.acc == 1) {
    if (sh.dtype == 1)
      return sh.vec_ok ? launch_rkab_t<float, float, 4>(geo, a, s)
                       : launch_rkab_t<float, float, 1>(geo, a, s);
    return sh.vec_ok ? launch_rkab_t<bf16_t, float, 8>(geo, a, s)
                     : launch_rkab_t<bf16_t, float, 1>(geo, a, s);
  }
  switch (sh.dtype) {
    case 0:
      return sh.vec_ok ? launch_rkab_t<double, double, 2>(geo, a, s)
                       : launch_rkab_t<double, double, 1>(geo, a, s);
    case 1:
      return sh.vec_ok ? launch_rkab_t<float, double, 4>(geo, a, s)
                       : launch_rkab_t<float, double, 1>(geo, a, s);
    default:
      return sh.vec_ok ? launch_rkab_t<bf16_t, double, 8>(geo, a, s)
                       : launch_rkab_t<bf16_t, double, 1>(geo, a, s);
  }
}

}  // namespace rka
