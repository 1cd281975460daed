// rka_sstep.hip -- RKA (Eq. (7), arXiv 2401.17474 Sec. 3.3.1) with several
// iterations per cross-workgroup exchange, for small q.
//
// The column-split kernel (rka_iter.hip) crosses the chip twice per
// iteration: the q partial dot products go out, the q scales come back.  For
// small q that round trip, not the row gather, sets the iteration time -- the
// synchronisation the paper names as the reason RKA parallelizes poorly.  The
// rows of the next p iterations do not depend on x (they are drawn ahead), and
// since x^(k+l+1) - x^(k+l) = (1/q) sum_r s_{l,r} a_{l,r}, the dot product of
// a row a with any iterate of the block is
//
//   <a, x^(k+j)> = <a, x^(k)> + (1/q) sum_{l<j} sum_r s_{l,r} <a, a_{l,r}>.
//
// So one exchange per block of p iterations carries the p q dot products with
// x^(k) and the q^2 p(p-1)/2 inner products between rows of different
// iterations of the block.  Every workgroup then forms the p rounds of scales
// one after the other from those sums (a few hundred flops) and applies the
// p averaged updates to its slice of x in one pass over the rows, which are
// still in registers.  This is the same iteration in exact arithmetic; the
// floating-point scales differ from the one-iteration kernel's by rounding.
//
// A block never runs across a stopping test: blocks end where a test falls,
// and the test at iteration k sees x^(k), as in the one-iteration kernel.
// The arithmetic is FP64 for every storage type (narrow storage widens
// exactly).  All sums have a fixed order: results are bitwise reproducible
// for a given launch geometry.
#include <math.h>

#include <algorithm>

#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// Phase timing of workgroups 0 and G/2 (printed at the end of a launch), for
// builds with RKA_SSTEP_PROF defined only.
#ifdef RKA_SSTEP_PROF
#define SPROF_DECL                              \
  uint64_t sp_t[8] = {0, 0, 0, 0, 0, 0, 0, 0};  \
  int64_t sp_blocks = 0;                        \
  uint64_t sp_last = __builtin_readcyclecounter();
#define SPROF(i)                                   \
  do {                                             \
    const uint64_t sp_now = __builtin_readcyclecounter(); \
    sp_t[i] += sp_now - sp_last;                   \
    sp_last = sp_now;                              \
  } while (0)
#else
#define SPROF_DECL
#define SPROF(i) \
  do {           \
  } while (0)
#endif

struct SstepArgs {
  const void* A;
  int64_t lda, nvec;
  const RowRec* rec;  // K x q row records of the chunk
  double* x;
  const double* x_ref;
  double inv_q;
  int32_t q, p;       // workers, iterations per exchange (at most)
  int32_t bs;         // projections per worker per iteration (1: RKA; > 1: RKAB, p = 1)
  int32_t c;          // RKAB: projections per worker per exchange (sub-block, <= bs)
  int32_t nsv, rg, G;
  int32_t nv_max;     // exchange values of a full block
  int32_t tr;         // lanes per row for the slice sums of the dot products
  int32_t trp;        // lanes per value in the reduce-scatter
  int32_t trs;        // lanes per row for the scale sums (one wave: trs q <= 64)
  int32_t cg;         // lanes (column groups) per 4 x 4 tile of inner products
  int32_t pg_in_s;    // the reduce-scatter gathers into the row-slice buffer
  int32_t pg_len;     // its own buffer's length otherwise
  int32_t nt;         // threads of a workgroup (blockDim.x: a 32-bit argument
                      // keeps its reads off the vector memory counter)
  int64_t k0, K, check_every;
  uint64_t* part;     // G x nv_max tagged slots: per-workgroup partial sums
  uint64_t* red;      // kSumCopies x nv_max tagged slots: the summed values
  DevStatus* st;
};

// Column stride of the row-slice tile for blocks of at most rmax rows: at
// least rmax + 4 (slack for the 4 x 4 inner-product tiles), even (pairs of
// rows stay 16-byte aligned) and not a multiple of 4, so that the lanes of a
// wave, which stage consecutive columns, spread over 8 of the 16 double-word
// LDS banks instead of 2 or 4.
__host__ __device__ constexpr int sstep_rs(int rmax) {
  const int even = (rmax + 5) & ~1;  // rmax + 4 rounded up to even
  return even % 4 == 0 ? even + 2 : even;
}

constexpr int kSMaxRows = 64;      // q * p (RKA)
constexpr int kSMaxRowsB = 256;    // q * bs (RKAB)
constexpr int kSMaxP = 8;
constexpr int kSPoll = 8;          // slots one lane polls in either phase
constexpr int kSBatch = 4;         // poll loads in flight per lane
constexpr int kSThreads = 512;
constexpr size_t kSMaxLds = 150 * 1024;  // of the 160 KiB of a CU

// Exchange values of an RKA block of L iterations: [0, L q) the dot products
// <a_{j,r}, x^(k)> at j q + r; then for every pair l < j (pair index
// j (j-1) / 2 + l) a q x q tile of <a_{j,r}, a_{l,s}> at r q + s; last, the
// squared error of x^(k) against x_ref (0 when the block has no test).
__device__ __forceinline__ int sv_count(int L, int q) {
  return L * q + q * q * (L * (L - 1) / 2) + 1;
}
__device__ __forceinline__ int sv_gram(int L, int q, int j, int l) {
  return L * q + (j * (j - 1) / 2 + l) * q * q;
}
// RKAB (Sec. 3.4.1): worker w projects its bs rows in order on its own
// iterate v_w, which every workgroup keeps for its slice.  An outer iteration
// runs as sub-blocks of c rows per worker; in a sub-block row jb of a worker
// needs its dot product with v_w and <a_{w,jb}, a_{w,jb'}> for jb' < jb only.
// Values of a sub-block of cs rows per worker: [0, q cs) the dot products;
// then worker w's pairs at q cs + w cs (cs-1) / 2 + jb (jb-1) / 2 + jb';
// last, the squared error of x^(k) (first sub-block of a tested iteration).
__device__ __forceinline__ int svb_count(int q, int bs) { return q * bs + q * (bs * (bs - 1) / 2) + 1; }
__device__ __forceinline__ int svb_pair(int q, int bs, int w, int jb, int jb2) {
  return q * bs + w * (bs * (bs - 1) / 2) + jb * (jb - 1) / 2 + jb2;
}

// Orders a wave's LDS writes before its later LDS reads by other lanes of
// the same wave: the LDS serves one wave's accesses in order, the fences keep
// the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// B: the RKAB instance (separate, so that the RKA instance carries none of
// the workers' state in its registers)
template <typename T, int V, int RPT, bool B>
__global__ __launch_bounds__(kSThreads) void rka_sstep_kernel(SstepArgs p) {
  using raw_t = typename Vec<T, V>::raw_t;
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, g = blockIdx.x, NT = p.nt;
  const int q = p.q, nsv = p.nsv, rg = p.rg, G = p.G;
  // B: RKAB, bs > 1 projections per worker with sub-blocks of p.c rows per
  // worker (the host launches bs = 1 as RKA, B false)
  const int bs = B ? p.bs : 1;
  const int W = nsv * V;          // slice width in elements
  const int Rmax = B ? q * p.c : p.p * q;  // rows of the largest block
  const bool active = t < nsv * rg;
  const int j = active ? t % nsv : 0;
  const int rgi = active ? t / nsv : rg;
  const int64_t cv = (int64_t)g * nsv + j;
  const bool colv = active && cv < p.nvec;
  const int64_t cvl = cv < p.nvec ? cv : p.nvec - 1;

  extern __shared__ double lds[];
  double* RED = lds;                      // 16
  double* SC = RED + 16;                  // Rmax        scales of the block
  double* RB = SC + Rmax;                 // Rmax        b_i of the block's rows
  double* RW = RB + Rmax;                 // Rmax        ||a_i||^2
  double* RA = RW + Rmax;                 // Rmax        weights
  double* HV = RA + Rmax;                 // nv_max      summed exchange values
  // row slices of the block, column-major: S[s RS + row], RS = sstep_rs(Rmax);
  // element e of column vector jv of the slice (column jv V + e) sits in slot
  // s = e nsv + jv, so that the lanes of a wave (consecutive jv) stage
  // consecutive slots
  const int RS = sstep_rs(Rmax);
  double* S = HV + ((p.nv_max + 1) & ~1);  // W * RS (16-byte aligned)
  double* P = S + (size_t)W * RS;         // Rmax * nsv  dot partials per vec
  double* U = P + (size_t)Rmax * nsv;     // NT * V      update partials per thread
  double* XS = U + (size_t)NT * V;        // W           new slice of x
  double* UP = XS + W;                    // max(NT, W)  partial column sums of the update
  double* E = UP + (NT > W ? NT : W);     // nsv         error partials
  // G * ceil(nv / G) gathered partials of the reduce-scatter: in the row
  // slices (free by then) when they are large enough, else after E
  double* PG = p.pg_in_s ? S : E + nsv;
  // RKAB: the workers' iterates for this slice, q x W (after PG); unused
  // (pointed at XS) for RKA
  double* VW = B ? E + nsv + (p.pg_in_s ? 0 : p.pg_len) : XS;
  const int NE = W;
  const int NP = NT / NE > 1 ? NT / NE : 1;

  double xv[V];
#pragma unroll
  for (int e = 0; e < V; ++e) xv[e] = colv ? p.x[cv * V + e] : 0.0;

  // length of the block that starts at chunk iteration kl: at most p, not past
  // the chunk, and ending where a stopping test falls
  auto block_len = [&](int64_t kl) -> int {
    int64_t L = p.K - kl;
    if (L > p.p) L = p.p;
    if (p.check_every > 0) {
      const int64_t k = p.k0 + kl;
      const int64_t nxt = (k / p.check_every + 1) * p.check_every;
      if (nxt - k < L) L = nxt - k;
    }
    return (int)L;
  };
  // RKAB sub-blocks: sub-block sb of an outer iteration holds rows
  // sb c .. sb c + cs - 1 of every worker (block row br = w cs + jj)
  const int cblk = B ? p.c : 1;
  const int nsub = (bs + cblk - 1) / cblk;
  auto sub_len = [&](int sb) { return bs - sb * cblk < cblk ? bs - sb * cblk : cblk; };
  auto block_rows = [&](int sb, int L) { return B ? q * sub_len(sb) : L * q; };
  auto rec_index = [&](int64_t kl, int sb, int br) -> int64_t {
    if (!B) return kl * q + br;
    const int cs = sub_len(sb), w = br / cs;
    return (kl * q + w) * (int64_t)bs + sb * cblk + (br - w * cs);
  };
  // the block after (kl, sb, L): the next sub-block, or the next iteration
  auto advance = [&](int64_t& kl2, int& sb2, int& L2) {
    if (B) {
      if (++sb2 == nsub) {
        sb2 = 0;
        ++kl2;
      }
      L2 = 1;
    } else {
      kl2 += L2;
      L2 = kl2 < p.K ? block_len(kl2) : L2;
    }
  };
  // row indices of a block (rows clamped to the block: masked later)
  auto load_rows = [&](int64_t kl2, int sb2, int L2, int* rows) {
    const int R2 = block_rows(sb2, L2);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int br = rgi + rg * i;
      rows[i] = (int)p.rec[rec_index(kl2, sb2, br < R2 ? br : R2 - 1)].row;
    }
  };

  raw_t a[RPT], an[RPT];
  int rows_n[RPT];
  double mb = 0.0, mw = 1.0, ma = 0.0;  // record of block row t (t < R)
  int64_t kl = 0;
  int sb = 0;
  int L = B ? 1 : block_len(0);
  {
    int rows0[RPT];
    load_rows(0, 0, L, rows0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) a[i] = load_raw<T, V>(A + (int64_t)rows0[i] * p.lda + cvl * V);
    if (t < block_rows(0, L)) {
      const RowRec r = p.rec[rec_index(0, 0, t)];
      mb = r.b;
      mw = r.wn;
      ma = r.alpha;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) rows_n[i] = rows0[i];
    int64_t k1 = 0;
    int s1 = 0, L1 = L;
    advance(k1, s1, L1);
    if (k1 < p.K) load_rows(k1, s1, L1, rows_n);
  }
  // RKAB: every worker's iterate starts each outer iteration at x
  if (B) {
    if (active && rgi == 0) {
#pragma unroll
      for (int e = 0; e < V; ++e) XS[j * V + e] = xv[e];
    }
    __syncthreads();
    for (int Lx = t; Lx < q * W; Lx += NT) VW[Lx] = XS[Lx % W];
    __syncthreads();
  }

  // Poll `total` tagged slots, slot idx(L) for L = t + NT s (at most kSPoll
  // per lane), until every tag matches, and store the values to dst[L].  A
  // sweep issues a lane's loads kSBatch at a time before it waits for them;
  // slots already read, and lanes past the end, load at `oob`, out of the
  // buffer's range (zero, no memory access).  False if the wait gave up (in
  // every thread).
  auto gather = [&](const TagSlots& sl, int oob, int total, uint32_t tg, auto idx,
                    double* dst) -> bool {
    const int ns = (total + NT - 1) / NT;  // loads per lane and sweep, uniform
    uint32_t need = 0;                     // bit s: slot t + NT s still to read
#pragma unroll
    for (int s = 0; s < kSPoll; ++s)
      if (t + NT * s < total) need |= 1u << s;
    for (unsigned spins = 0;; ++spins) {
#pragma unroll
      for (int s0 = 0; s0 < kSPoll; s0 += kSBatch) {
        if (s0 < ns) {
          uint64_t lo[kSBatch], hi[kSBatch];
#pragma unroll
          for (int s = 0; s < kSBatch; ++s) {
            lo[s] = hi[s] = 0;
            if (s0 + s < ns) {
              // recomputed every sweep rather than held in registers
              int Lx = t + NT * (s0 + s);
              __asm__ volatile("" : "+v"(Lx));
              sl.fetch16((need >> (s0 + s)) & 1u ? (int)idx(Lx) : oob, lo[s], hi[s]);
            }
          }
#pragma unroll
          for (int s = 0; s < kSBatch; ++s) {
            double v;
            if (s0 + s < ns && ((need >> (s0 + s)) & 1u) && TagSlots::decode(lo[s], hi[s], tg, v)) {
              dst[t + NT * (s0 + s)] = v;
              need &= ~(1u << (s0 + s));
            }
          }
        }
      }
      if (__syncthreads_and(need == 0)) return true;
      if (spins >= kSpinLimit) return false;
      __builtin_amdgcn_s_sleep(1);
    }
  };

  bool stopped = false;
  SPROF_DECL
  while (kl < p.K) {
    const int64_t k = p.k0 + kl;
    const int cs = B ? sub_len(sb) : 1;  // rows per worker in this sub-block
    const int R = block_rows(sb, L);
    const int nv = B ? svb_count(q, cs) : sv_count(L, q);
    const bool check = sb == 0 && p.check_every > 0 && k > 0 && (k % p.check_every) == 0;
    // one tag per exchange of the solve: iteration, then sub-block
    const uint32_t tag = (uint32_t)(k * nsub + sb + 1);
    const TagSlots part(p.part, (int64_t)G * p.nv_max);
    const TagSlots red(p.red, (int64_t)kSumCopies * p.nv_max);

    if (t < R) {
      RB[t] = mb;
      RW[t] = mw;
      RA[t] = ma;
    }
    // stage the slices of the block's rows and form their dot products with x
    // (RKAB: with the iterate of the row's worker)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int br = rgi + rg * i;
      const double* vw = VW + (size_t)((B && br < R) ? br / cs : 0) * W + j * V;
      double s = 0.0;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double v = colv ? raw_elem<T, V>(a[i], e) : 0.0;
        s = fma(v, B ? vw[e] : xv[e], s);
        if (active && br < R) S[(size_t)(e * nsv + j) * RS + br] = v;
      }
      if (active && br < R) P[br * nsv + j] = s;
    }
    if (check && active && rgi == 0) {
      double s = 0.0;
      if (colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const double d = xv[e] - p.x_ref[cv * V + e];
          s = fma(d, d, s);
        }
      }
      E[j] = s;
    }
    __syncthreads();
    SPROF(0);
    // (1) dot products: a team of tr lanes per row, fixed order
    {
      const int TR = p.tr, team = t / TR, u = t & (TR - 1), nteams = NT / TR;
      for (int r0 = 0; r0 < R; r0 += nteams) {
        const int br = r0 + team;
        double d = 0.0;
        if (br < R)
          for (int jj = u; jj < nsv; jj += TR) d += P[br * nsv + jj];
        d = team_sum(d, TR);
        if (u == 0 && br < R) HV[br] = d;
      }
    }
    // (2) inner products between rows of different iterations: 4 x 4 tiles,
    // cg lanes per tile over consecutive column ranges, folded in lane order
    if (!B) {
      const int q4 = (q + 3) / 4;
      const int ntile = (L * (L - 1) / 2) * q4 * q4;
      const int CG = p.cg, per = NT / CG;
      const int cu = t & (CG - 1);
      const int c0 = cu * W / CG, c1 = (cu + 1) * W / CG;
      for (int tb = 0; tb < ntile; tb += per) {
        const int tile = tb + t / CG;
        const bool tin = tile < ntile;
        int jj = 1, ll = 0, rb = 0, sb = 0;
        if (tin) {
          int pi = tile / (q4 * q4);
          const int rem = tile % (q4 * q4);
          rb = (rem / q4) * 4;
          sb = (rem % q4) * 4;
          while (pi >= jj) {  // pair index -> (jj, ll), ll < jj
            pi -= jj;
            ++jj;
          }
          ll = pi;
        }
        double acc[16];  // acc[4 u1 + u2] = <row rb + u1, row sb + u2> over the range
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        if (tin) {
          // rows jj q + rb .. + 3 and ll q + sb .. + 3 are contiguous in a
          // column of S (past the block's rows the values are unused)
          const double* Sa = S + jj * q + rb;
          const double* Sb = S + ll * q + sb;
#pragma unroll 2
          for (int c = c0; c < c1; ++c) {
            double va[4], vb[4];
            if (q % 2 == 0) {  // 16-byte aligned pairs
              const double2 a01 = *(const double2*)(Sa + (size_t)c * RS);
              const double2 a23 = *(const double2*)(Sa + (size_t)c * RS + 2);
              const double2 b01 = *(const double2*)(Sb + (size_t)c * RS);
              const double2 b23 = *(const double2*)(Sb + (size_t)c * RS + 2);
              va[0] = a01.x, va[1] = a01.y, va[2] = a23.x, va[3] = a23.y;
              vb[0] = b01.x, vb[1] = b01.y, vb[2] = b23.x, vb[3] = b23.y;
            } else {
#pragma unroll
              for (int u1 = 0; u1 < 4; ++u1) {
                va[u1] = Sa[(size_t)c * RS + u1];
                vb[u1] = Sb[(size_t)c * RS + u1];
              }
            }
#pragma unroll
            for (int u1 = 0; u1 < 4; ++u1)
#pragma unroll
              for (int u2 = 0; u2 < 4; ++u2) acc[4 * u1 + u2] = fma(va[u1], vb[u2], acc[4 * u1 + u2]);
          }
        }
        team_sum_n(acc, CG);
        if (tin && cu == 0) {
          const int base = sv_gram(L, q, jj, ll);
#pragma unroll
          for (int u1 = 0; u1 < 4; ++u1)
#pragma unroll
            for (int u2 = 0; u2 < 4; ++u2)
              if (rb + u1 < q && sb + u2 < q) HV[base + (rb + u1) * q + sb + u2] = acc[4 * u1 + u2];
        }
      }
    } else {
      // RKAB: the pairs within each worker's rows, 4 x 4 tiles (ta, tb), tb <= ta
      const int b4 = (cs + 3) / 4, tpw = b4 * (b4 + 1) / 2;
      const int ntile = q * tpw;
      const int CG = p.cg, per = NT / CG;
      const int cu = t & (CG - 1);
      const int c0 = cu * W / CG, c1 = (cu + 1) * W / CG;
      for (int tb0 = 0; tb0 < ntile; tb0 += per) {
        const int tile = tb0 + t / CG;
        const bool tin = tile < ntile;
        int w = 0, ta = 0, tb = 0;
        if (tin) {
          w = tile / tpw;
          int rem = tile - w * tpw;
          while (rem >= ta + 1) {
            rem -= ta + 1;
            ++ta;
          }
          tb = rem;
        }
        double acc[16];  // acc[4 u1 + u2] = <row 4 ta + u1, row 4 tb + u2> of worker w
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u] = 0.0;
        if (tin) {
          const double* Sa = S + w * cs + 4 * ta;
          const double* Sb = S + w * cs + 4 * tb;
#pragma unroll 2
          for (int c = c0; c < c1; ++c) {
            double va[4], vb[4];
            if (cs % 2 == 0) {  // 16-byte aligned pairs
              const double2 a01 = *(const double2*)(Sa + (size_t)c * RS);
              const double2 a23 = *(const double2*)(Sa + (size_t)c * RS + 2);
              const double2 b01 = *(const double2*)(Sb + (size_t)c * RS);
              const double2 b23 = *(const double2*)(Sb + (size_t)c * RS + 2);
              va[0] = a01.x, va[1] = a01.y, va[2] = a23.x, va[3] = a23.y;
              vb[0] = b01.x, vb[1] = b01.y, vb[2] = b23.x, vb[3] = b23.y;
            } else {
#pragma unroll
              for (int u1 = 0; u1 < 4; ++u1) {
                va[u1] = Sa[(size_t)c * RS + u1];
                vb[u1] = Sb[(size_t)c * RS + u1];
              }
            }
#pragma unroll
            for (int u1 = 0; u1 < 4; ++u1)
#pragma unroll
              for (int u2 = 0; u2 < 4; ++u2) acc[4 * u1 + u2] = fma(va[u1], vb[u2], acc[4 * u1 + u2]);
          }
        }
        team_sum_n(acc, CG);
        if (tin && cu == 0) {
#pragma unroll
          for (int u1 = 0; u1 < 4; ++u1)
#pragma unroll
            for (int u2 = 0; u2 < 4; ++u2) {
              const int jb = 4 * ta + u1, jb2 = 4 * tb + u2;
              if (jb < cs && jb2 < jb) HV[svb_pair(q, cs, w, jb, jb2)] = acc[4 * u1 + u2];
            }
        }
      }
    }
    // (3) the error partial of this slice (0 without a test)
    if (t < kWave) {
      double s = 0.0;
      if (check)
        for (int jj = t; jj < nsv; jj += kWave) s += E[jj];
      s = wave_sum(s);
      if (t == 0) HV[nv - 1] = s;
    }
    SPROF(1);

    // the next block's rows and records (independent of x) are requested now.
    // The exchange's first poll waits for them (the vector memory counter
    // drains in order), but they overlap the other workgroups' arrival;
    // issuing them after the exchange instead is slower (80000 x 10000, q 16).
    int64_t kn = kl;
    int sbn = sb, Ln = L;
    advance(kn, sbn, Ln);
#pragma unroll
    for (int i = 0; i < RPT; ++i) an[i] = load_raw<T, V>(A + (int64_t)rows_n[i] * p.lda + cvl * V);
    if (kn < p.K && t < block_rows(sbn, Ln)) {
      const RowRec r = p.rec[rec_index(kn, sbn, t)];
      mb = r.b;
      mw = r.wn;
      ma = r.alpha;
    }
    if (kn < p.K) {
      int64_t knn = kn;
      int sbnn = sbn, Lnn = Ln;
      advance(knn, sbnn, Lnn);
      if (knn < p.K) load_rows(knn, sbnn, Lnn, rows_n);
    }

    // the workgroup's nv partial sums leave in one coalesced pass (a fixed
    // number of stores per lane: an index past the slots drops the store).
    // Value-major slots (a value's G partials contiguous, as in kernel 4)
    // measured slower here: the scattered stores cost more than the polls
    // save (80000 x 10000 FP64, RKAB q = 16, bs = 10: 22.3 against 20.5 us
    // per outer iteration).
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kSPoll; ++s) {
      const int v = t + NT * s;
      const int64_t slot = v < nv ? (int64_t)g * p.nv_max + v : (int64_t)G * p.nv_max;
      part.put16(slot, HV[v < nv ? v : 0], tag);
    }
    SPROF(2);
    bool ok = true;
    // phase 1: workgroup g sums the values [g C, g C + C) of every
    // workgroup's partials (contiguous reads), gathering them in LDS first
    {
      const int C = (nv + G - 1) / G;
      const int v0 = g * C;
      const int cnt = nv - v0 < C ? (nv - v0 > 0 ? nv - v0 : 0) : C;
      ok = gather(part, G * p.nv_max, G * cnt, tag,
                  [&](int Lx) {
                    const int gg = Lx / cnt, c = Lx - gg * cnt;
                    return gg * p.nv_max + v0 + c;
                  },
                  PG);
      // value c: a team of trp lanes, lane u adding workgroups u, u + trp, ...
      // in order, then the team fold (one round: cnt <= NT / trp)
      const int TR = p.trp, team = t / TR, u = t & (TR - 1);
      double sum = 0.0;
      if (team < cnt)
        for (int gg = u; gg < G; gg += TR) sum += PG[gg * cnt + team];
      sum = team_sum(sum, TR);  // in every lane of the team
      if (ok && team < cnt)
        for (int c = u; c < kSumCopies; c += TR) red.put16(c * p.nv_max + v0 + team, sum, tag);
    }
    SPROF(3);
    // phase 2: every workgroup reads all nv sums (from its copy)
    if (__syncthreads_and(ok)) {
      const int cpo = (g % kSumCopies) * p.nv_max;
      ok = gather(red, kSumCopies * p.nv_max, nv, tag, [&](int Lx) { return cpo + Lx; }, HV);
    }
    if (!__syncthreads_and(ok)) {
      if (t == 0) note_timeout(p.st);
      stopped = true;
      break;
    }
    SPROF(4);
    if (check) {
      const double e2 = HV[nv - 1];
      const bool conv = e2 <= p.st->thresh2;
      const bool div = !isfinite(e2);
      if (conv || div) {
        if (g == 0 && t == 0) {
          p.st->iterations = k;
          p.st->rel2 = e2 / p.st->ref2;
          p.st->status = conv ? 0 : -3;
          p.st->done = 1;
        }
        stopped = true;
        break;
      }
    }
    // the scales, one iteration of the block after the other:
    // D_{j,r} = <a_{j,r}, x^(k)> + (1/q) sum_{l<j} sum_s s_{l,s} <a_{j,r}, a_{l,s}>
    // (RKAB: one worker's projections after the other, weight 1:
    //  D_{w,jb} = <a_{w,jb}, v_w> + sum_{jb'<jb} s_{w,jb'} <a_{w,jb}, a_{w,jb'}>).
    // The rounds are short and dependent, so one wave runs them (teams of trs
    // lanes per row, trs q <= 64) with no workgroup barrier between rounds;
    // one barrier hands the scales to the other waves.
    if (t < kWave) {
      const int TR = p.trs, team = t / TR, u = t & (TR - 1), nteams = kWave / TR;
      if (!B) {
        for (int jj = 0; jj < L; ++jj) {
          for (int r0 = 0; r0 < q; r0 += nteams) {
            const int r = r0 + team;
            double acc = 0.0;
            if (r < q)
              for (int l = 0; l < jj; ++l) {
                const double* Gr = HV + sv_gram(L, q, jj, l) + r * q;
                const double* Sl = SC + l * q;
                for (int s = u; s < q; s += TR) acc = fma(Sl[s], Gr[s], acc);
              }
            acc = team_sum(acc, TR);
            if (u == 0 && r < q) {
              const int br = jj * q + r;
              const double D = HV[br] + p.inv_q * acc;
              SC[br] = RA[br] * (RB[br] - D) / RW[br];
            }
          }
          wave_lds_sync();
        }
      } else {
        for (int jb = 0; jb < cs; ++jb) {
          for (int w0 = 0; w0 < q; w0 += nteams) {
            const int w = w0 + team;
            double acc = 0.0;
            if (w < q)
              for (int f = u; f < jb; f += TR)
                acc = fma(SC[w * cs + f], HV[svb_pair(q, cs, w, jb, f)], acc);
            acc = team_sum(acc, TR);
            if (u == 0 && w < q) {
              const int br = w * cs + jb;
              const double D = HV[br] + acc;
              SC[br] = RA[br] * (RB[br] - D) / RW[br];
            }
          }
          wave_lds_sync();
        }
      }
    }
    __syncthreads();
    SPROF(5);
    if (B) {
      // each worker's slice: v_w += sum_jj s_{w,jj} A[i_{w,jj}, slice], rows in order
      for (int Lx = t; Lx < q * W; Lx += NT) {
        const int w = Lx / W, c = Lx - w * W;
        double acc = 0.0;
        const double* Sc = S + (size_t)((c % V) * nsv + c / V) * RS + w * cs;
        for (int jj = 0; jj < cs; ++jj) acc = fma(SC[w * cs + jj], Sc[jj], acc);
        VW[Lx] += acc;
      }
      __syncthreads();
      if (sb == nsub - 1) {
        // end of the outer iteration: x = (1/q) sum_w v_w, and every v_w restarts at x
        for (int c = t; c < W; c += NT) {
          double acc = 0.0;
          for (int w = 0; w < q; ++w) acc += VW[w * W + c];
          XS[c] = acc / (double)q;
        }
        __syncthreads();
        for (int Lx = t; Lx < q * W; Lx += NT) VW[Lx] = XS[Lx % W];
        if (colv) {
#pragma unroll
          for (int e = 0; e < V; ++e) xv[e] = XS[j * V + e];
        }
        __syncthreads();
      }
    } else {
      // x_slice += (1/q) sum over the block's rows of s * A[i, slice]
      double uu[V];
#pragma unroll
      for (int e = 0; e < V; ++e) uu[e] = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int br = rgi + rg * i;
        const double s = (colv && br < R) ? SC[br < R ? br : 0] : 0.0;
#pragma unroll
        for (int e = 0; e < V; ++e) uu[e] = fma(s, raw_elem<T, V>(a[i], e), uu[e]);
      }
      if (active) {
#pragma unroll
        for (int e = 0; e < V; ++e) U[t * V + e] = uu[e];
      }
      __syncthreads();
      for (int Lx = t; Lx < NE * NP; Lx += NT) {
        const int je = Lx % NE, pp = Lx / NE;
        const int jj = je / V, e = je % V;
        const int g0 = pp * rg / NP, g1 = (pp + 1) * rg / NP;
        double acc = 0.0;
        for (int gg = g0; gg < g1; ++gg) acc += U[(gg * nsv + jj) * V + e];
        UP[Lx] = acc;
      }
      __syncthreads();
      if (colv && rgi == 0) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          double acc = 0.0;
          for (int pp = 0; pp < NP; ++pp) acc += UP[pp * NE + j * V + e];
          xv[e] = fma(acc, p.inv_q, xv[e]);
          XS[j * V + e] = xv[e];
        }
      }
      __syncthreads();
      if (colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) xv[e] = XS[j * V + e];
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) a[i] = an[i];
    kl = kn;
    sb = sbn;
    L = Ln;
    SPROF(6);
#ifdef RKA_SSTEP_PROF
    ++sp_blocks;
#endif
  }
#ifdef RKA_SSTEP_PROF
  if (t == 0 && (g == 0 || g == G / 2))
    printf("sstep-prof g=%d blocks=%lld stage=%llu dots+gram+put=%llu prefetch=%llu phase1=%llu "
           "phase2=%llu scales=%llu update=%llu\n",
           g, (long long)sp_blocks, (unsigned long long)sp_t[0], (unsigned long long)sp_t[1],
           (unsigned long long)sp_t[2], (unsigned long long)sp_t[3], (unsigned long long)sp_t[4],
           (unsigned long long)sp_t[5], (unsigned long long)sp_t[6]);
#endif
  if (colv && rgi == 0) {
#pragma unroll
    for (int e = 0; e < V; ++e) p.x[cv * V + e] = xv[e];
  }
  if (!stopped && g == 0 && t == 0) p.st->iterations = p.k0 + p.K;
}

static int sstep_bucket(int need) {
  if (need <= 1) return 1;
  if (need <= 2) return 2;
  if (need <= 4) return 4;
  if (need <= 8) return 8;
  return 0;
}

static int pow2_floor_cap(int64_t cap, int limit) {
  int v = 1;
  while ((int64_t)v * 2 <= cap && v * 2 <= limit) v *= 2;
  return v;
}

static bool sstep_plan_at(const SolveShape& sh, int p_req, int c, RkaSstepGeom* geo);

static bool sstep_plan_c(const SolveShape& sh, int p_req, int c, RkaSstepGeom* geo) {
  if (sstep_plan_at(sh, p_req, c, geo)) return true;
  if (sh.grid > 0) return false;
  SolveShape wide = sh;  // slices too wide for the tile at half the CUs
  wide.grid = sh.num_cu;
  return sstep_plan_at(wide, p_req, c, geo);
}

bool rka_sstep_plan(const SolveShape& sh, int p_req, RkaSstepGeom* geo) {
  if (sh.bs <= 1) return sstep_plan_c(sh, p_req, 1, geo);
  // RKAB: the longest sub-block that fits (the whole outer iteration if it can)
  int c = (int)std::min<int64_t>(sh.bs, kSMaxRowsB / sh.q);
  for (; c >= 1; --c)
    if (sstep_plan_c(sh, p_req, c, geo)) return true;
  return false;
}

static bool sstep_plan_at(const SolveShape& sh, int p_req, int c, RkaSstepGeom* geo) {
  if (sh.acc != 0 || sh.q < 1) return false;
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  const int64_t nvec = sh.n / V;
  const int bs = sh.bs;
  int pp;
  if (bs > 1) {  // RKAB: sub-blocks of c projections per worker
    if (p_req > 1 || c < 1 || c > bs || (int64_t)sh.q * c > kSMaxRowsB) return false;
    pp = 1;
  } else {
    int pmax = kSMaxRows / sh.q;
    if (pmax > kSMaxP) pmax = kSMaxP;
    pp = p_req > 0 ? p_req : pmax;
    if (pp < 2 || pp > pmax) return false;
  }
  // half the CUs by default: a block's exchange is large enough that fewer,
  // wider slices win (measured at 80000 x 10000 FP64, q = 16 and 8)
  const int target = sh.grid > 0 ? sh.grid : std::max(2, sh.num_cu / 2);
  const int64_t g0 = nvec < target ? nvec : target;
  const int nsv = (int)((nvec + g0 - 1) / g0);
  const int G = (int)((nvec + nsv - 1) / nsv);
  if (nsv > kSThreads || G < 2) return false;
  const int R = bs > 1 ? sh.q * c : pp * sh.q;
  int rg = kSThreads / nsv;
  if (rg > R) rg = R;
  const int rpt = sstep_bucket((R + rg - 1) / rg);
  // largest spill-free tile per storage type
  const int rpt_max = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  if (rpt == 0 || rpt > rpt_max) return false;
  const int W = nsv * V;
  const int nv = bs > 1 ? sh.q * c + sh.q * (c * (c - 1) / 2) + 1
                       : pp * sh.q + sh.q * sh.q * (pp * (pp - 1) / 2) + 1;
  // threads: the row tile, at least 256, more if the exchange needs them:
  // the reduce-scatter gathers G x C partials (C = ceil(nv / G) values per
  // workgroup) with at most kSPoll slots per lane, the all-gather nv sums
  const int64_t cmax = (nv + G - 1) / G;
  const int64_t gathered = (int64_t)G * cmax;
  int nt = ((nsv * rg + kWave - 1) / kWave) * kWave;
  if (nt < 256) nt = 256;
  auto fits = [&](int th) {
    return (gathered + th - 1) / th <= kSPoll && (nv + th - 1) / th <= kSPoll && cmax <= th;
  };
  if (!fits(nt)) nt = kSThreads;
  if (!fits(nt)) return false;
  const int trp = pow2_floor_cap(nt / cmax, kWave);
  // RKAB reads the row slices after the exchange (the workers' updates), so
  // its reduce-scatter gathers into a buffer of its own
  const bool pg_in_s = bs == 1 && (int64_t)sstep_rs(R) * W >= gathered;
  const size_t lds = sizeof(double) * (16 + 4 * (size_t)R + ((nv + 1) & ~1) + (size_t)sstep_rs(R) * W +
                                       (size_t)R * nsv +
                                       (size_t)nt * V + W + std::max(nt, W) + nsv +
                                       (pg_in_s ? 0 : (size_t)gathered) +
                                       (bs > 1 ? (size_t)sh.q * W : 0));
  if (lds > kSMaxLds) return false;
  const int q4 = (sh.q + 3) / 4, b4 = (c + 3) / 4;
  const int64_t ntile = bs > 1 ? (int64_t)sh.q * (b4 * (b4 + 1) / 2)
                               : (int64_t)(pp * (pp - 1) / 2) * q4 * q4;
  geo->G = G;
  geo->nsv = nsv;
  geo->rg = rg;
  geo->nt = nt;
  geo->rpt = rpt;
  geo->p = pp;
  geo->bs = bs;
  geo->c = bs > 1 ? c : 1;
  geo->nv = nv;
  geo->lds = lds;
  geo->tr = pow2_floor_cap(std::min<int64_t>(nt / R, nsv), kWave);
  geo->trp = trp;
  geo->pg_in_s = pg_in_s ? 1 : 0;
  geo->pg_len = pg_in_s ? 0 : (int)gathered;
  geo->trs = pow2_floor_cap(kWave / sh.q, kWave);
  geo->cg = pow2_floor_cap(std::min<int64_t>(ntile > 0 ? nt / ntile : nt, W), 16);
  return true;
}

template <typename T, int V, bool B>
static const void* sstep_fn(int rpt) {
  // tiles instantiated only where they do not spill (rka_sstep_plan keeps to them)
  const void* fn = rpt == 1 ? (const void*)rka_sstep_kernel<T, V, 1, B>
                            : (const void*)rka_sstep_kernel<T, V, 2, B>;
  if constexpr (sizeof(T) >= 4) {
    if (rpt == 4) fn = (const void*)rka_sstep_kernel<T, V, 4, B>;
  }
  if constexpr (sizeof(T) == 8) {
    if (rpt == 8) fn = (const void*)rka_sstep_kernel<T, V, 8, B>;
  }
  return fn;
}

template <typename T, int V>
static hipError_t launch_sstep_t(const RkaSstepGeom& geo, SstepArgs& a, hipStream_t s) {
  void* args[] = {&a};
  const void* fn = geo.bs > 1 ? sstep_fn<T, V, true>(geo.rpt) : sstep_fn<T, V, false>(geo.rpt);
  size_t lds = geo.lds;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return launch_persistent(fn, dim3(geo.G), dim3(geo.nt), args, (unsigned)lds, s);
}

hipError_t launch_sstep_chunk(const SolveShape& sh, const RkaSstepGeom& geo, const RowRec* rec,
                              int64_t k0, int64_t K, int64_t check_every, uint64_t* part,
                              uint64_t* red, DevStatus* st, hipStream_t s) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  SstepArgs a;
  a.A = sh.A;
  a.lda = sh.lda;
  a.nvec = sh.n / V;
  a.rec = rec;
  a.x = sh.x;
  a.x_ref = sh.x_ref;
  a.inv_q = 1.0 / (double)sh.q;
  a.q = sh.q;
  a.p = geo.p;
  a.bs = geo.bs;
  a.c = geo.c;
  a.nsv = geo.nsv;
  a.rg = geo.rg;
  a.G = geo.G;
  a.nv_max = geo.nv;
  a.tr = geo.tr;
  a.trp = geo.trp;
  a.pg_in_s = geo.pg_in_s;
  a.pg_len = geo.pg_len;
  a.trs = geo.trs;
  a.cg = geo.cg;
  a.nt = geo.nt;
  a.k0 = k0;
  a.K = K;
  a.check_every = check_every;
  a.part = part;
  a.red = red;
  a.st = st;
  switch (sh.dtype) {
    case 0:
      return sh.vec_ok ? launch_sstep_t<double, 2>(geo, a, s) : launch_sstep_t<double, 1>(geo, a, s);
    case 1:
      return sh.vec_ok ? launch_sstep_t<float, 4>(geo, a, s) : launch_sstep_t<float, 1>(geo, a, s);
    default:
      return sh.vec_ok ? launch_sstep_t<bf16_t, 8>(geo, a, s) : launch_sstep_t<bf16_t, 1>(geo, a, s);
  }
}

}  // namespace rka
