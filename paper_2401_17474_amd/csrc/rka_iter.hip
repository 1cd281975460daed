// rka_iter.hip -- RKA (Eq. (7), arXiv 2401.17474 Sec. 3.3.1) on gfx950, and
// the stopping measures shared by both solvers.
//
// RKA is an HBM-bound random row gather: a projection reads one row once and
// does two flops per element with it (dot product, then update).  The kernel
// is persistent and cooperatively launched, so one launch runs a whole chunk
// of iterations with grid barriers in place of kernel boundaries.
//
// Column-split: workgroup g owns a fixed slice of the columns of x and keeps
// that slice of x on chip for the whole chunk.  Per iteration it gathers the
// slice of each of the q sampled rows into registers, forms q partial dot
// products, and exchanges only those partials (q doubles per workgroup)
// through a two-barrier all-reduce; the scales then update the slice of x
// from the row data still in registers.  Each element of A is read from HBM
// exactly once per iteration and x never leaves the chip.  This replaces the
// serial critical section of Algorithm 1 (and the averaging alternatives
// discussed with it) with a fixed-order, atomic-free reduction.
//
// Sums are always taken in a fixed order, so a given launch geometry gives
// bitwise-reproducible results.
#include <math.h>

#include <algorithm>

#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// ===========================================================================
// RKA, column-split persistent kernel.
// ===========================================================================
struct RkaColArgs {
  const void* A;
  int64_t lda, nvec;
  const RowRec* rec;  // K x q row records of the chunk
  double* x;
  const double* x_ref;
  double alpha, inv_q;
  int32_t q, nsv, rg, G;
  int32_t gather;     // 1: one-barrier all-gather of the partials; 0: two barriers
  int32_t tr;         // lanes that sum one row's nsv slice partials (power of two <= 64)
  int32_t tr_g;       // lanes that sum one row's G gathered partials (all-gather only)
  int64_t k0, K, check_every;
  uint64_t* part;  // tagged slots: gather 2 x G x (q+1) (by iteration parity); else G x (q+1)
  uint64_t* scal;  // tagged slots: kSumCopies x (q+1) scales (two-phase exchange)
  DevStatus* st;
};

constexpr int kPollMax = 4;  // tagged slots one thread polls per exchange

constexpr int kMaxColThreads = 512;

// C is the accumulation type: double, or float for narrow storage (the
// inner solves of the precision form).  With C = float the slice of x, the
// products and the in-workgroup sums are FP32; the per-workgroup partial
// sums are combined across workgroups in FP64 and rounded once.
template <typename T, typename C, int V, int RPT, bool GATHER>
__global__ __launch_bounds__(kMaxColThreads) void rka_col_kernel(RkaColArgs p) {
  using raw_t = typename Vec<T, V>::raw_t;
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, g = blockIdx.x, NT = blockDim.x;
  const int q = p.q, nsv = p.nsv, rg = p.rg, G = p.G;
  const bool active = t < nsv * rg;
  const int j = active ? t % nsv : 0;
  const int rgi = active ? t / nsv : rg;
  const int64_t cv = (int64_t)g * nsv + j;
  const bool colv = active && cv < p.nvec;
  const bool gather = GATHER && G > 1;

  extern __shared__ double lds[];
  double* E = lds;                    // nsv          error partials
  double* RED = E + nsv;              // 16           block_sum scratch
  double* SC = RED + 16;              // q + 1        dot totals, then scales
  double* PG = SC + q + 1;            // G * (q+1)    gathered partials (gather only)
  C* P = (C*)(PG + (gather ? (size_t)G * (q + 1) : 0));  // q * nsv   row partials per vec
  C* U = P + (size_t)q * nsv;         // NT * V       update partials per thread
  C* XS = U + (size_t)NT * V;         // nsv * V      new slice of x
  C* UP = XS + (size_t)nsv * V;       // max(NT, nsv*V)  partial column sums of the update
  // the update's column sums over the rg row groups are split into NP parts
  // of consecutive groups (all threads busy even when the slice is narrow)
  const int NE = nsv * V;
  const int NP = NT / NE > 1 ? NT / NE : 1;

  // the scale alpha_w (b_i - <a_i, x>) / ||a_i||^2 in the accumulation type
  // (alpha_w: the weight of the drawing worker, carried by the row record)
  auto scale_of = [&](double ai, double bi, double wi, double D) -> double {
    return (double)((C)ai * ((C)bi - (C)D) / (C)wi);
  };

  C xv[V];
#pragma unroll
  for (int e = 0; e < V; ++e) xv[e] = colv ? (C)p.x[cv * V + e] : (C)0;

  // Loads are unconditional (indices clamped to valid rows/vecs; the surplus
  // entries are masked in the arithmetic): a load under a branch would make
  // the compiler drain every in-flight load where the branches join.
  const int64_t cvl = cv < p.nvec ? cv : p.nvec - 1;
  // the row whose scale this thread forms (first round of its team)
  const int tr_s = G == 1 ? p.tr : (gather ? p.tr_g : 1);
  const int tq = t / tr_s < q ? t / tr_s : q - 1;
  raw_t a[RPT], an[RPT];
  int rows[RPT], rows_n[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = rgi + rg * i;
    rows[i] = (int)p.rec[r < q ? r : q - 1].row;
    a[i] = load_raw<T, V>(A + (int64_t)rows[i] * p.lda + cvl * V);
  }
  // records needed one iteration ahead: the next rows (for the prefetch) and
  // b_i, ||a_i||^2 of row t (used where a workgroup forms every scale itself:
  // one workgroup, or the all-gather)
  double mine_b, mine_w, mine_a;
  auto load_next = [&](int64_t kn, int64_t kc) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = rgi + rg * i;
      rows_n[i] = (int)p.rec[kn * q + (r < q ? r : q - 1)].row;
    }
    mine_b = p.rec[kc * q + tq].b;
    mine_w = p.rec[kc * q + tq].wn;
    mine_a = p.rec[kc * q + tq].alpha;
  };
  load_next(p.K > 1 ? 1 : 0, 0);

  int64_t kl = 0;
  bool stopped = false;
  for (; kl < p.K; ++kl) {
    const int64_t k = p.k0 + kl;
    const bool check = p.check_every > 0 && k > 0 && (k % p.check_every) == 0;
    const int nr = q + (check ? 1 : 0);
    const uint32_t tag = (uint32_t)(k + 1);
    const TagSlots part(p.part + (gather ? (size_t)(kl & 1) * G * (q + 1) * 2 : 0),
                        (int64_t)G * (q + 1));
    // partial dot products of this slice, one per (row, vec)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = rgi + rg * i;
      C s = 0;  // xv is 0 past the last column
#pragma unroll
      for (int e = 0; e < V; ++e) s = fma(raw_elem_c<C, T, V>(a[i], e), xv[e], s);
      if (active && r < q) P[r * nsv + j] = s;
    }
    if (check && active && rgi == 0) {
      // x_ref is read here, before this iteration's prefetch is issued, so
      // waiting for it cannot drain the prefetch
      double s = 0.0;
      if (colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const double d = (double)xv[e] - p.x_ref[cv * V + e];
          s = fma(d, d, s);
        }
      }
      E[j] = s;
    }
    __syncthreads();
    // row r's nsv partials: a team of tr lanes, lane u adding entries u,
    // u + tr, ... in order, then an xor fold over the team (fixed order).
    // The loop bound is uniform, so every lane takes part in the folds.
    {
      const int TR = p.tr, team = t / TR, u = t & (TR - 1), nteams = NT / TR;
      for (int r0 = 0; r0 < q; r0 += nteams) {
        const int r = r0 + team;
        C d = 0;
        if (r < q)
          for (int jj = u; jj < nsv; jj += TR) d += P[r * nsv + jj];
        d = team_sum(d, TR);
        if (u == 0 && r < q) {
          if (G > 1)
            part.put((int64_t)r * G + g, (double)d, tag);
          else
            SC[r] = (r0 == 0) ? scale_of(mine_a, mine_b, mine_w, (double)d)
                              : scale_of(p.rec[kl * q + r].alpha, p.rec[kl * q + r].b,
                                         p.rec[kl * q + r].wn, (double)d);
        }
      }
    }
    if (check && t < kWave) {  // the whole first wave
      double s = 0.0;
      for (int jj = t; jj < nsv; jj += kWave) s += E[jj];
      s = wave_sum(s);
      if (t == 0) {
        if (G > 1)
          part.put((int64_t)q * G + g, s, tag);
        else
          SC[q] = s;
      }
    }
    // the next iteration's rows (independent of x) are requested now, so that
    // they stream in while the exchange below is in progress
#pragma unroll
    for (int i = 0; i < RPT; ++i) an[i] = load_raw<T, V>(A + (int64_t)rows_n[i] * p.lda + cvl * V);
    bool ok = true;
    if (G > 1) {
      if constexpr (GATHER) {
        // every workgroup polls every row's partials and sums them in the
        // same fixed order (slot L = r G + gg of this thread's share: the
        // slots are value-major, row r's G partials contiguous)
        const int total = G * nr;
        bool have[kPollMax];
#pragma unroll
        for (int u = 0; u < kPollMax; ++u) have[u] = t + NT * u >= total;
        for (unsigned spins = 0;; ++spins) {
          uint64_t lo[kPollMax], hi[kPollMax];
#pragma unroll
          for (int u = 0; u < kPollMax; ++u) {
            const int L = t + NT * u < total ? t + NT * u : total - 1;
            part.fetch(L, lo[u], hi[u]);
          }
          bool all = true;
#pragma unroll
          for (int u = 0; u < kPollMax; ++u) {
            double v;
            if (!have[u] && TagSlots::decode(lo[u], hi[u], tag, v)) {
              const int L = t + NT * u;
              PG[(L % G) * (q + 1) + L / G] = v;
              have[u] = true;
            }
            all = all && have[u];
          }
          if (__syncthreads_and(all)) break;
          if (spins >= kSpinLimit) {
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        // row r's G partials: a team of tr_g lanes, as for the slice sums
        {
          const int TR = p.tr_g, team = t / TR, u = t & (TR - 1), nteams = NT / TR;
          for (int r0 = 0; r0 < nr; r0 += nteams) {
            const int r = r0 + team;
            double D = 0.0;
            if (r < nr)
              for (int gg = u; gg < G; gg += TR) D += PG[gg * (q + 1) + r];
            D = team_sum(D, TR);
            if (u == 0 && r < nr) {
              if (r < q) {
                const bool mine = r0 == 0;
                const double rb = mine ? mine_b : p.rec[kl * q + r].b;
                const double rw = mine ? mine_w : p.rec[kl * q + r].wn;
                const double ra = mine ? mine_a : p.rec[kl * q + r].alpha;
                SC[r] = scale_of(ra, rb, rw, D);
              } else {
                SC[r] = D;
              }
            }
          }
        }
      } else if constexpr (!GATHER) {
        // phase 1: workgroup g sums the partials of rows g, g + G, ...
        // the q + 1 sums go to kSumCopies copies; workgroup g polls
        // copy g % kSumCopies
        const TagSlots scal(p.scal, (int64_t)kSumCopies * (q + 1));
        for (int r = g; r < nr; r += G) {
          RowRec rr;
          if (t == 0 && r < q) rr = p.rec[kl * q + r];  // in flight with the polls
          double v = 0.0;
          bool have = t >= G;
          for (unsigned spins = 0;; ++spins) {
            uint64_t lo, hi;
            part.fetch((int64_t)r * G + (t < G ? t : G - 1), lo, hi);
            double pv;
            if (!have && TagSlots::decode(lo, hi, tag, pv)) {
              v = pv;
              have = true;
            }
            if (__syncthreads_and(have)) break;
            if (spins >= kSpinLimit) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          // slots beyond the thread count (G > NT), under the same bounded
          // wait: a slot that never arrives makes the whole solve report
          // RKA_EDEVICE instead of adding zero
          bool got_all = true;
          for (int gg = t + NT; gg < G; gg += NT) {
            uint64_t lo, hi;
            double pv = 0.0;
            bool got = false;
            for (unsigned spins = 0; spins < kSpinLimit; ++spins) {
              part.fetch((int64_t)r * G + gg, lo, hi);
              if (TagSlots::decode(lo, hi, tag, pv)) {
                got = true;
                break;
              }
              __builtin_amdgcn_s_sleep(1);
            }
            got_all = got_all && got;
            v += pv;
          }
          if (!__syncthreads_and(got_all)) ok = false;
          const double D = block_sum(v, RED);
          if (t == 0) {
            const double sv = r < q ? scale_of(rr.alpha, rr.b, rr.wn, D) : D;
            for (int c = 0; c < kSumCopies; ++c) scal.put(c * (q + 1) + r, sv, tag);
          }
        }
        // phase 2: every workgroup polls the q scales (one slot per thread
        // per round; one round unless q + 1 exceeds the thread count)
        for (int L0 = 0; L0 < nr && ok; L0 += NT) {
          const int L = L0 + t;
          bool have = L >= nr;
          for (unsigned spins = 0;; ++spins) {
            uint64_t lo, hi;
            scal.fetch((g % kSumCopies) * (q + 1) + (L < nr ? L : nr - 1), lo, hi);
            double v;
            if (!have && TagSlots::decode(lo, hi, tag, v)) {
              SC[L] = v;
              have = true;
            }
            if (__syncthreads_and(have)) break;
            if (spins >= kSpinLimit) {
              ok = false;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
      }
      if (!__syncthreads_and(ok)) {
        if (t == 0) note_timeout(p.st);
        stopped = true;
        break;
      }
    }
    __syncthreads();
    if (check) {
      const double e2 = SC[q];
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
    // x_slice += (1/q) sum_r s_r * A[i_r, slice]   (fixed row order)
    C u[V];
#pragma unroll
    for (int e = 0; e < V; ++e) u[e] = 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = rgi + rg * i;
      const C s = (colv && r < q) ? (C)SC[r < q ? r : 0] : (C)0;
#pragma unroll
      for (int e = 0; e < V; ++e) u[e] = fma(s, raw_elem_c<C, T, V>(a[i], e), u[e]);
    }
    if (active) {
#pragma unroll
      for (int e = 0; e < V; ++e) U[t * V + e] = u[e];
    }
    __syncthreads();
    for (int L = t; L < NE * NP; L += NT) {
      const int je = L % NE, part = L / NE;
      const int jj = je / V, e = je % V;
      const int g0 = part * rg / NP, g1 = (part + 1) * rg / NP;
      C acc = 0;
      for (int gg = g0; gg < g1; ++gg) acc += U[(gg * nsv + jj) * V + e];
      UP[L] = acc;
    }
    __syncthreads();
    if (colv && rgi == 0) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        C acc = 0;
        for (int pp = 0; pp < NP; ++pp) acc += UP[pp * NE + j * V + e];
        xv[e] = fma(acc, (C)p.inv_q, xv[e]);
        XS[j * V + e] = xv[e];
      }
    }
    __syncthreads();
    if (colv) {
#pragma unroll
      for (int e = 0; e < V; ++e) xv[e] = XS[j * V + e];
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      a[i] = an[i];
      rows[i] = rows_n[i];
    }
    // records for the iterations ahead (clamped at the chunk end)
    const int64_t k2 = kl + 2 < p.K ? kl + 2 : p.K - 1;
    const int64_t k1 = kl + 1 < p.K ? kl + 1 : p.K - 1;
    load_next(k2, k1);
  }
  if (colv && rgi == 0) {
#pragma unroll
    for (int e = 0; e < V; ++e) p.x[cv * V + e] = (double)xv[e];
  }
  if (!stopped && g == 0 && t == 0) p.st->iterations = p.k0 + p.K;
}

static int rpt_bucket(int need) {
  if (need <= 1) return 1;
  if (need <= 2) return 2;
  if (need <= 4) return 4;
  if (need <= 8) return 8;
  if (need <= 11) return 11;
  if (need <= 16) return 16;
  return 0;
}

// Column slices.  Measured on MI355X with FP64 storage: at q = 16 and below
// 48 workgroups take 5.5 us per iteration against 7.0 us on 250 (80000 x
// 10000), since the rows of one iteration are few and the exchange with fewer
// participants is shorter; for q = 32 .. 128 about 5/8 of the CUs is fastest
// (q = 64: 8.3 us on 157 workgroups against 8.7 on 250 at 80000 x 10000, 9.5
// against 9.8 on 179 at 200000 x 20000), and where the q rows do not fit
// the tiles of that grid the full grid takes them (q = 256 at 80000 x
// 10000).  Other storage types keep one workgroup per CU.  Tiny problems
// (<= 64 KB of rows per iteration, one slice that fits a workgroup) run in
// one workgroup with no exchange at all.
constexpr int kSmallQ = 16;
constexpr int kSmallQGrid = 48;
constexpr int kWideGridNum = 5, kWideGridDen = 8;
constexpr int64_t kOneGroupBytes = 64 << 10;
// one-barrier all-gather while every workgroup reads at most this many partials
constexpr int kGatherMax = 2048;

static bool col_plan_at(const SolveShape& sh, int target, RkaColGeom* geo);

bool rka_col_plan(const SolveShape& sh, RkaColGeom* geo) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int64_t bytes_per_iter = (int64_t)sh.q * sh.n * esz;
  if (sh.grid > 0) return col_plan_at(sh, sh.grid, geo);
  if (bytes_per_iter <= kOneGroupBytes) return col_plan_at(sh, 1, geo);
  // small q: a few dozen workgroups, unless slices that wide do not fit a
  // workgroup (very long rows), then the wider grids below
  if (sh.q <= kSmallQ && col_plan_at(sh, std::min(sh.num_cu, kSmallQGrid), geo)) return true;
  if (sh.dtype == 0 && col_plan_at(sh, sh.num_cu * kWideGridNum / kWideGridDen, geo)) return true;
  return col_plan_at(sh, sh.num_cu, geo);
}

static bool col_plan_at(const SolveShape& sh, int target, RkaColGeom* geo) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  const int64_t nvec = sh.n / V;
  int G, nsv;
  if (target == 1 && nvec <= kMaxColThreads) {
    G = 1;
    nsv = (int)nvec;
  } else {
    const int64_t g0 = nvec < target ? nvec : target;
    nsv = (int)((nvec + g0 - 1) / g0);
    G = (int)((nvec + nsv - 1) / nsv);
    if (nsv > kMaxColThreads) return false;
  }
  int rg = kMaxColThreads / nsv;
  if (rg > sh.q) rg = sh.q;
  if (rg < 1) rg = 1;
  const int rpt = rpt_bucket((sh.q + rg - 1) / rg);
  if (rpt == 0) return false;
  // largest spill-free bucket per storage type; wider q runs on the worker kernel
  const int rpt_max = !sh.vec_ok ? 11 : ((sh.dtype == 0 || (sh.acc == 1 && sh.dtype == 1)) ? 11 : 4);
  if (rpt > rpt_max) return false;
  const int nt = ((nsv * rg + kWave - 1) / kWave) * kWave;
  int gather = 0;
  if (G > 1) {
    const bool fits = (int64_t)G * (sh.q + 1) <= (int64_t)kPollMax * nt;
    if (sh.allreduce == 1) {
      if (!fits) return false;
      gather = 1;
    } else if (sh.allreduce == 0) {
      gather = fits && (int64_t)G * (sh.q + 1) <= kGatherMax;
    }
    if (gather && rpt == 11) {
      if (sh.allreduce == 1) return false;
      gather = 0;
    }
    if (!gather && sh.q + 1 > kPollMax * nt) return false;
  }
  const size_t pg = gather ? (size_t)G * (sh.q + 1) : 0;
  const size_t csz = sh.acc == 1 ? sizeof(float) : sizeof(double);
  const size_t lds = sizeof(double) * (nsv + 16 + sh.q + 1 + pg) +
                     csz * ((size_t)sh.q * nsv + (size_t)nt * V + (size_t)nsv * V +
                            (size_t)std::max(nt, nsv * V));
  if (lds > 64 * 1024) return false;
  // reduction teams: as many lanes per row as keep every row in one round
  auto pow2_team = [](int64_t cap) {
    int tr = 1;
    while (tr * 2 <= cap && tr * 2 <= kWave) tr *= 2;
    return tr;
  };
  geo->tr = pow2_team(std::min<int64_t>(nt / sh.q, nsv));
  geo->tr_g = gather ? pow2_team(std::min<int64_t>(nt / (sh.q + 1), G)) : 1;
  geo->G = G;
  geo->nsv = nsv;
  geo->rg = rg;
  geo->nt = nt;
  geo->rpt = rpt;
  geo->lds = lds;
  geo->gather = gather;
  return true;
}

template <typename T, typename C, int V, bool GATHER>
static const void* col_fn(int rpt) {
  switch (rpt) {
    case 1: return (const void*)rka_col_kernel<T, C, V, 1, GATHER>;
    case 2: return (const void*)rka_col_kernel<T, C, V, 2, GATHER>;
    case 4: return (const void*)rka_col_kernel<T, C, V, 4, GATHER>;
    default: return (const void*)rka_col_kernel<T, C, V, 8, GATHER>;
  }
}

template <typename T, typename C, int V>
static hipError_t launch_col_t(const RkaColGeom& geo, RkaColArgs& a, hipStream_t s) {
  void* args[] = {&a};
  const void* fn = geo.rpt == 11 ? (const void*)rka_col_kernel<T, C, V, 11, false>
                   : geo.gather  ? col_fn<T, C, V, true>(geo.rpt)
                                 : col_fn<T, C, V, false>(geo.rpt);
  return launch_persistent(fn, dim3(geo.G), dim3(geo.nt), args, (unsigned)geo.lds, s);
}

hipError_t launch_rka_chunk(const SolveShape& sh, const RkaColGeom& geo, const RowRec* rec,
                            int64_t k0, int64_t K, int64_t check_every, uint64_t* part,
                            uint64_t* scal, DevStatus* st, hipStream_t s) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  RkaColArgs a;
  a.A = sh.A;
  a.lda = sh.lda;
  a.nvec = sh.n / V;
  a.rec = rec;
  a.x = sh.x;
  a.x_ref = sh.x_ref;
  a.alpha = sh.alpha;
  a.inv_q = 1.0 / (double)sh.q;
  a.q = sh.q;
  a.nsv = geo.nsv;
  a.rg = geo.rg;
  a.G = geo.G;
  a.gather = geo.gather;
  a.tr = geo.tr;
  a.tr_g = geo.tr_g;
  a.k0 = k0;
  a.K = K;
  a.check_every = check_every;
  a.part = part;
  a.scal = scal;
  a.st = st;
  if (sh.acc == 1) {
    if (sh.dtype == 1)
      return sh.vec_ok ? launch_col_t<float, float, 4>(geo, a, s)
                       : launch_col_t<float, float, 1>(geo, a, s);
    return sh.vec_ok ? launch_col_t<bf16_t, float, 8>(geo, a, s)
                     : launch_col_t<bf16_t, float, 1>(geo, a, s);
  }
  switch (sh.dtype) {
    case 0:
      return sh.vec_ok ? launch_col_t<double, double, 2>(geo, a, s)
                       : launch_col_t<double, double, 1>(geo, a, s);
    case 1:
      return sh.vec_ok ? launch_col_t<float, double, 4>(geo, a, s)
                       : launch_col_t<float, double, 1>(geo, a, s);
    default:
      return sh.vec_ok ? launch_col_t<bf16_t, double, 8>(geo, a, s)
                       : launch_col_t<bf16_t, double, 1>(geo, a, s);
  }
}

// ===========================================================================
// Stopping measures (Sec. 3.1: the error to the solution; without one, the
// relative residual).  Fixed-order sums; the decision is written to the
// device status so that later kernels of the solve return immediately.
// ===========================================================================
__global__ void status_init_kernel(DevStatus* st, double tol) {
  st->iterations = 0;
  st->done = 0;
  st->status = tol > 0.0 ? 1 : 0;  // RKA_NOT_CONVERGED until the test passes
  st->rel2 = __builtin_nan("");
  st->ref2 = 1.0;
  st->thresh2 = 0.0;
  st->last_pos = -1;
}

__global__ __launch_bounds__(1024) void ref_norm_kernel(const double* __restrict__ v, int64_t len,
                                                         double tol, DevStatus* st) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s = fma(v[i], v[i], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    st->ref2 = s;
    st->thresh2 = tol * tol * s;
  }
}

__global__ __launch_bounds__(1024) void measure_xref_kernel(const double* __restrict__ x,
                                                             const double* __restrict__ xr,
                                                             int64_t n, int64_t k, DevStatus* st) {
  __shared__ double red[16];
  if (st->done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = x[i] - xr[i];
    s = fma(d, d, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    st->rel2 = s / st->ref2;
    if (!isfinite(s)) {
      st->status = -3;
      st->done = 1;
      st->iterations = k;
    } else if (s <= st->thresh2) {
      st->status = 0;
      st->done = 1;
      st->iterations = k;
    }
  }
}

constexpr int kResidRowsPerBlock = 64;

int resid_blocks(int64_t m) { return (int)((m + kResidRowsPerBlock - 1) / kResidRowsPerBlock); }

// One wave per row, 4 waves per block, kResidRowsPerBlock rows per block:
// partial[blk] = sum over the block's rows of (b_i - <A_i, x>)^2.
template <typename T>
__global__ __launch_bounds__(256) void resid_kernel(const T* __restrict__ A, int64_t m, int64_t n,
                                                    int64_t lda, const double* __restrict__ b,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ part,
                                                    const DevStatus* st) {
  __shared__ double red[4];
  if (st->done) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc = 0.0;
  for (int rr = wv; rr < kResidRowsPerBlock; rr += 4) {
    const int64_t i = (int64_t)blockIdx.x * kResidRowsPerBlock + rr;
    if (i >= m) break;
    double d = 0.0;
    for (int64_t c = lane; c < n; c += 64) d = fma(widen(A[i * lda + c]), x[c], d);
    d = wave_sum(d);
    const double r = b[i] - d;
    acc = fma(r, r, acc);
  }
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(1024) void resid_finish_kernel(const double* __restrict__ part,
                                                             int nb, int64_t k, DevStatus* st) {
  __shared__ double red[16];
  if (st->done) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    st->rel2 = s / st->ref2;
    if (!isfinite(s)) {
      st->status = -3;
      st->done = 1;
      st->iterations = k;
    } else if (s <= st->thresh2) {
      st->status = 0;
      st->done = 1;
      st->iterations = k;
    }
  }
}

hipError_t launch_status_init(DevStatus* st, double tol, hipStream_t s) {
  hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(1), 0, s, st, tol);
  return hipGetLastError();
}

hipError_t launch_ref_norm(const double* ref, int64_t len, double tol, DevStatus* st,
                           hipStream_t s) {
  hipLaunchKernelGGL(ref_norm_kernel, dim3(1), dim3(1024), 0, s, ref, len, tol, st);
  return hipGetLastError();
}

hipError_t launch_measure(const SolveShape& sh, int64_t k, double* part, DevStatus* st,
                          hipStream_t s) {
  if (sh.x_ref) {
    hipLaunchKernelGGL(measure_xref_kernel, dim3(1), dim3(1024), 0, s, sh.x, sh.x_ref, sh.n, k,
                       st);
    return hipGetLastError();
  }
  const int nb = resid_blocks(sh.m);
  switch (sh.dtype) {
    case 0:
      hipLaunchKernelGGL(resid_kernel<double>, dim3(nb), dim3(256), 0, s, (const double*)sh.A,
                         sh.m, sh.n, sh.lda, sh.b, sh.x, part, st);
      break;
    case 1:
      hipLaunchKernelGGL(resid_kernel<float>, dim3(nb), dim3(256), 0, s, (const float*)sh.A, sh.m,
                         sh.n, sh.lda, sh.b, sh.x, part, st);
      break;
    default:
      hipLaunchKernelGGL(resid_kernel<bf16_t>, dim3(nb), dim3(256), 0, s, (const bf16_t*)sh.A,
                         sh.m, sh.n, sh.lda, sh.b, sh.x, part, st);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(resid_finish_kernel, dim3(1), dim3(1024), 0, s, part, nb, k, st);
  return hipGetLastError();
}

}  // namespace rka
