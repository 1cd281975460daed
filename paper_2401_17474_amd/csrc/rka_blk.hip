// rka_blk.hip -- RKA (Eq. (7), arXiv 2401.17474 Sec. 3.3.1) in blocks of p
// iterations per cross-workgroup exchange, with the block's x-independent
// coefficients computed by a separate streaming pass.
//
// Within a block of iterations k .. k+p-1 the rows are drawn in advance, and
// x^(k+j) - x^(k) = (1/q) sum_{l<j} sum_r s_{l,r} a_{l,r}.  The scale of row
// r (iteration j) is s_r = alpha_r (b_r - <a_r, x^(k+j)>) / w_r, so with
// c_r = alpha_r (b_r - <a_r, x^(k)>) / w_r and
//     N_{r,c} = alpha_r / (q w_r) <a_r, a_c>   (c drawn in an earlier
//                                              iteration of the block, else 0)
// the block's scales solve (I + N) s = c, i.e. s = M c with M = (I + N)^-1,
// unit lower triangular in q x q blocks.  M depends on the rows only, not on
// x: blk_coef_kernel forms it for every block of a chunk ahead of the
// iterations (inner products over the full rows, then block forward
// substitution), streaming the rows once more.  The iteration kernel then
// exchanges only the p q dot products with x^(k) (and the error of a
// stopping test) per block: one reduce-scatter + broadcast of p q + 1
// values, after which every workgroup forms s = M c and updates its slice of
// x from the rows it holds in registers.  Same iteration in exact
// arithmetic; the floating-point scales differ from one-iteration RKA's by
// rounding.
//
// Blocks never run across a stopping test (they end where a test falls) or a
// chunk end; both kernels locate blocks the same way (BlkLayout).  All sums
// have a fixed order: results are bitwise reproducible for a given launch
// geometry.
#include <math.h>

#include <algorithm>

#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// Phase timing of workgroups 0 and G/2 of the iteration kernel (printed at
// the end of a launch), for builds with RKA_BLK_PROF defined only.
#ifdef RKA_BLK_PROF
#define BPROF_DECL                             \
  uint64_t bp_t[8] = {0, 0, 0, 0, 0, 0, 0, 0}; \
  uint64_t bp_last = __builtin_readcyclecounter();
#define BPROF(i)                                          \
  do {                                                    \
    const uint64_t bp_now = __builtin_readcyclecounter(); \
    bp_t[i] += bp_now - bp_last;                          \
    bp_last = bp_now;                                     \
  } while (0)
#else
#define BPROF_DECL
#define BPROF(i) \
  do {           \
  } while (0)
#endif

// Blocks of a chunk [k0, k0 + K): segments end at multiples of C (the
// stopping-test interval, 0 = none) and at K; a segment of S iterations holds
// ceil(S / p) blocks of p iterations (the last one shorter).  The host fills
// the segment counts once (make); locate() then needs one 32-bit division,
// and only with stopping tests.
struct BlkLayout {
  int64_t k0;         // first iteration of the chunk
  int64_t C;          // stopping-test interval (0: none)
  int32_t K, p;       // iterations of the chunk, iterations per block
  int32_t f;          // iterations of the first segment
  int32_t nbf, nbc;   // blocks of the first segment, of a full segment
  int32_t nblk;       // blocks of the chunk
  int32_t first_test; // the chunk starts at a stopping test
  static BlkLayout make(int64_t k0, int64_t K, int64_t C, int p) {
    BlkLayout l{};
    l.k0 = k0;
    l.C = C > 0 ? C : 0;
    l.K = (int32_t)K;
    l.p = p;
    int64_t f = K;
    if (l.C > 0) {
      f = l.C - k0 % l.C;
      if (f > K) f = K;
    }
    l.f = (int32_t)f;
    l.nbf = (int32_t)((f + p - 1) / p);
    l.nblk = l.nbf;
    l.nbc = 0;
    if (l.C > 0 && f < K) {
      // here C < K + C - f, and whole segments exist only if C <= K < 2^31
      const int64_t rest = K - f, full = rest / l.C, tail = rest % l.C;
      const int64_t nbc = (l.C + p - 1) / p;
      l.nbc = (int32_t)(nbc < INT32_MAX ? nbc : INT32_MAX);
      l.nblk += (int32_t)(full * nbc + (tail + p - 1) / p);
    }
    l.first_test = l.C > 0 && k0 > 0 && k0 % l.C == 0;
    return l;
  }
  // block b: first chunk-local iteration, length, and whether a stopping
  // test falls at its start
  __device__ __forceinline__ void locate(int b, int* kl, int* L, bool* test) const {
    int64_t s0, slen;
    int i;
    if (b < nbf) {
      s0 = 0;
      slen = f;
      i = b;
      *test = first_test && b == 0;
    } else {
      const int bb = b - nbf, seg = bb / nbc;
      i = bb - seg * nbc;
      s0 = f + (int64_t)seg * C;
      slen = (int64_t)K - s0 < C ? (int64_t)K - s0 : C;
      *test = i == 0;
    }
    const int64_t k = s0 + (int64_t)i * p;
    const int64_t left = s0 + slen - k;
    *kl = (int)k;
    *L = (int)(left < p ? left : p);
  }
};

// strictly lower q x q blocks (j, l), l < j, of M, in pair order
__host__ __device__ constexpr int blk_pair(int j, int l) { return j * (j - 1) / 2 + l; }
__host__ __device__ constexpr int blk_ncoef(int q, int p) { return q * q * (p * (p - 1) / 2); }

constexpr int kBMaxRows = 128;   // q p
constexpr int kBThreads = 512;   // iteration kernel
constexpr int kBPoll = 2;        // slots one lane polls in either phase
constexpr int kBBatch = 4;       // poll loads in flight per lane
constexpr int kCThreads = 512;   // coefficient kernel: 8 waves, two per SIMD (an FP64 MFMA
                                 // issues every ~60 ns from one wave per SIMD; two waves
                                 // per SIMD reach the unit's ~48 TF/s)
constexpr int kCWaves = kCThreads / 64;
constexpr int kCElems = 4096;    // elements of a staged chunk (rows x columns)
constexpr int kCPre = kCElems / kCThreads;  // staged elements per lane
constexpr int kCMaxSlots = 5;    // 16 x 16 Gram tiles per wave (36 = 8 * 9 / 2 over 8 waves)

// ===========================================================================
// The coefficient pass: M of every block of a chunk.
// ===========================================================================
struct CoefArgs {
  const void* A;
  int64_t lda, n;
  const RowRec* rec;  // K x q records of the chunk
  BlkLayout lay;
  int32_t q;
  int32_t RS;         // column stride of the staged chunk (doubles, >= rows rounded to 16)
  int32_t lcw;        // log2 of the columns of a staged chunk
  double inv_q;
  double* coef;       // nblk x cstride
  int32_t ncoef;      // coefficients of a full block
  int32_t cstride;    // doubles between blocks in coef (a multiple of 128)
  int32_t cbuf;       // LDS-direct staging: bytes per chunk buffer
  const DevStatus* st;  // a solve that has stopped needs no more coefficients
};

template <typename T>
__device__ __forceinline__ double elem_at(const T* A, int64_t off) {
  return widen(A[off]);
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Offset of row r = jr q + rho in the row-major packing of M's strictly lower
// part: row r holds its jr q coefficients (iterations 0 .. jr-1) contiguously.
__host__ __device__ __forceinline__ int blk_rowoff(int q, int jr, int rho) {
  return q * q * (jr * (jr - 1) / 2) + rho * jr * q;
}

// Wave W's part of a block's Gram tiles: stage the rows chunk by chunk
// (every wave takes part and meets every barrier), accumulate the wave's
// tiles, then write its entries of N into NB (over S, once every wave is
// done with S).
//
// Tiles: the lower 16 x 16 tiles (I, J), J <= I, that hold a pair of rows
// from different iterations, in the order I = 0, 1, ...; J = 0 .. I; wave W
// takes every eighth from the W-th into its NS slots (slots past its share
// repeat tile (0, 0); their sums are never used).  Per 4 columns a lane loads
// both fragments of every slot (lane l: column c + l / 16, row 16 I + l % 16),
// the next 4 columns' while the current ones feed v_mfma_f64_16x16x4f64.
//
// Chunks of CW columns (RP x CW <= 4096 elements) are staged in LDS, the next
// chunk's elements in flight in registers while the current one is used.
// Element e: row e >> lcw, column e & (CW - 1) -- consecutive lanes read
// consecutive columns of a row.  Loads are unconditional (clamped rows and
// columns); elements past the block's rows or past n are zero.
// This wave's tiles (see above): slot u holds tile (tI[u], tJ[u]); returns
// the number of slots used.
template <int NS>
__device__ __forceinline__ int coef_tiles(int R, int RG, int q, int wv, int (&tI)[NS],
                                          int (&tJ)[NS]) {
  int nt = 0;
#pragma unroll
  for (int u = 0; u < NS; ++u) tI[u] = tJ[u] = 0;
  int idx = 0;
  for (int I = 0; I < RG; ++I)
    for (int J = 0; J <= I; ++J) {
      const int rlast = (16 * I + 15 < R ? 16 * I + 15 : R - 1);
      if (rlast / q > (16 * J) / q) {  // some row of I is of a later iteration
        if (idx % kCWaves == wv && nt < NS) {
#pragma unroll
          for (int u = 0; u < NS; ++u)
            if (u == nt) {
              tI[u] = I;
              tJ[u] = J;
            }
          ++nt;
        }
        ++idx;
      }
    }
  return nt;
}

// Row of a 16-row tile that fragment lane i (0..15) supplies on the
// LDS-direct path: the 8 lanes of a fragment read served together take
// rows of 8 different pairs (see kCPairBytes).
__device__ __forceinline__ int frag_row(int i) { return 2 * (i & 7) + (i >> 3); }

// N = alpha_r / (q w_r) <a_r, a_c> for rows r, c of iterations j > l, from
// this wave's tiles, into NB (q x q blocks by pair).  FR: the tiles' rows
// were supplied in frag_row order.
template <int NS, bool FR = false>
__device__ __forceinline__ void coef_store_n(const f64x4 (&acc)[NS], const int (&tI)[NS],
                                             const int (&tJ)[NS], int nt, int lane, int R, int q,
                                             const double* FAC, double* NB) {
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    if (u < nt) {
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int ri = lane / 16 + 4 * rr, ci = lane & 15;
        const int r = 16 * tI[u] + (FR ? frag_row(ri) : ri), c = 16 * tJ[u] + (FR ? frag_row(ci) : ci);
        if (r < R && c < R) {
          const int jr = r / q, lc = c / q;
          if (jr > lc)
            NB[blk_pair(jr, lc) * q * q + (r - jr * q) * q + (c - lc * q)] = FAC[r] * acc[u][rr];
        }
      }
    }
  }
}

template <typename T, int NS>
__device__ __forceinline__ void coef_gram(const CoefArgs& p, const T* __restrict__ A, double* S,
                                          double* NB, const double* FAC, const int64_t* ROW, int R,
                                          int RG) {
  const int t = threadIdx.x, q = p.q, lane = t & (kWave - 1), wv = t / kWave;
  const int CW = 1 << p.lcw, RP = 16 * RG;
  int tI[NS], tJ[NS];
  const int nt = coef_tiles<NS>(R, RG, q, wv, tI, tJ);
  f64x4 acc[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) acc[u] = (f64x4){0.0, 0.0, 0.0, 0.0};
  // (the loads only: zeroing happens at the LDS store, so that no load waits
  // for the one before it)
  double nxt[kCPre];
  const T* rowp[kCPre];
#pragma unroll
  for (int i = 0; i < kCPre; ++i) {
    const int r = (t + kCThreads * i) >> p.lcw;
    rowp[i] = A + ROW[r < R ? r : R - 1] * p.lda;
  }
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int i = 0; i < kCPre; ++i) {
      const int c = (t + kCThreads * i) & (CW - 1);
      nxt[i] = elem_at<T>(rowp[i], c0 + c < p.n ? c0 + c : p.n - 1);
    }
  };
  const double* base = S + (size_t)(lane >> 4) * p.RS + (lane & 15);
  double fa[2 * NS], fb[2 * NS];
  auto load = [&](double(&f)[2 * NS], int c) {
    const double* Sc = base + (size_t)c * p.RS;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      f[2 * u] = Sc[16 * tI[u]];
      f[2 * u + 1] = Sc[16 * tJ[u]];
    }
  };
  auto step = [&](const double(&f)[2 * NS]) {
#pragma unroll
    for (int u = 0; u < NS; ++u)
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[2 * u], f[2 * u + 1], acc[u], 0, 0, 0);
  };
  fetch(0);
  for (int64_t c0 = 0; c0 < p.n; c0 += CW) {
    __syncthreads();  // the previous chunk has been used
#pragma unroll
    for (int i = 0; i < kCPre; ++i) {
      const int e = t + kCThreads * i;
      const int r = e >> p.lcw, c = e & (CW - 1);
      if (r < RP) S[(size_t)c * p.RS + r] = (r < R && c0 + c < p.n) ? nxt[i] : 0.0;
    }
    __syncthreads();
    if (c0 + CW < p.n) fetch(c0 + CW);
    load(fa, 0);
    for (int c = 0; c < CW; c += 8) {  // CW is a multiple of 8
      load(fb, c + 4);
      step(fa);
      if (c + 8 < CW) load(fa, c + 8);
      step(fb);
    }
  }
  __syncthreads();  // every wave is done with S: NB takes its place
  coef_store_n<NS>(acc, tI, tJ, nt, lane, R, q, FAC, NB);
}

// The same on the 16-byte vector path, staged by LDS-direct loads
// (global_load_lds: lane l of a wave writes its 16 bytes at the
// instruction's LDS base + 16 l): one instruction carries rows 2k (lanes
// 0..31) and 2k + 1 (lanes 32..63) of a 512-byte column segment, CW = 512 /
// sizeof(T) columns; a row pair takes kCPairBytes of LDS (16 bytes of
// padding: pairs lie 16 bytes apart modulo 128, so the 8 lanes a 16-byte
// fragment read serves together, taking rows of 8 different pairs in
// frag_row order, fall on 8 different 16-byte bank groups; with the rows in
// order, rows 2k and 2k + 1 of a pair lie 512 bytes apart, on the same
// banks).
// Two buffers of cbuf bytes: the next chunk's 64 KB are in flight during the
// current chunk's MFMAs, with no registers spent on them.  Rows past the
// block load a clamped row (they only reach products that are never
// stored); columns past n are zeroed in LDS after the last chunk lands.
constexpr int kCPairBytes = 1024 + 16;
template <typename T, int NS>
__device__ __forceinline__ void coef_gram_dma(const CoefArgs& p, const T* __restrict__ A,
                                              char* SB, double* NB, const double* FAC,
                                              const int64_t* ROW, int R, int RG) {
  constexpr int EPL = 16 / (int)sizeof(T);  // elements per lane per load
  constexpr int CW = 32 * EPL;              // columns per chunk
  const int t = threadIdx.x, q = p.q, lane = t & (kWave - 1), wv = t / kWave;
  const int npairs = 8 * RG;                // row pairs staged (16 RG rows)
  int tI[NS], tJ[NS];
  const int nt = coef_tiles<NS>(R, RG, q, wv, tI, tJ);
  f64x4 acc[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) acc[u] = (f64x4){0.0, 0.0, 0.0, 0.0};
  // this lane's rows: pair wv + 4 i, row 2 (wv + 4 i) + lane / 32
  constexpr int kMaxPI = kBMaxRows / 2 / kCWaves;  // row pairs per wave
  const T* rowp[kMaxPI];
#pragma unroll
  for (int i = 0; i < kMaxPI; ++i) {
    const int r = 2 * (wv + kCWaves * i) + (lane >> 5);
    rowp[i] = A + ROW[r < R ? r : R - 1] * p.lda + (lane & 31) * EPL;
  }
  const int nch = (int)((p.n + CW - 1) / CW);
  auto issue = [&](int c, int buf) {
    const int64_t c0 = (int64_t)c * CW;
    // the last chunk's lanes past n read the row's last 16 bytes instead
    const int64_t shift = c0 + (lane & 31) * EPL + EPL > p.n ? p.n - EPL - (c0 + (lane & 31) * EPL) : 0;
    char* base = SB + (size_t)buf * p.cbuf;
#pragma unroll
    for (int i = 0; i < kMaxPI; ++i) {
      const int k = wv + kCWaves * i;
      if (k < npairs)
        __builtin_amdgcn_global_load_lds((const void*)(rowp[i] + c0 + shift),
                                         (__attribute__((address_space(3))) void*)(base + k * kCPairBytes),
                                         16, 0, 0);
    }
  };
  // fragment byte offsets of each slot's two rows within a buffer
  int offI[NS], offJ[NS];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int ri = 16 * tI[u] + frag_row(lane & 15), rj = 16 * tJ[u] + frag_row(lane & 15);
    offI[u] = (ri >> 1) * kCPairBytes + (ri & 1) * 512 + 2 * (lane >> 4) * (int)sizeof(T);
    offJ[u] = (rj >> 1) * kCPairBytes + (rj & 1) * 512 + 2 * (lane >> 4) * (int)sizeof(T);
  }
  // Two MFMA steps per fragment read: over 8 columns 8P .. 8P + 7, lane l
  // reads columns 8P + 2 (l / 16) and 8P + 2 (l / 16) + 1 of each of its
  // slots' rows with one LDS read (two elements), the first feeding step
  // 2P and the second step 2P + 1 (each step still sums 4 distinct columns;
  // together the 8).  Half the LDS reads, and few enough in flight for the
  // wait counter to track them one step ahead.
  struct Pair2 {
    T v[2];
  };
  double fa[4 * NS], fb[4 * NS];
  // NA: the slots a wave runs; a wave holding fewer tiles than slots skips
  // its last (dummy) slot's reads and MFMAs (at q = 16, 28 tiles over 8
  // waves of 4 slots: 1/8 of the MFMA time of the SIMDs that carry them)
  auto load = [&](auto na, double(&f)[4 * NS], const char* base, int c) {
    constexpr int NA = decltype(na)::value;
    const char* bc = base + c * (int)sizeof(T);
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const Pair2 a = *(const Pair2*)(bc + offI[u]);
      const Pair2 bb = *(const Pair2*)(bc + offJ[u]);
      f[4 * u] = widen(a.v[0]);
      f[4 * u + 1] = widen(bb.v[0]);
      f[4 * u + 2] = widen(a.v[1]);
      f[4 * u + 3] = widen(bb.v[1]);
    }
  };
  auto step2 = [&](auto na, const double(&f)[4 * NS]) {
    constexpr int NA = decltype(na)::value;
#pragma unroll
    for (int u = 0; u < NA; ++u)
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[4 * u], f[4 * u + 1], acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < NA; ++u)
      acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[4 * u + 2], f[4 * u + 3], acc[u], 0, 0, 0);
  };
  // every wave meets the same barriers in either instance
  auto run = [&](auto na) {
    issue(0, 0);
    for (int c = 0; c < nch; ++c) {
      // this wave's loads of chunk c have landed; after the barrier every
      // wave's have, and every wave is done with chunk c - 1's buffer
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      const char* base = SB + (size_t)(c & 1) * p.cbuf;
      const int64_t c0 = (int64_t)c * CW;
      if (c0 + CW > p.n) {  // the last chunk: zero the columns past n
        const int valid = (int)(p.n - c0);
        for (int e = t; e < 2 * npairs * (CW - valid); e += kCThreads) {
          const int r = e / (CW - valid), col = valid + e - r * (CW - valid);
          *(T*)((char*)base + (r >> 1) * kCPairBytes + (r & 1) * 512 + col * (int)sizeof(T)) = T{};
        }
        __syncthreads();
      }
      if (c + 1 < nch) issue(c + 1, (c + 1) & 1);
      load(na, fa, base, 0);
      for (int k = 0; k < CW; k += 16) {  // CW is a multiple of 16
        load(na, fb, base, k + 8);
        step2(na, fa);
        if (k + 16 < CW) load(na, fa, base, k + 16);
        step2(na, fb);
      }
    }
  };
  if (__builtin_amdgcn_readfirstlane(nt) >= NS)
    run(std::integral_constant<int, NS>{});
  else
    run(std::integral_constant<int, NS - 1>{});
  __syncthreads();  // every wave is done with both buffers: NB takes their place
  coef_store_n<NS, true>(acc, tI, tJ, nt, lane, R, q, FAC, NB);
}

// The inner products of a block's rows are the needed lower 16 x 16 tiles of
// its R x R Gram matrix, each accumulated over the columns with
// v_mfma_f64_16x16x4f64: lane l supplies row 16 I + l % 16 and row
// 16 J + l % 16 at column c + l / 16, and holds D[l / 16 + 4 r][l % 16] in
// register r (D[i][j] = the inner product of rows 16 I + i and 16 J + j).
// The staged chunk and N (then M) share LDS: N is written once the last
// chunk has been used.
template <typename T, int NS, bool DMA>
__global__ __launch_bounds__(kCThreads) void blk_coef_kernel(CoefArgs p) {
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, q = p.q;
  extern __shared__ double lds[];
  // S: the staged chunk (column-major S[c RS + r], or the two LDS-direct
  // buffers); NB: N (then M) in q x q blocks by pair, over S once the Gram
  // tiles are complete
  const int CW = 1 << p.lcw;
  double* S = lds;
  double* NB = lds;                                                     // ncoef
  const int nSt = DMA ? p.cbuf / 4 : CW * p.RS;                         // doubles
  const int nS = nSt > p.ncoef ? nSt : p.ncoef;
  double* FAC = lds + nS;                        // kBMaxRows  alpha_r / (q w_r)
  int64_t* ROW = (int64_t*)(FAC + kBMaxRows);    // kBMaxRows
  for (int b = blockIdx.x; b < p.lay.nblk; b += gridDim.x) {
    int kl, L;
    bool test;
    p.lay.locate(b, &kl, &L, &test);
    const int R = L * q, RG = (R + 15) / 16;
    __syncthreads();  // the previous block's LDS reads are done
    for (int r = t; r < R; r += kCThreads) {
      const RowRec rc = p.rec[(int64_t)kl * q + r];
      ROW[r] = rc.row;
      FAC[r] = rc.alpha * p.inv_q / rc.wn;
    }
    __syncthreads();  // ROW and FAC are complete
    if constexpr (DMA)  // the Gram tiles, then N into NB
      coef_gram_dma<T, NS>(p, A, (char*)S, NB, FAC, ROW, R, RG);
    else
      coef_gram<T, NS>(p, A, S, NB, FAC, ROW, R, RG);
    __syncthreads();
    // block forward substitution, in place (N_{j,l} becomes M_{j,l}):
    //   M_{j,l} = -N_{j,l} - sum_{t=l+1}^{j-1} N_{j,t} M_{t,l}
    // for j ascending and, within j, l ascending: N_{j,t} (t > l) is not yet
    // overwritten when used, M_{t,l} (t < j) is final, and every element of
    // the (j, l) block reads only its own old value of that block.
    for (int jj = 1; jj < L; ++jj) {
      for (int ll = 0; ll < jj; ++ll) {
        double* Mjl = NB + blk_pair(jj, ll) * q * q;
        for (int e = t; e < q * q; e += kCThreads) {
          const int rr = e / q, cc = e - rr * q;
          double sacc = Mjl[e];
          for (int tt = ll + 1; tt < jj; ++tt) {
            const double* Njt = NB + blk_pair(jj, tt) * q * q + rr * q;
            const double* Mtl = NB + blk_pair(tt, ll) * q * q + cc;
            for (int k2 = 0; k2 < q; ++k2) sacc = fma(Njt[k2], Mtl[k2 * q], sacc);
          }
          Mjl[e] = -sacc;
        }
        __syncthreads();
      }
    }
    // out: row r = jr q + rho holds M_{r, c} for c < jr q contiguously
    double* out = p.coef + (size_t)b * p.cstride;
    for (int e = t; e < q * q * (L * (L - 1) / 2); e += kCThreads) {
      // e walks the pair blocks: block (jr, lc), entry (rho, sg)
      const int pb = e / (q * q), rem = e - pb * q * q;
      int jr = 1, lc = pb;
      while (lc >= jr) {
        lc -= jr;
        ++jr;
      }
      const int rho = rem / q, sg = rem - rho * q;
      out[blk_rowoff(q, jr, rho) + lc * q + sg] = NB[e];
    }
  }
}

// ===========================================================================
// Column-split RKAB, one block per outer iteration (Sec. 3.4.1).  Worker w
// projects its bs rows in order starting from x^(k), so its scales satisfy
// (I + N_w) s_w = c_w with c_j = alpha_j (b_j - <a_j, x^(k)>) / ||a_j||^2 and
// N_w[j][l] = alpha_j <a_j, a_l> / ||a_j||^2 for l < j (the worker's own
// earlier rows, weight 1), and x^(k+1) = x^(k) + (1/q) sum_w sum_j s_{w,j}
// a_{w,j} is the average of the workers' iterates.  This pass forms
// M_w = (I + N_w)^-1 for every (block, worker) task: one workgroup per task,
// lanes over the columns with the bs (bs - 1) / 2 inner products in
// registers, the workgroup's sums in wave order, then the forward
// substitution on one lane.  Output per block: worker w's strictly lower
// part at w bs (bs - 1) / 2, row j's j coefficients contiguous.
// ===========================================================================
constexpr int kRThreads = 256;

struct CoefRkabArgs {
  const void* A;
  int64_t lda, nvec;
  const RowRec* rec;  // K x q x bs records of the chunk
  BlkLayout lay;      // per outer iteration
  int32_t q;          // workers
  int32_t bs;         // projections per worker per outer iteration
  int32_t nsub;       // blocks per outer iteration (sub-blocks of BS projections, the last shorter)
  int32_t cstride;    // doubles between blocks in coef
  double* coef;
  const DevStatus* st;  // a solve that has stopped needs no more coefficients
};

template <typename T, int V, int BS>
__global__ __launch_bounds__(kRThreads) void blk_coef_rkab_kernel(CoefRkabArgs p) {
  using raw_t = typename Vec<T, V>::raw_t;
  constexpr int NP = BS * (BS - 1) / 2;
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  __shared__ double RED[kRThreads / kWave][NP];
  __shared__ double GR[NP];
  __shared__ double FAC[BS];
  __shared__ int64_t ROW[BS];
  const int64_t ntask = (int64_t)p.lay.nblk * p.nsub * p.q;
  for (int64_t task = blockIdx.x; task < ntask; task += gridDim.x) {
    const int b = (int)(task / p.q), w = (int)(task - (int64_t)b * p.q);
    const int bo = b / p.nsub, sb = b - bo * p.nsub;
    const int cs = BS < p.bs - sb * BS ? BS : p.bs - sb * BS;  // this sub-block's steps
    int kl, L;
    bool test;
    p.lay.locate(bo, &kl, &L, &test);
    __syncthreads();  // the previous task's LDS reads are done
    if (t < BS) {
      // steps past a short last sub-block repeat its last row: their
      // products are formed but their coefficients never read
      const RowRec rc =
          p.rec[((int64_t)kl * p.q + w) * p.bs + sb * BS + (t < cs ? t : cs - 1)];
      ROW[t] = rc.row;
      FAC[t] = rc.alpha / rc.wn;
    }
    __syncthreads();
    double acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = 0.0;
    for (int64_t c = t; c < p.nvec; c += kRThreads) {
      raw_t a[BS];
#pragma unroll
      for (int j = 0; j < BS; ++j) a[j] = load_raw<T, V>(A + ROW[j] * p.lda + c * V);
#pragma unroll
      for (int j = 1; j < BS; ++j) {
#pragma unroll
        for (int l = 0; l < j; ++l) {
#pragma unroll
          for (int e = 0; e < V; ++e)
            acc[j * (j - 1) / 2 + l] =
                fma(raw_elem<T, V>(a[j], e), raw_elem<T, V>(a[l], e), acc[j * (j - 1) / 2 + l]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double v = wave_sum(acc[i]);
      if (lane == 0) RED[wv][i] = v;
    }
    __syncthreads();
    if (t < NP) {
      double sum = 0.0;
      for (int u = 0; u < kRThreads / kWave; ++u) sum += RED[u][t];
      GR[t] = sum;
    }
    __syncthreads();
    if (t == 0) {
      // M[j][l] = -N[j][l] - sum_{tt = l+1}^{j-1} N[j][tt] M[tt][l], j ascending
      double M[NP];
      double* out = p.coef + (size_t)b * p.cstride + (size_t)w * NP;
#pragma unroll
      for (int j = 1; j < BS; ++j) {
#pragma unroll
        for (int l = 0; l < j; ++l) {
          double sacc = FAC[j] * GR[j * (j - 1) / 2 + l];
#pragma unroll
          for (int tt = l + 1; tt < j; ++tt)
            sacc = fma(FAC[j] * GR[j * (j - 1) / 2 + tt], M[tt * (tt - 1) / 2 + l], sacc);
          M[j * (j - 1) / 2 + l] = -sacc;
          out[j * (j - 1) / 2 + l] = -sacc;
        }
      }
    }
  }
}

// ===========================================================================
// The iteration kernel.
// ===========================================================================
struct BlkArgs {
  const void* A;
  int64_t lda, nvec;
  const RowRec* rec;  // K x q records of the chunk
  const double* coef; // nblk x cstride (blk_coef_kernel): M's rows packed
  double* x;
  const double* x_ref;
  double inv_q;
  BlkLayout lay;
  int32_t q, nsv, rg, G, nt;
  int32_t nsvp;       // lanes per row group: nsv rounded up to a power of two <= 64
  int32_t nv_max;     // exchange values of a full block: p q + 1
  int32_t cstride;    // doubles between blocks in coef (a multiple of 128)
  int32_t tr;         // lanes per row for the slice sums of the dot products
  int32_t trp;        // lanes per value in the reduce-scatter
  int32_t trm;        // lanes per row of s = M c
  int32_t rkab_bs;    // column-split RKAB: projections per worker (0: RKA)
  int32_t rkab_c;     // column-split RKAB: projections per worker per block (c <= bs)
  int32_t nsub;       // column-split RKAB: blocks per outer iteration (1: RKA)
  int32_t ncoef_rkab; // column-split RKAB: coefficients per block, workers x c (c - 1) / 2
  uint64_t* part;     // nv_max x G tagged slots, value-major
  uint64_t* red;      // kSumCopies x nv_max tagged slots
  DevStatus* st;
};

// Poll `total` tagged slots, slot idx(L) for L = t + NT s (at most kBPoll per
// lane), until every tag matches, storing the values to dst[L].  A sweep
// issues kBBatch loads per lane before waiting for any; slots already read,
// and lanes past the end, load at `oob`, out of the buffer's range (zero, no
// memory access).  False (in every thread) if the wait gave up.
template <typename IdxFn>
__device__ __forceinline__ bool blk_gather(const TagSlots& sl, int oob, int total, uint32_t tg,
                                           IdxFn idx, double* dst, int t, int NT) {
  const int ns = (total + NT - 1) / NT;
  uint32_t need = 0;
#pragma unroll
  for (int s = 0; s < kBPoll; ++s)
    if (t + NT * s < total) need |= 1u << s;
  for (unsigned spins = 0;; ++spins) {
#pragma unroll
    for (int s0 = 0; s0 < kBPoll; s0 += kBBatch) {
      if (s0 < ns) {
        uint64_t lo[kBBatch], hi[kBBatch];
#pragma unroll
        for (int s = 0; s < kBBatch; ++s) {
          lo[s] = hi[s] = 0;
          if (s0 + s < ns) {
            int Lx = t + NT * (s0 + s);
            __asm__ volatile("" : "+v"(Lx));
            sl.fetch16((need >> (s0 + s)) & 1u ? (int)idx(Lx) : oob, lo[s], hi[s]);
          }
        }
#pragma unroll
        for (int s = 0; s < kBBatch; ++s) {
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
}

// MODE 0: RKA; 1: column-split RKAB, one block per outer iteration; 2:
// column-split RKAB in sub-blocks (every worker's iterate kept for the slice).
// Compile-time, so that each instance carries only its own paths (the RKA
// instances measured 2-4 % slower with the RKAB branches taken at run time).
template <typename T, int V, int RPT, int MODE>
__global__ __launch_bounds__(kBThreads) void rka_blk_kernel(BlkArgs p) {
  using raw_t = typename Vec<T, V>::raw_t;
  if (p.st->done) return;
  const T* __restrict__ A = (const T*)p.A;
  const int t = threadIdx.x, g = blockIdx.x, NT = p.nt;
  const int q = p.q, nsv = p.nsv, rg = p.rg, G = p.G, NSVP = p.nsvp;
  // lane j of row group rgi holds vec j of the slice (lanes j >= nsv idle):
  // a row group is an aligned team of NSVP lanes inside one wave
  const int j = t & (NSVP - 1);
  const int rgi = t / NSVP;
  const bool active = j < nsv;
  const int64_t cv = (int64_t)g * nsv + j;
  const bool colv = active && cv < p.nvec;
  const int64_t cvl = cv < p.nvec ? cv : p.nvec - 1;
  const int Rmax = p.nv_max - 1;

  extern __shared__ double lds[];
  double* MC = lds;                       // cstride  M of the block (16-byte aligned)
  double* HV = MC + p.cstride;            // nv_max   this slice's partials, then the sums
  double* CC = HV + p.nv_max;             // Rmax     c_r, then the scales s_r
  double* RB = CC + Rmax;                 // Rmax     b_r
  double* RW = RB + Rmax;                 // Rmax     ||a_r||^2
  double* RA = RW + Rmax;                 // Rmax     weights
  double* U = RA + Rmax;                  // (NT / 64) * NSVP * V  update sums per wave
  double* XS = U + (size_t)(NT / kWave) * NSVP * V;  // NSVP * V  new slice of x
  double* PG = XS + (size_t)NSVP * V;     // G * ceil(nv_max / G)  gathered partials
  // column-split RKAB in several blocks per outer iteration: every worker's
  // iterate for the slice, and the row groups' update sums
  double* VW = PG + (size_t)G * ((p.nv_max + G - 1) / G);  // q * NSVP * V
  double* UW = VW + (size_t)q * NSVP * V;                   // NT * V
  const int nwaves = NT / kWave;
  const int nsub = MODE == 2 ? p.nsub : 1;

  double xv[V];
#pragma unroll
  for (int e = 0; e < V; ++e) xv[e] = colv ? p.x[cv * V + e] : 0.0;
  if (t < NSVP) {  // the slice's x, kept in LDS: the update adds to it
#pragma unroll
    for (int e = 0; e < V; ++e) XS[t * V + e] = xv[e];
  }
  if constexpr (MODE == 2) {  // every worker starts the outer iteration from x
    __syncthreads();
    for (int i = t; i < q * NSVP * V; i += NT) VW[i] = XS[i % (NSVP * V)];
  }

  // Block b of the chunk: its first chunk-local iteration kl, its length L
  // (iterations; for RKAB the steps of each worker), a test at its start,
  // and its sub-block sb.  RKAB: blocks are the nsub sub-blocks of each
  // outer iteration.  With one block per outer iteration its rows are
  // worker-major (row r = w L + jj), as the records lie; with sub-blocks
  // step-major (row r = jj q + w: worker w's step sb c + jj), so that with
  // q dividing the row groups every row a thread holds belongs to worker
  // rgi mod q (the records then lie bs apart: step-major cost 1.5 us per
  // outer iteration at q = 16, bs = 10, where no sub-blocks need it).
  auto locate = [&](int bb, int* kl_, int* L_, bool* test_, int* sb_) {
    if constexpr (MODE != 0) {
      const int bo = bb / nsub, sb2 = bb - bo * nsub;
      int L1;
      p.lay.locate(bo, kl_, &L1, test_);
      *test_ = *test_ && sb2 == 0;
      *sb_ = sb2;
      *L_ = p.rkab_c < p.rkab_bs - sb2 * p.rkab_c ? p.rkab_c : p.rkab_bs - sb2 * p.rkab_c;
    } else {
      p.lay.locate(bb, kl_, L_, test_);
      *sb_ = 0;
    }
  };
  // the record of row r of a block
  auto recidx = [&](int kl_, int sb_, int r) -> int64_t {
    if constexpr (MODE == 2) {
      const int jj = r / q, w = r - jj * q;
      return ((int64_t)kl_ * q + w) * p.rkab_bs + sb_ * p.rkab_c + jj;
    } else if constexpr (MODE == 1) {
      return (int64_t)kl_ * q * p.rkab_bs + r;
    } else {
      return (int64_t)kl_ * q + r;
    }
  };

  const TagSlots part(p.part, (int64_t)G * p.nv_max);
  const TagSlots red(p.red, (int64_t)kSumCopies * p.nv_max);

  auto load_rows = [&](int kl2, int L2, int sb2, int* rows) {
    const int R2 = L2 * q;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int br = rgi + rg * i;
      rows[i] = (int)p.rec[recidx(kl2, sb2, br < R2 ? br : R2 - 1)].row;
    }
  };
  raw_t a[RPT], an[RPT];
  int rows_n[RPT];
  double mb = 0.0, mw = 1.0, ma = 0.0;  // record of block row t
  int b = 0, kl = 0, L = 1, sb = 0;
  bool check = false;
  locate(0, &kl, &L, &check, &sb);
  const int nblk = p.lay.nblk * nsub;
  {
    int rows0[RPT];
    load_rows(kl, L, sb, rows0);
#pragma unroll
    for (int i = 0; i < RPT; ++i) a[i] = load_raw<T, V>(A + (int64_t)rows0[i] * p.lda + cvl * V);
    if (t < L * q) {
      const RowRec r = p.rec[recidx(kl, sb, t)];
      mb = r.b;
      mw = r.wn;
      ma = r.alpha;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) rows_n[i] = rows0[i];
    if (nblk > 1) {
      int kl1, L1, sb1;
      bool t1;
      locate(1, &kl1, &L1, &t1, &sb1);
      load_rows(kl1, L1, sb1, rows_n);
    }
  }

  bool stopped = false;
  BPROF_DECL
  while (b < nblk) {
    const int64_t k = p.lay.k0 + kl;
    const int R = L * q, nv = R + 1;
    const uint32_t tag = (uint32_t)(k * nsub + sb + 1);  // one per exchange
    if (t < R) {
      RB[t] = mb;
      RW[t] = mw;
      RA[t] = ma;
    }
    // (1) the dot products of the block's rows with this slice of x^(k): a
    // lane's products, then the row group's fixed DPP / swizzle fold
    {
      double sd[RPT];
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        double s = 0.0;
#pragma unroll
        for (int e = 0; e < V; ++e) s = fma(colv ? raw_elem<T, V>(a[i], e) : 0.0, xv[e], s);
        sd[i] = s;
      }
      team_sum_n(sd, NSVP);
      if (j == 0) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int br = rgi + rg * i;
          if (br < R) HV[br] = sd[i];
        }
      }
    }
    if (t < kWave) {  // row group 0's lanes: the error of this slice (0 without a test)
      double s = 0.0;
      if (check && t < NSVP && colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const double d = xv[e] - p.x_ref[cv * V + e];
          s = fma(d, d, s);
        }
      }
      s = team_sum(s, NSVP);
      if (t == 0) HV[R] = s;
    }
    BPROF(0);
    __syncthreads();
    // (2) the nv partials leave, value-major (slot v G + g), so that a
    // reducer's G slots of one value are contiguous
    for (int v = t; v < nv; v += NT) part.put16((int64_t)v * G + g, HV[v], tag);
    // (3) the block's coefficients M (L2-resident) straight into LDS, 16 bytes
    // a lane and 1 KB a wave per load, in flight across the exchange (issued
    // after the barrier above, which would otherwise wait for them)
    {
      const double* Mg = p.coef + (size_t)b * p.cstride;
      const int ncur = MODE != 0 ? p.ncoef_rkab : q * q * (L * (L - 1) / 2);
      const int npieces = (ncur + 127) / 128;  // within cstride
      const int wv = t / kWave, lane = t & (kWave - 1);
      for (int i = wv; i < npieces; i += NT / kWave)
        __builtin_amdgcn_global_load_lds((const void*)(Mg + 128 * i + 2 * lane),
                                         (__attribute__((address_space(3))) void*)(MC + 128 * i),
                                         16, 0, 0);
    }
    BPROF(1);
    // phase 1: workgroup g sums the values [g C, g C + C) over all workgroups
    bool ok = true;
    {
      const int C = (nv + G - 1) / G;
      const int v0 = g * C;
      const int cnt = nv - v0 < C ? (nv - v0 > 0 ? nv - v0 : 0) : C;
      // consecutive lanes poll consecutive slots: L = c G + gg is slot
      // (v0 + c) G + gg
      ok = blk_gather(part, G * p.nv_max, G * cnt, tag,
                      [&](int Lx) { return v0 * G + Lx; }, PG, t, NT);
      const int TR = p.trp, team = t / TR, u = t & (TR - 1);
      double sum = 0.0;
      if (team < cnt)
        for (int gg = u; gg < G; gg += TR) sum += PG[team * G + gg];
      sum = team_sum(sum, TR);  // in every lane of the team
      if (ok && team < cnt)
        for (int c = u; c < kSumCopies; c += TR) red.put16(c * p.nv_max + v0 + team, sum, tag);
    }
    BPROF(2);
    // The next block's rows and records, issued while the other workgroups'
    // phase-1 sums arrive: the issue stalls on the CU's outstanding-load
    // limit wherever it sits, and here the stall overlaps a wait.  Measured
    // at q = 16, p = 8, us per iteration: 1.92 here; 2.02 with the issue at
    // the start of the block (phase 2 no longer waits for the rows, but the
    // stalled issue delays the dot products and partial sums by ~5k
    // cycles); 1.96 with half the rows issued before the partial sums and
    // half here; 2.15 with the issue after the exchange.  Their addresses
    // use the row indices loaded one block earlier.
    int kn = kl, Ln = L, sbn = sb;
    bool checkn = false;
    if (b + 1 < nblk) locate(b + 1, &kn, &Ln, &checkn, &sbn);
#pragma unroll
    for (int i = 0; i < RPT; ++i) an[i] = load_raw<T, V>(A + (int64_t)rows_n[i] * p.lda + cvl * V);
    if (b + 1 < nblk && t < Ln * q) {
      const RowRec r = p.rec[recidx(kn, sbn, t)];
      mb = r.b;
      mw = r.wn;
      ma = r.alpha;
    }
    if (b + 2 < nblk) {
      int kn2, Ln2;
      int sb2;
      bool t2;
      locate(b + 2, &kn2, &Ln2, &t2, &sb2);
      load_rows(kn2, Ln2, sb2, rows_n);
    }
    // phase 2: every workgroup reads all nv sums (from its copy)
    if (__syncthreads_and(ok)) {
      const int cp = (g % kSumCopies) * p.nv_max;
      ok = blk_gather(red, kSumCopies * p.nv_max, nv, tag, [&](int Lx) { return cp + Lx; }, HV,
                      t, NT);
    }
    BPROF(3);
    if (!__syncthreads_and(ok)) {
      if (t == 0) note_timeout(p.st);
      stopped = true;
      break;
    }
    if (check) {
      const double e2 = HV[R];
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
    // This wave's loads of M landed before its phase-1 poll loads returned
    // (loads return in order); the wait makes that explicit at no cost.
    __builtin_amdgcn_s_waitcnt(0);
    // (4) c_r = alpha_r (b_r - <a_r, x^(k)>) / w_r, then s = M c: row r of
    // iteration jr adds M_{r,c} c_c over the jr q rows c of earlier
    // iterations (contiguous in M's row packing); a team of trm lanes per
    // row, lane u taking every trm-th term into four running sums
    if (t < R) CC[t] = RA[t] * (RB[t] - HV[t]) / RW[t];
    __syncthreads();
    double sr = 0.0;
    {
      const int TR = p.trm, r = t / TR, u = t & (TR - 1);
      // row r = jr q + rho's coefficients (contiguous in M) and the rows they
      // multiply: RKA, the jr q rows of earlier iterations; RKAB, worker
      // rho's jr earlier steps of the block, rows l q + rho (M_rho packed at
      // rho c (c - 1) / 2)
      // (one RKAB block per outer iteration: row r = w L + jj, the worker's
      // earlier steps contiguous)
      const int jr = r < R ? r / q : 0, rho = r - jr * q;
      int rowoff, nterm, cstep, cbase;
      if constexpr (MODE == 2) {
        rowoff = rho * (p.rkab_c * (p.rkab_c - 1) / 2) + jr * (jr - 1) / 2;
        nterm = jr;
        cstep = q;
        cbase = rho;
      } else if constexpr (MODE == 1) {
        const int w = r < R ? r / L : 0, jj = r < R ? r - w * L : 0;
        rowoff = w * (p.rkab_c * (p.rkab_c - 1) / 2) + jj * (jj - 1) / 2;
        nterm = jj;
        cstep = 1;
        cbase = w * L;
      } else {
        rowoff = blk_rowoff(q, jr, rho);
        nterm = jr * q;
        cstep = 1;
        cbase = 0;
      }
      const double* mr = MC + rowoff;
      const double* cc = CC + cbase;
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
      int c = u;
      // eight terms' loads in flight before the first multiply-add
      for (; c + 7 * TR < nterm; c += 8 * TR) {
        double mv[8], cv[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          mv[i] = mr[c + i * TR];
          cv[i] = cc[(c + i * TR) * cstep];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) a4[i & 3] = fma(mv[i], cv[i], a4[i & 3]);
      }
      for (; c < nterm; c += TR) a4[0] = fma(mr[c], cc[c * cstep], a4[0]);
      double acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      acc = team_sum(acc, TR);
      if (r < R) sr = CC[r] + acc;
    }
    __syncthreads();
    if ((t & (p.trm - 1)) == 0 && t / p.trm < R) CC[t / p.trm] = sr;
    __syncthreads();
    BPROF(4);
    // (5) x_slice += (1/q) sum over the block's rows of s_r A[i_r, slice]: a
    // lane's rows, then the row groups of a wave (xor folds), then the waves
    // in order
    double uu[V];
#pragma unroll
    for (int e = 0; e < V; ++e) uu[e] = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int br = rgi + rg * i;
      const double s = (colv && br < R) ? CC[br < R ? br : 0] : 0.0;
#pragma unroll
      for (int e = 0; e < V; ++e) uu[e] = fma(s, raw_elem<T, V>(a[i], e), uu[e]);
    }
    if constexpr (MODE == 2) {
      // RKAB in sub-blocks: every row of this thread is worker rgi mod q's,
      // whose iterate takes the sum with weight 1; the row groups of a
      // worker add in order, and the last sub-block of an outer iteration
      // forms x^(k+1) = (1/q) sum_w v_w, from which every worker restarts
      const int SW = NSVP * V;
#pragma unroll
      for (int e = 0; e < V; ++e) UW[rgi * SW + j * V + e] = uu[e];
      __syncthreads();
      for (int i = t; i < q * SW; i += NT) {
        const int w = i / SW, rest = i - w * SW;
        double acc = 0.0;
        for (int gi = w; gi < rg; gi += q) acc += UW[gi * SW + rest];
        VW[i] += acc;
      }
      __syncthreads();
      if (sb == nsub - 1) {
        if (t < SW) {
          double acc = 0.0;
          for (int w = 0; w < q; ++w) acc += VW[w * SW + t];
          XS[t] = acc * p.inv_q;
        }
        __syncthreads();
        for (int i = t; i < q * SW; i += NT) VW[i] = XS[i % SW];
        __syncthreads();
      }
      if (colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) xv[e] = VW[(rgi % q) * SW + j * V + e];
      }
    } else {
      for (int off = NSVP; off < kWave; off *= 2) {
#pragma unroll
        for (int e = 0; e < V; ++e) uu[e] += __shfl_xor(uu[e], off, kWave);
      }
      if ((t & (kWave - 1)) < NSVP) {
#pragma unroll
        for (int e = 0; e < V; ++e) U[((t / kWave) * NSVP + j) * V + e] = uu[e];
      }
      __syncthreads();
      if (t < NSVP * V) {
        const int jj = t / V, e = t - jj * V;
        double acc = 0.0;
        for (int w = 0; w < nwaves; ++w) acc += U[(w * NSVP + jj) * V + e];
        XS[t] = fma(acc, p.inv_q, XS[t]);
      }
      __syncthreads();
      if (colv) {
#pragma unroll
        for (int e = 0; e < V; ++e) xv[e] = XS[j * V + e];
      }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) a[i] = an[i];
    ++b;
    kl = kn;
    L = Ln;
    sb = sbn;
    check = checkn;
    BPROF(5);
  }
#ifdef RKA_BLK_PROF
  if (t == 0 && (g == 0 || g == G / 2))
    printf("blk-prof g=%d blocks=%lld dots=%llu put=%llu phase1=%llu phase2=%llu scales=%llu "
           "update=%llu\n",
           g, (long long)b, (unsigned long long)bp_t[0], (unsigned long long)bp_t[1],
           (unsigned long long)bp_t[2], (unsigned long long)bp_t[3], (unsigned long long)bp_t[4],
           (unsigned long long)bp_t[5]);
#endif
  if (colv && rgi == 0) {
#pragma unroll
    for (int e = 0; e < V; ++e) p.x[cv * V + e] = xv[e];
  }
  if (!stopped && g == 0 && t == 0) p.st->iterations = p.lay.k0 + p.lay.K;
}

// ===========================================================================
// Host side: geometry and launches.
// ===========================================================================
static int pow2_at_most(int v) {
  int r = 1;
  while (r * 2 <= v) r *= 2;
  return r;
}

static size_t blk_lds_bytes_c(int cstride, int Rmax, int nsvp, int V, int NT, int G) {
  const int nv = Rmax + 1;
  size_t d = (size_t)cstride + nv + 4 * Rmax + (size_t)(NT / kWave) * nsvp * V + (size_t)nsvp * V +
             (size_t)G * ((nv + G - 1) / G);
  return d * sizeof(double);
}
static size_t blk_lds_bytes(int q, int p, int nsvp, int V, int NT, int G) {
  return blk_lds_bytes_c((blk_ncoef(q, p) + 127) & ~127, q * p, nsvp, V, NT, G);
}

constexpr size_t kBMaxLds = 150 * 1024;
constexpr int kBMaxRPT = 11;  // 16 rows per thread (two register tiles of them) spill

// Vecs per column slice. With a requested grid: as many as spread the row over
// it. Automatic: one slice per CU, then rounded up to whole 128-byte lines when
// the rows start on lines (consecutive workgroups run on different XCDs, whose
// L2s would each fetch a line two slices share) where that costs at most a
// quarter more vecs, or with `team` to the whole power-of-two team of lanes a
// row group has, where that costs at most 60 % more (at 80000 x 10000 FP64,
// q = 16: RKA 2 % faster with 384-byte slices, RKAB 4-5 % with 512-byte ones).
static int64_t blk_slice_vecs(const SolveShape& sh, int64_t nvec, int vbytes, bool team) {
  const int target = sh.grid > 0 ? sh.grid : sh.num_cu;
  const int64_t nsv = std::max<int64_t>(1, (nvec + target - 1) / target);
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const bool lines = (sh.lda * esz) % 128 == 0 && reinterpret_cast<uintptr_t>(sh.A) % 128 == 0;
  const int64_t lv = std::max(1, 128 / vbytes);
  if (sh.grid > 0 || !lines || nsv < lv || nsv > kWave) return nsv;
  int64_t nsvp = 1;
  while (nsvp < nsv) nsvp *= 2;
  if (team && 5 * nsvp <= 8 * nsv) return nsvp;
  const int64_t al = (nsv + lv - 1) / lv * lv;
  return 4 * al <= 5 * nsv ? al : nsv;
}

bool rka_blk_plan(const SolveShape& sh, int p_req, RkaBlkGeom* geo) {
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  if (sh.acc != 0 || sh.bs != 1) return false;
  const int64_t nvec = sh.vec_ok ? sh.n / V : sh.n;
  const int q = sh.q;
  // rows per block: at most 128 (256 with one iteration per block, which
  // needs no coefficients); by default as many as fit (at 80000 x 10000
  // FP64, q = 16: 2.1 us per iteration with 128 rows, 3.3 us with 64)
  const int rmax = kBMaxRows;
  int p = p_req > 0 ? p_req : std::max(1, rmax / q);
  if (p > 1 && p > rmax / q) p = rmax / q;
  if (p < 1 || (p == 1 && q > 2 * rmax)) return false;
  const int64_t nsv = blk_slice_vecs(sh, nvec, V * esz, false);
  if (nsv > kWave) return false;  // a row group is one team of lanes inside a wave
  const int G = (int)((nvec + nsv - 1) / nsv);
  if (G < 2) return false;  // one slice: no exchange to save
  const int NT = kBThreads;
  int nsvp = 1;
  while (nsvp < nsv) nsvp *= 2;
  const int rg = NT / nsvp;
  // the largest p whose rows fit the register tile and LDS (narrow storage
  // on the vector path: fewer rows per thread, the widened rows taking more
  // registers; the larger tiles spill on gfx950)
  const int rpt_cap = V == 1 ? kBMaxRPT : (sh.dtype == 0 ? kBMaxRPT : (sh.dtype == 1 ? 6 : 4));
  for (; p >= 1; --p) {
    const int R = q * p;
    const int rpt = (R + rg - 1) / rg;
    if (rpt > rpt_cap) continue;
    if (blk_lds_bytes(q, p, nsvp, V, NT, G) > kBMaxLds) continue;
    if (R + 1 > kBPoll * NT || (int64_t)G * ((R + 1 + G - 1) / G) > (int64_t)kBPoll * NT) continue;
    break;
  }
  if (p < 1) return false;
  // left to the library, one iteration per block only where q itself fills
  // a block (q > 64); below, a block cut to one iteration by the register
  // tile is the column kernel's job
  if (p_req == 0 && p == 1 && q <= kBMaxRows / 2) return false;
  const int R = q * p;
  int rpt = (R + rg - 1) / rg;
  const int buckets[] = {1, 2, 3, 4, 6, 8, 11};
  for (int bk : buckets)
    if (rpt <= bk) {
      rpt = bk;
      break;
    }
  geo->G = G;
  geo->nsv = (int)nsv;
  geo->nsvp = nsvp;
  geo->rg = rg;
  geo->nt = NT;
  geo->rpt = rpt;
  geo->p = p;
  geo->nv = R + 1;
  geo->ncoef = blk_ncoef(q, p);
  geo->tr = 1;
  {
    const int C = (R + 1 + G - 1) / G;
    geo->trp = pow2_at_most(std::max(1, std::min(64, NT / C)));
  }
  geo->trm = pow2_at_most(std::max(1, std::min(64, NT / R)));
  geo->lds = blk_lds_bytes(q, p, nsvp, V, NT, G);
  geo->cstride = (geo->ncoef + 127) & ~127;
  // coefficient pass: rows padded to 16, an odd column stride (staging
  // writes of consecutive columns spread over the banks), chunks of
  // 4096 / (rows rounded up to a power of two) columns
  const int RP = 16 * ((R + 15) / 16);
  geo->crs = RP + 1;
  {
    int rp = 1, l = 12;
    while (rp < RP) {
      rp *= 2;
      --l;
    }
    geo->clcw = l;
  }
  // Gram tiles of a full block (those of a shorter block are among them),
  // spread over the waves
  {
    int nt = 0;
    for (int I = 0; I < RP / 16; ++I)
      for (int J = 0; J <= I; ++J)
        if (std::min(16 * I + 15, R - 1) / q > (16 * J) / q) ++nt;
    const int per = (nt + kCWaves - 1) / kCWaves;
    geo->cslots = per <= 2 ? 2 : per <= 3 ? 3 : per <= 4 ? 4 : kCMaxSlots;
  }
  // the staged chunk and N share LDS
  geo->clds = (std::max((size_t)(1 << geo->clcw) * geo->crs, (size_t)blk_ncoef(q, p)) + kBMaxRows) *
                  sizeof(double) + kBMaxRows * sizeof(int64_t);
  if (geo->clds > kBMaxLds) return false;
  // LDS-direct staging: two buffers of (rows rounded to 16) / 2 row pairs
  geo->cbuf = (RP / 2) * kCPairBytes;
  geo->clds_dma = (std::max((size_t)2 * geo->cbuf, (size_t)blk_ncoef(q, p) * sizeof(double)) +
                   kBMaxRows * sizeof(double)) + kBMaxRows * sizeof(int64_t);
  if (geo->clds_dma > kBMaxLds) geo->clds_dma = 0;  // register staging only
  return true;
}

bool rka_blk_plan_rkab(const SolveShape& sh, RkaBlkGeom* geo) {
  const int qw = sh.q, bs = sh.bs;
  if (sh.acc != 0 || bs < 2) return false;
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  const int V = sh.vec_ok ? 16 / esz : 1;
  const int64_t nvec = sh.vec_ok ? sh.n / V : sh.n;
  const int64_t nsv = blk_slice_vecs(sh, nvec, V * esz, true);
  if (nsv > kWave) return false;
  const int G = (int)((nvec + nsv - 1) / nsv);
  if (G < 2) return false;
  const int NT = kBThreads;
  int nsvp = 1;
  while (nsvp < nsv) nsvp *= 2;
  const int rg = NT / nsvp;
  const int rpt_cap = V == 1 ? kBMaxRPT : (sh.dtype == 0 ? kBMaxRPT : (sh.dtype == 1 ? 6 : 4));
  // c steps per worker per block: the whole outer iteration if its q bs rows
  // fit, else nsub sub-blocks of at most c (then every row group must serve
  // one worker: q divides the row groups)
  auto lds_of = [&](int c, int nsub) {
    const int cstride = ((qw * (c * (c - 1) / 2)) + 127) & ~127;
    size_t l = blk_lds_bytes_c(cstride, qw * c, nsvp, V, NT, G);
    if (nsub > 1) l += ((size_t)qw * nsvp * V + (size_t)NT * V) * sizeof(double);
    return l;
  };
  auto fits = [&](int c, int nsub) {
    const int R = qw * c;
    if (R > 2 * kBMaxRows || (R + rg - 1) / rg > rpt_cap) return false;
    if (R + 1 > kBPoll * NT || (int64_t)G * ((R + 1 + G - 1) / G) > (int64_t)kBPoll * NT) return false;
    if (nsub > 1 && rg % qw != 0) return false;
    return lds_of(c, nsub) <= kBMaxLds;
  };
  int c = std::min(bs, kRkabBlkMaxBs);
  for (; c >= 2; --c)
    if (fits(c, (bs + c - 1) / c)) break;
  if (c < 2) return false;
  const int nsub = (bs + c - 1) / c;
  c = (bs + nsub - 1) / nsub;  // balanced sub-blocks (no longer than before: still fits)
  const int R = qw * c;
  int rpt = (R + rg - 1) / rg;
  const int buckets[] = {1, 2, 3, 4, 6, 8, 11};
  for (int bk : buckets)
    if (rpt <= bk) {
      rpt = bk;
      break;
    }
  geo->G = G;
  geo->nsv = (int)nsv;
  geo->nsvp = nsvp;
  geo->rg = rg;
  geo->nt = NT;
  geo->rpt = rpt;
  geo->p = 1;  // blocks are laid out per outer iteration, nsub of them each
  geo->nv = R + 1;
  geo->tr = 1;
  {
    const int C = (R + 1 + G - 1) / G;
    geo->trp = pow2_at_most(std::max(1, std::min(64, NT / C)));
  }
  geo->trm = pow2_at_most(std::max(1, std::min(64, NT / R)));
  geo->rkab_bs = bs;
  geo->rkab_q = qw;
  geo->rkab_c = c;
  geo->rkab_nsub = nsub;
  geo->ncoef = qw * (c * (c - 1) / 2);
  geo->cstride = (geo->ncoef + 127) & ~127;
  geo->lds = lds_of(c, nsub);
  return true;
}

int64_t rka_blk_nblk(const RkaBlkGeom& geo, int64_t k0, int64_t K, int64_t check_every) {
  return BlkLayout::make(k0, K, check_every, geo.p).nblk;
}

template <typename T, int NS, bool DMA>
static hipError_t launch_coef_ns(const RkaBlkGeom& geo, CoefArgs& a, int grid, hipStream_t s) {
  const void* fn = (const void*)blk_coef_kernel<T, NS, DMA>;
  const size_t lds = DMA ? geo.clds_dma : geo.clds;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((blk_coef_kernel<T, NS, DMA>), dim3(grid), dim3(kCThreads), lds, s, a);
  return hipGetLastError();
}

template <typename T, bool DMA>
static hipError_t launch_coef_d(const RkaBlkGeom& geo, CoefArgs& a, int grid, hipStream_t s) {
  switch (geo.cslots) {
    case 2: return launch_coef_ns<T, 2, DMA>(geo, a, grid, s);
    case 3: return launch_coef_ns<T, 3, DMA>(geo, a, grid, s);
    case 4: return launch_coef_ns<T, 4, DMA>(geo, a, grid, s);
    default: return launch_coef_ns<T, kCMaxSlots, DMA>(geo, a, grid, s);
  }
}

// LDS-direct staging on the 16-byte vector path (rows 16-byte aligned, n a
// multiple of the vector), register staging otherwise
template <typename T>
static hipError_t launch_coef_t(const RkaBlkGeom& geo, CoefArgs& a, int grid, bool vec,
                                hipStream_t s) {
  return vec && geo.clds_dma > 0 ? launch_coef_d<T, true>(geo, a, grid, s)
                                 : launch_coef_d<T, false>(geo, a, grid, s);
}

template <typename T, int V, int RPT, int MODE>
static hipError_t launch_blk_t(const RkaBlkGeom& geo, BlkArgs& a, hipStream_t s) {
  const void* fn = (const void*)rka_blk_kernel<T, V, RPT, MODE>;
  if (geo.lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)geo.lds);
    if (e != hipSuccess) return e;
  }
  void* args[] = {&a};
  return launch_persistent(fn, dim3(geo.G), dim3(geo.nt), args, (unsigned)geo.lds, s);
}

template <typename T, int V, int MODE>
static hipError_t launch_blk_rpt_s(const RkaBlkGeom& geo, BlkArgs& a, hipStream_t s) {
  switch (geo.rpt) {
    case 1: return launch_blk_t<T, V, 1, MODE>(geo, a, s);
    case 2: return launch_blk_t<T, V, 2, MODE>(geo, a, s);
    case 3: return launch_blk_t<T, V, 3, MODE>(geo, a, s);
    case 4: return launch_blk_t<T, V, 4, MODE>(geo, a, s);
    case 6: return launch_blk_t<T, V, 6, MODE>(geo, a, s);
    case 8: return launch_blk_t<T, V, 8, MODE>(geo, a, s);
    default: return launch_blk_t<T, V, 11, MODE>(geo, a, s);
  }
}

template <typename T, int V>
static hipError_t launch_blk_rpt(const RkaBlkGeom& geo, BlkArgs& a, hipStream_t s) {
  if (!geo.rkab_bs) return launch_blk_rpt_s<T, V, 0>(geo, a, s);
  return geo.rkab_nsub > 1 ? launch_blk_rpt_s<T, V, 2>(geo, a, s)
                           : launch_blk_rpt_s<T, V, 1>(geo, a, s);
}

template <typename T, int V, int BS>
static hipError_t launch_coef_rkab_bs(CoefRkabArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((blk_coef_rkab_kernel<T, V, BS>), dim3(grid), dim3(kRThreads), 0, s, a);
  return hipGetLastError();
}

template <typename T, int V>
static hipError_t launch_coef_rkab_t(CoefRkabArgs& a, int bs, int grid, hipStream_t s) {
  switch (bs) {
    case 2: return launch_coef_rkab_bs<T, V, 2>(a, grid, s);
    case 3: return launch_coef_rkab_bs<T, V, 3>(a, grid, s);
    case 4: return launch_coef_rkab_bs<T, V, 4>(a, grid, s);
    case 5: return launch_coef_rkab_bs<T, V, 5>(a, grid, s);
    case 6: return launch_coef_rkab_bs<T, V, 6>(a, grid, s);
    case 7: return launch_coef_rkab_bs<T, V, 7>(a, grid, s);
    case 8: return launch_coef_rkab_bs<T, V, 8>(a, grid, s);
    case 9: return launch_coef_rkab_bs<T, V, 9>(a, grid, s);
    case 10: return launch_coef_rkab_bs<T, V, 10>(a, grid, s);
    case 11: return launch_coef_rkab_bs<T, V, 11>(a, grid, s);
    default: return launch_coef_rkab_bs<T, V, kRkabBlkMaxBs>(a, grid, s);
  }
}

static hipError_t launch_blk_coef_rkab(const SolveShape& sh, const RkaBlkGeom& geo,
                                       const RowRec* rec, int64_t k0, int64_t K,
                                       int64_t check_every, double* coef, const DevStatus* st,
                                       hipStream_t s) {
  const BlkLayout lay = BlkLayout::make(k0, K, check_every, 1);
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  CoefRkabArgs a{};
  a.A = sh.A;
  a.lda = sh.lda;
  a.nvec = sh.vec_ok ? sh.n / (16 / esz) : sh.n;
  a.rec = rec;
  a.lay = lay;
  a.q = geo.rkab_q;
  a.bs = geo.rkab_bs;
  a.nsub = geo.rkab_nsub;
  a.cstride = geo.cstride;
  a.coef = coef;
  a.st = st;
  const int64_t ntask = lay.nblk * (int64_t)geo.rkab_nsub * geo.rkab_q;
  const int grid = (int)std::min<int64_t>(ntask, (int64_t)sh.num_cu * 8);
  if (grid < 1) return hipSuccess;
  const int bs = geo.rkab_c;
  switch (sh.dtype) {
    case 0:
      return sh.vec_ok ? launch_coef_rkab_t<double, 2>(a, bs, grid, s)
                       : launch_coef_rkab_t<double, 1>(a, bs, grid, s);
    case 1:
      return sh.vec_ok ? launch_coef_rkab_t<float, 4>(a, bs, grid, s)
                       : launch_coef_rkab_t<float, 1>(a, bs, grid, s);
    default:
      return sh.vec_ok ? launch_coef_rkab_t<bf16_t, 8>(a, bs, grid, s)
                       : launch_coef_rkab_t<bf16_t, 1>(a, bs, grid, s);
  }
}

hipError_t launch_blk_coef(const SolveShape& sh, const RkaBlkGeom& geo, const RowRec* rec,
                           int64_t k0, int64_t K, int64_t check_every, double* coef,
                           const DevStatus* st, hipStream_t s) {
  if (geo.rkab_bs > 0)
    return launch_blk_coef_rkab(sh, geo, rec, k0, K, check_every, coef, st, s);
  if (geo.p <= 1) return hipSuccess;  // one iteration per block: no coefficients
  const BlkLayout lay = BlkLayout::make(k0, K, check_every, geo.p);
  const int64_t nblk = lay.nblk;
  CoefArgs c{};
  c.A = sh.A;
  c.lda = sh.lda;
  c.n = sh.n;
  c.rec = rec;
  c.lay = lay;
  c.q = sh.q;
  c.RS = geo.crs;
  c.lcw = geo.clcw;
  c.cstride = geo.cstride;
  c.inv_q = 1.0 / (double)sh.q;
  c.coef = coef;
  c.ncoef = geo.ncoef;
  c.cbuf = geo.cbuf;
  c.st = st;
  const int grid = (int)std::min<int64_t>(nblk, (int64_t)sh.num_cu * 4);
  switch (sh.dtype) {
    case 0: return launch_coef_t<double>(geo, c, grid, sh.vec_ok, s);
    case 1: return launch_coef_t<float>(geo, c, grid, sh.vec_ok, s);
    default: return launch_coef_t<bf16_t>(geo, c, grid, sh.vec_ok, s);
  }
}

hipError_t launch_blk_iter(const SolveShape& sh, const RkaBlkGeom& geo, const RowRec* rec,
                           int64_t k0, int64_t K, int64_t check_every, const double* coef,
                           uint64_t* part, uint64_t* red, DevStatus* st, hipStream_t s) {
  const BlkLayout lay = BlkLayout::make(k0, K, check_every, geo.p);
  const int esz = sh.dtype == 0 ? 8 : (sh.dtype == 1 ? 4 : 2);
  BlkArgs a{};
  a.A = sh.A;
  a.lda = sh.lda;
  a.nvec = sh.vec_ok ? sh.n / (16 / esz) : sh.n;
  a.rec = rec;
  a.coef = coef;
  a.x = sh.x;
  a.x_ref = sh.x_ref;
  // column-split RKAB: a block is one outer iteration of q bs rows, and the
  // update averages over the q workers
  a.inv_q = 1.0 / (double)(geo.rkab_bs ? geo.rkab_q : sh.q);
  a.lay = lay;
  a.q = geo.rkab_bs ? geo.rkab_q : sh.q;  // RKAB: rows step-major, q workers per step
  a.rkab_bs = geo.rkab_bs;
  a.rkab_c = geo.rkab_c;
  a.nsub = geo.rkab_bs ? geo.rkab_nsub : 1;
  a.ncoef_rkab = geo.rkab_bs ? geo.ncoef : 0;
  a.nsv = geo.nsv;
  a.nsvp = geo.nsvp;
  a.rg = geo.rg;
  a.G = geo.G;
  a.nt = geo.nt;
  a.nv_max = geo.nv;
  a.cstride = geo.cstride;
  a.tr = geo.tr;
  a.trp = geo.trp;
  a.trm = geo.trm;
  a.part = part;
  a.red = red;
  a.st = st;
  switch (sh.dtype) {
    case 0:
      return sh.vec_ok ? launch_blk_rpt<double, 2>(geo, a, s) : launch_blk_rpt<double, 1>(geo, a, s);
    case 1:
      return sh.vec_ok ? launch_blk_rpt<float, 4>(geo, a, s) : launch_blk_rpt<float, 1>(geo, a, s);
    default:
      return sh.vec_ok ? launch_blk_rpt<bf16_t, 8>(geo, a, s) : launch_blk_rpt<bf16_t, 1>(geo, a, s);
  }
}

}  // namespace rka
