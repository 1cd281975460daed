// rka_device.hpp -- device-side building blocks shared by the RKA/RKAB
// kernels for gfx950 (CDNA4): 16-byte row loads for every storage type,
// Philox4x32-10, deterministic wave/workgroup reductions, and a grid barrier
// for persistent (cooperatively launched) kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rka {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Storage types.  Narrow types are widened exactly to double before use.
// bf16 is carried as its raw 16-bit pattern (upper half of a binary32).
// ---------------------------------------------------------------------------
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(bf16_t v) {
  return (double)__uint_as_float((uint32_t)v.bits << 16);
}

// Widening to an accumulation type C (double, or float for narrow storage):
// exact for every storage type a C instance accepts.
template <typename C>
__device__ __forceinline__ C widen_c(double v) {
  return (C)v;
}
template <typename C>
__device__ __forceinline__ C widen_c(float v) {
  return (C)v;
}
template <typename C>
__device__ __forceinline__ C widen_c(bf16_t v) {
  return (C)__uint_as_float((uint32_t)v.bits << 16);
}

// A "vec" is the unit one lane loads from a row: V elements of T, which is
// 16 bytes on the vector path and one element on the scalar path.
template <typename T, int V>
struct Vec {
  static constexpr int kBytes = (int)sizeof(T) * V;
  static_assert(kBytes == 16 || V == 1, "vector path loads 16 bytes");
  using raw_t = typename std::conditional<
      kBytes == 16, uint4,
      typename std::conditional<kBytes == 8, uint2,
                                typename std::conditional<kBytes == 4, uint32_t, uint16_t>::type>::
          type>::type;
};

template <typename T, int V>
__device__ __forceinline__ typename Vec<T, V>::raw_t load_raw(const T* p) {
  return *reinterpret_cast<const typename Vec<T, V>::raw_t*>(p);
}

// Element e (0 <= e < V) of a raw vec, widened to double.
template <typename T, int V>
__device__ __forceinline__ double raw_elem(const typename Vec<T, V>::raw_t& r, int e) {
  union {
    typename Vec<T, V>::raw_t raw;
    T el[V];
  } u;
  u.raw = r;
  return widen(u.el[e]);
}

// Element e of a raw vec, widened to the accumulation type C.
template <typename C, typename T, int V>
__device__ __forceinline__ C raw_elem_c(const typename Vec<T, V>::raw_t& r, int e) {
  union {
    typename Vec<T, V>::raw_t raw;
    T el[V];
  } u;
  u.raw = r;
  return widen_c<C>(u.el[e]);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Counter for the row
// stream: (k_lo, k_hi, worker, j | dom << 24); key: (seed_lo, seed_hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint2 key) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * ctr.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, ctr.x);
    const uint32_t lo1 = 0xCD9E8D57u * ctr.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, ctr.z);
    ctr = make_uint4(hi1 ^ ctr.y ^ key.x, lo1, hi0 ^ ctr.w ^ key.y, lo0);
    key.x += 0x9E3779B9u;
    key.y += 0xBB67AE85u;
  }
  return ctr;
}

// 53-bit uniform in [0, 1) from the first two output words.
__device__ __forceinline__ double draw_uniform(uint64_t seed, uint64_t k, uint32_t w, uint32_t j,
                                               uint32_t dom) {
  const uint4 ctr = make_uint4((uint32_t)k, (uint32_t)(k >> 32), w, j | (dom << 24));
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  const uint4 r = philox4x32_10(ctr, key);
  const uint64_t bits = (((uint64_t)r.x << 32) | (uint64_t)r.y) >> 11;
  return (double)bits * 0x1.0p-53;
}

// Inverse-CDF pick of Eq. (4): t = u * W (one rounded multiply), the smallest
// l with c_l > t; if there is none (t rounded up to W), `last` -- the largest
// row with a positive weight.
__device__ __forceinline__ int64_t pick_row(const double* __restrict__ c, int64_t m, double W,
                                            double u, int64_t last) {
  const double tt = __dmul_rn(u, W);
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (c[mid] > tt)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo < m ? lo : last;
}

// ---------------------------------------------------------------------------
// Deterministic reductions.  The xor butterfly combines the same pairs in
// the same tree on every lane, so every lane ends with the bitwise-same sum.
// Blocks must be a whole number of waves.
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ U wave_sum(U v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Lane exchanges for team reductions.  Within a row of 16 lanes the data
// moves through DPP (a VALU operand modifier, no LDS round trip): quad
// permutes [1,0,3,2] and [2,3,0,1], then the half-row and row mirrors
// (lane i <-> 7 - i within 8, i <-> 15 - i within 16).  Across rows:
// ds_swizzle (xor 16 within 32 lanes) and a full-wave permute (xor 32).
constexpr int kDppQuadXor1 = 0xB1;
constexpr int kDppQuadXor2 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;
constexpr int kSwizzleXor16 = 0x1F | (0x10 << 10);

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = dpp_u32<CTRL>((uint32_t)b), hi = dpp_u32<CTRL>((uint32_t)(b >> 32));
  return __builtin_bit_cast(double, (hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp_u32<CTRL>(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double swizzle_xor16(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)b, kSwizzleXor16);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(b >> 32), kSwizzleXor16);
  return __builtin_bit_cast(double, (hi << 32) | lo);
}
__device__ __forceinline__ float swizzle_xor16(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), kSwizzleXor16));
}

// Sum over aligned teams of tr lanes (tr a power of two <= 64, uniform over
// the wave): every lane of a team receives its team's sum, and the order of
// the additions is fixed (a + b == b + a exactly, so partners agree).  All
// lanes of the wave must take part.
template <typename U>
__device__ __forceinline__ U team_sum(U v, int tr) {
  if (tr >= 2) v += dpp_move<kDppQuadXor1>(v);
  if (tr >= 4) v += dpp_move<kDppQuadXor2>(v);
  if (tr >= 8) v += dpp_move<kDppRowHalfMirror>(v);
  if (tr >= 16) v += dpp_move<kDppRowMirror>(v);
  if (tr >= 32) v += swizzle_xor16(v);
  if (tr >= 64) v += __shfl_xor(v, 32, kWave);
  return v;
}

// team_sum of N independent values, step by step (the N exchanges of a step
// are in flight together).
template <typename U, int N>
__device__ __forceinline__ void team_sum_n(U (&v)[N], int tr) {
  if (tr >= 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppQuadXor1>(v[i]);
  }
  if (tr >= 4) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppQuadXor2>(v[i]);
  }
  if (tr >= 8) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppRowHalfMirror>(v[i]);
  }
  if (tr >= 16) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += dpp_move<kDppRowMirror>(v[i]);
  }
  if (tr >= 32) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += swizzle_xor16(v[i]);
  }
  if (tr >= 64) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 32, kWave);
  }
}

// Sum over the block; every thread receives the same value.  `scratch` holds
// at least blockDim.x / 64 values of LDS and is free for reuse on return.
template <typename U>
__device__ __forceinline__ U block_sum(U v, U* scratch) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  U s = 0;
  for (int i = 0; i < nw; ++i) s += scratch[i];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Coherent (agent-scope) loads and stores for data exchanged between
// workgroups that may sit on different XCDs (each XCD has its own L2).
// ---------------------------------------------------------------------------
template <typename U>
__device__ __forceinline__ U load_agent(const U* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename U>
__device__ __forceinline__ void store_agent(U* p, U v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bulk device-coherent access: raw buffer loads/stores carrying the SC1
// cache-policy bit, which makes them coherent at device scope across XCDs.
// Unlike atomic loads they are ordinary loads to the compiler, so many can be
// in flight at once.  Out-of-range offsets read 0 / drop the write.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr int kCoherentSC1 = 1 << 4;       // buffer cache policy: device scope
constexpr int kRawBufferWord3 = 0x00020000;  // gfx9 raw-buffer descriptor word 3

struct CoherentBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ CoherentBuf(const double* base, int64_t count)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0,
                                            (int)(count * 8), kRawBufferWord3)) {}
  __device__ __forceinline__ double load(int64_t i) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 8), 0,
                                                                           kCoherentSC1));
  }
  __device__ __forceinline__ void store(int64_t i, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)(i * 8), 0,
                                          kCoherentSC1);
  }
};

// The same for 4-byte elements (FP32 worker iterates).
struct CoherentBuf32 {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ CoherentBuf32(const float* base, int64_t count)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)(count * 4),
                                            kRawBufferWord3)) {}
  __device__ __forceinline__ float load(int64_t i) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(i * 4), 0,
                                                                         kCoherentSC1));
  }
  __device__ __forceinline__ void store(int64_t i, float v) const {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)(i * 4), 0,
                                          kCoherentSC1);
  }
};
template <typename U>
using CoherentOf = typename std::conditional<sizeof(U) == 8, CoherentBuf, CoherentBuf32>::type;

// Tagged exchange slots: a double travels as two 64-bit words, each holding
// 32 payload bits and a 32-bit tag (the iteration it belongs to).  A word is
// written with one aligned 8-byte device-coherent store, which lands
// whole, so a reader that sees both tags equal to the expected one has the
// value -- no separate flag, counter or store acknowledgement is needed.
// Slots start zeroed (tag 0 never matches: tags are iteration + 1).
struct TagSlots {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ TagSlots(uint64_t* base, int64_t nslots)
      : r(__builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)(nslots * 16), kRawBufferWord3)) {}
  __device__ __forceinline__ void put(int64_t i, double v, uint32_t tag) const {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t lo = ((uint64_t)tag << 32) | (b & 0xffffffffull);
    const uint64_t hi = ((uint64_t)tag << 32) | (b >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, lo), r, (int)(i * 16), 0,
                                          kCoherentSC1);
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, hi), r, (int)(i * 16 + 8), 0,
                                          kCoherentSC1);
  }
  __device__ __forceinline__ void fetch(int64_t i, uint64_t& lo, uint64_t& hi) const {
    lo = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 16), 0,
                                                                          kCoherentSC1));
    hi = __builtin_bit_cast(uint64_t, __builtin_amdgcn_raw_buffer_load_b64(r, (int)(i * 16 + 8), 0,
                                                                          kCoherentSC1));
  }
  // The same slot written or read with one 16-byte access.  Each word still
  // carries its own tag, so an access that lands in two halves is harmless:
  // the reader simply sees one half early and polls again.
  __device__ __forceinline__ void put16(int64_t i, double v, uint32_t tag) const {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const u32x4_t w = {(uint32_t)(b & 0xffffffffull), tag, (uint32_t)(b >> 32), tag};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)(i * 16), 0, kCoherentSC1);
  }
  __device__ __forceinline__ void fetch16(int64_t i, uint64_t& lo, uint64_t& hi) const {
    const u32x4_t w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(i * 16), 0, kCoherentSC1);
    lo = ((uint64_t)w[1] << 32) | w[0];
    hi = ((uint64_t)w[3] << 32) | w[2];
  }
  static __device__ __forceinline__ bool decode(uint64_t lo, uint64_t hi, uint32_t tag, double& v) {
    if ((uint32_t)(lo >> 32) != tag || (uint32_t)(hi >> 32) != tag) return false;
    v = __builtin_bit_cast(double, ((hi & 0xffffffffull) << 32) | (lo & 0xffffffffull));
    return true;
  }
};

// Upper bound on polling rounds of any wait (each round sleeps ~64 clocks):
// a wait that exceeds it records kStatusTimeout and the kernel winds down
// instead of hanging.
constexpr unsigned kSpinLimit = 1u << 22;
constexpr int kStatusTimeout = -5;  // reported as RKA_EDEVICE

// One sampled row as the iteration kernels consume it: the sampler writes
// the right-hand side entry, the squared norm and the relaxation weight of
// the drawing worker next to the index, so that a kernel gets everything
// with one 32-byte read.
struct alignas(16) RowRec {
  double b;
  double wn;
  int64_t row;
  double alpha;
};

// Wait until every memory operation this wave has issued -- in particular
// its agent-coherent stores -- has completed.  On gfx9 loads and stores
// share one counter, so this also drains the wave's outstanding loads:
// issue prefetches after it, not before.
__device__ __forceinline__ void wait_memory() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Grid barrier for a cooperatively launched grid of `nblocks` workgroups
// (all co-resident).  Protocol: data that other workgroups read after the
// barrier is written with store_agent() and every writing wave calls
// wait_memory() before arriving; readers use load_agent().  Agent-coherent
// accesses go to the coherence point shared by all XCDs, so no L2
// write-back or invalidate is needed (those cost ~40 us per barrier at 256
// workgroups on MI355X).  `ctr` (kGridBarCounters words) is zeroed before the
// launch; `epoch` (barriers passed) advances identically in every workgroup.
//
// Word 0 counts arrivals.  The workgroup whose arrival completes the count
// writes the epoch into kBarGroups release flags, each on a 128-byte line of
// its own (word 32 (1 + k)), and workgroup g polls flag g % kBarGroups (with
// workgroups dealt round-robin over the XCDs, the workgroups of one XCD).
// When every workgroup polled the counter itself, the polls and the
// arrivals' atomics met on one line: at 256 workgroups the last workgroup to
// arrive saw the release ~8 us after its own arrival (2-3 us at 64).
constexpr int kBarGroups = 8;
constexpr int kGridBarCounters = 32 * (1 + kBarGroups);
// The barrier in two halves, so that a workgroup can issue work between its
// arrival and its wait: grid_arrive (every thread calls it, after its
// wait_memory) and grid_wait (every thread; false in every thread if the wait
// gave up).
__device__ __forceinline__ void grid_arrive(unsigned* ctr, unsigned& epoch, unsigned nblocks) {
  ++epoch;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned before =
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (before == epoch * nblocks - 1) {  // the last arrival: every data write is complete
#pragma unroll
      for (int k = 0; k < kBarGroups; ++k) store_agent(ctr + 32 * (1 + k), epoch);
    }
  }
}
__device__ __forceinline__ bool grid_wait(unsigned* ctr, unsigned epoch, unsigned nblocks) {
  (void)nblocks;
  __shared__ int timed_out;
  if (threadIdx.x == 0) {
    const unsigned* flag = ctr + 32 * (1 + blockIdx.x % kBarGroups);
    unsigned spins = 0;
    while (load_agent(flag) < epoch && ++spins < kSpinLimit) __builtin_amdgcn_s_sleep(1);
    timed_out = spins >= kSpinLimit;
  }
  __syncthreads();
  return !timed_out;
}
__device__ __forceinline__ bool grid_arrive_wait(unsigned* ctr, unsigned& epoch,
                                                 unsigned nblocks) {
  grid_arrive(ctr, epoch, nblocks);
  return grid_wait(ctr, epoch, nblocks);
}

// All workgroups of the grid (one workgroup: a block barrier), for callers
// that have nothing to overlap with the wait.
__device__ __forceinline__ bool sync_grid(unsigned* ctr, unsigned& epoch, unsigned nblocks) {
  wait_memory();
  if (nblocks > 1) return grid_arrive_wait(ctr, epoch, nblocks);
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// Solve status kept on the device across the kernels of one solve.
// ---------------------------------------------------------------------------
struct DevStatus {
  int64_t iterations;  // outer iterations completed
  int32_t done;        // nonzero: stop (converged, diverged or failed)
  int32_t status;      // rka_status value
  double rel2;         // last squared relative measure
  double ref2;         // squared norm of the measure's denominator
  double thresh2;      // tol^2 * ref2
  int64_t last_pos;    // largest row with a positive weight
};

// Record that a wait gave up (the solve then reports RKA_EDEVICE).
__device__ __forceinline__ void note_timeout(DevStatus* st) {
  __hip_atomic_store(&st->status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&st->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace rka
