// rka_dense.hip -- the dense FP64 steps around the Kaczmarz solves: the
// refinement residual r = b - A x and the normal-equations right-hand side
// g = A^T r (one streaming pass over the matrix each), the explicit
// transpose that turns columns of A into contiguous rows (so that the column
// solves stream coalesced rows like the row solves), x += d, fixed-order
// sums of squares for the stopping measures, and the rank-2 gradient
// dA = r lambda^T - z x^T of the differentiable solve.
//
// Every sum has a fixed order for a given shape, so results are bitwise
// reproducible.
#include <math.h>

#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

// ---------------------------------------------------------------------------
// out_i = (c ? c_i : 0) + gamma * <M_i, v>, FP64 accumulation.  One wave per
// row (4 rows per block); lane l takes vecs l, l + 64, ... of the row and the
// 64 lane sums meet in the xor butterfly.  Row data are read once.
// ---------------------------------------------------------------------------
constexpr int kGemvRowsPerBlock = 4;

template <typename T, int V>
__global__ __launch_bounds__(256) void gemv_kernel(const T* __restrict__ M, int64_t rows,
                                                   int64_t nvec, int64_t ld,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ c, double gamma,
                                                   double* __restrict__ out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t row = (int64_t)blockIdx.x * kGemvRowsPerBlock + (threadIdx.x / kWave);
  if (row >= rows) return;  // uniform over the wave
  const T* Mr = M + row * ld;
  double d0 = 0.0, d1 = 0.0;
  int64_t cv = lane;
  // two independent chains keep two loads in flight per lane
  for (; cv + kWave < nvec; cv += 2 * kWave) {
    const auto r0 = load_raw<T, V>(Mr + cv * V);
    const auto r1 = load_raw<T, V>(Mr + (cv + kWave) * V);
#pragma unroll
    for (int e = 0; e < V; ++e) d0 = fma(raw_elem<T, V>(r0, e), v[cv * V + e], d0);
#pragma unroll
    for (int e = 0; e < V; ++e) d1 = fma(raw_elem<T, V>(r1, e), v[(cv + kWave) * V + e], d1);
  }
  if (cv < nvec) {
    const auto r0 = load_raw<T, V>(Mr + cv * V);
#pragma unroll
    for (int e = 0; e < V; ++e) d0 = fma(raw_elem<T, V>(r0, e), v[cv * V + e], d0);
  }
  const double d = wave_sum(d0 + d1);
  if (lane == 0) out[row] = (c ? c[row] : 0.0) + gamma * d;
}

template <typename T, int V>
static hipError_t launch_gemv_t(const void* M, int64_t rows, int64_t cols, int64_t ld,
                                const double* v, const double* c, double gamma, double* out,
                                hipStream_t s) {
  const int64_t nb = (rows + kGemvRowsPerBlock - 1) / kGemvRowsPerBlock;
  hipLaunchKernelGGL((gemv_kernel<T, V>), dim3((unsigned)nb), dim3(256), 0, s, (const T*)M, rows,
                     cols / V, ld, v, c, gamma, out);
  return hipGetLastError();
}

hipError_t launch_gemv(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                       bool vec_ok, const double* v, const double* c, double gamma, double* out,
                       hipStream_t s) {
  switch (dtype) {
    case 0:
      return vec_ok ? launch_gemv_t<double, 2>(M, rows, cols, ld, v, c, gamma, out, s)
                    : launch_gemv_t<double, 1>(M, rows, cols, ld, v, c, gamma, out, s);
    case 1:
      return vec_ok ? launch_gemv_t<float, 4>(M, rows, cols, ld, v, c, gamma, out, s)
                    : launch_gemv_t<float, 1>(M, rows, cols, ld, v, c, gamma, out, s);
    default:
      return vec_ok ? launch_gemv_t<bf16_t, 8>(M, rows, cols, ld, v, c, gamma, out, s)
                    : launch_gemv_t<bf16_t, 1>(M, rows, cols, ld, v, c, gamma, out, s);
  }
}

// ---------------------------------------------------------------------------
// At[j, i] = A[i, j], raw element copy through a padded 64 x 64 LDS tile:
// both the reads (along rows of A) and the writes (along rows of At) are
// contiguous per wave.
// ---------------------------------------------------------------------------
template <typename E>
__global__ __launch_bounds__(256) void transpose_kernel(const E* __restrict__ A, int64_t m,
                                                        int64_t n, int64_t lda, E* __restrict__ At,
                                                        int64_t ldat) {
  __shared__ E tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int k = ty; k < 64; k += 4) {
    const int64_t r = r0 + k, c = c0 + tx;
    if (r < m && c < n) tile[k][tx] = A[r * lda + c];
  }
  __syncthreads();
  for (int k = ty; k < 64; k += 4) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (c < n && r < m) At[c * ldat + r] = tile[tx][k];
  }
}

hipError_t launch_transpose(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, void* At,
                            int64_t ldat, hipStream_t s) {
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((m + 63) / 64));
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(transpose_kernel<uint64_t>, grid, dim3(256), 0, s, (const uint64_t*)A, m,
                         n, lda, (uint64_t*)At, ldat);
      break;
    case 1:
      hipLaunchKernelGGL(transpose_kernel<uint32_t>, grid, dim3(256), 0, s, (const uint32_t*)A, m,
                         n, lda, (uint32_t*)At, ldat);
      break;
    default:
      hipLaunchKernelGGL(transpose_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t*)A, m,
                         n, lda, (uint16_t*)At, ldat);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// x += d
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void axpy_kernel(double* __restrict__ x,
                                                   const double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += d[i];
}

hipError_t launch_axpy(double* x, const double* d, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, d, n);
  return hipGetLastError();
}

// Zero `words` 8-byte words (a kernel rather than a memset node, so that the
// solve's launch sequence holds kernels and copies only).
__global__ __launch_bounds__(256) void zero_kernel(uint64_t* __restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t words = (int64_t)(bytes / 8);
  if (words == 0) return hipSuccess;
  int64_t nb = (words + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)nb), dim3(256), 0, s, (uint64_t*)p, words);
  return hipGetLastError();
}

// out = a - b
__global__ __launch_bounds__(256) void sub_kernel(double* __restrict__ out,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(sub_kernel, dim3((unsigned)nb), dim3(256), 0, s, out, a, b, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out[0] = sum_i (a_i - b_i)^2 (b may be NULL): per-block fixed-order partial
// sums, then one block adds the partials in block order.
// ---------------------------------------------------------------------------
constexpr int kSumsqBlocks = 256;

__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ a,
                                                    const double* __restrict__ b, int64_t len,
                                                    double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = b ? a[i] - b[i] : a[i];
    s = fma(d, d, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void sumsq_finish_kernel(const double* __restrict__ part, int nb,
                                                           double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = s;
}

int sumsq_part_len() { return kSumsqBlocks; }

hipError_t launch_sumsq(const double* a, const double* b, int64_t len, double* part, double* out,
                        hipStream_t s) {
  int64_t nb = (len + 255) / 256;
  if (nb > kSumsqBlocks) nb = kSumsqBlocks;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)nb), dim3(256), 0, s, a, b, len, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sumsq_finish_kernel, dim3(1), dim3(256), 0, s, part, (int)nb, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dA[i, j] = r_i lambda_j - z_i x_j, formed in FP64 and stored as O.
// One block per row (grid-strided), threads along the row.
// ---------------------------------------------------------------------------
template <typename O>
__global__ __launch_bounds__(256) void rank2_kernel(int64_t m, int64_t n,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ x,
                                                    O* __restrict__ out, int64_t ldo) {
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const double ri = r[i], zi = z[i];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
      out[i * ldo + j] = (O)(ri * lam[j] - zi * x[j]);
  }
}

hipError_t launch_rank2(int64_t m, int64_t n, const double* r, const double* lam, const double* z,
                        const double* x, void* out, int out_dtype, int64_t ldo, hipStream_t s) {
  const unsigned nb = (unsigned)(m < 65536 ? m : 65536);
  if (out_dtype == 0)
    hipLaunchKernelGGL(rank2_kernel<double>, dim3(nb), dim3(256), 0, s, m, n, r, lam, z, x,
                       (double*)out, ldo);
  else
    hipLaunchKernelGGL(rank2_kernel<float>, dim3(nb), dim3(256), 0, s, m, n, r, lam, z, x,
                       (float*)out, ldo);
  return hipGetLastError();
}

}  // namespace rka
