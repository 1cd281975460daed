// rka_spectral.hip -- the extreme eigenvalues of A^T A on the device, for
// the optimal weight alpha* of Eq. (6) (Sec. 2.3.1), which needs
// s = sigma^2(A) / ||A||_F^2 at both ends of the spectrum.  The paper obtains
// them from a full SVD (Table 2: ~2500 s on 64 CPU cores at 80000 x 10000);
// here a Lanczos iteration on A^T A with full reorthogonalisation needs two
// streaming passes over A per step (A v, then A^T t), and the extreme Ritz
// values of the small tridiagonal matrix come from Sturm-sequence bisection
// on the host.
//
// A^T t is formed without a transposed copy: blocks of rows produce partial
// column sums (coalesced along the rows), which are then added in block
// order -- a fixed order, so the result is bitwise reproducible.
#include <math.h>
#include <string.h>

#include <vector>

#include "rka.h"
#include "rka_device.hpp"
#include "rka_internal.hpp"

namespace rka {

constexpr int kTRows = 512;  // rows per partial block of A^T t

// part[blk * n + c] = sum over rows i of block blk of M[i, c] t_i
template <typename T>
__global__ __launch_bounds__(256) void gemvt_partial_kernel(const T* __restrict__ M, int64_t rows,
                                                            int64_t cols, int64_t ld,
                                                            const double* __restrict__ t,
                                                            double* __restrict__ part) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * kTRows;
  const int64_t r1 = r0 + kTRows < rows ? r0 + kTRows : rows;
  if (c >= cols) return;
  double acc = 0.0;
  for (int64_t i = r0; i < r1; ++i) acc = fma(widen(M[i * ld + c]), t[i], acc);
  part[(int64_t)blockIdx.y * cols + c] = acc;
}

// out_c = (c_in ? c_in[c] : 0) + gamma * sum_blk part[blk * n + c]
__global__ __launch_bounds__(256) void gemvt_finish_kernel(const double* __restrict__ part,
                                                           int64_t nblk, int64_t cols,
                                                           const double* __restrict__ cin,
                                                           double gamma,
                                                           double* __restrict__ out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblk; ++b) s += part[b * cols + c];
  out[c] = (cin ? cin[c] : 0.0) + gamma * s;
}

int64_t gemvt_part_len(int64_t rows, int64_t cols) {
  return ((rows + kTRows - 1) / kTRows) * cols;
}

hipError_t launch_gemvt(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                        const double* t, const double* cin, double gamma, double* out,
                        double* part, hipStream_t s) {
  const int64_t nblk = (rows + kTRows - 1) / kTRows;
  if (nblk > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((cols + 255) / 256), (unsigned)nblk);
  switch (dtype) {
    case 0:
      hipLaunchKernelGGL(gemvt_partial_kernel<double>, grid, dim3(256), 0, s, (const double*)M, rows,
                         cols, ld, t, part);
      break;
    case 1:
      hipLaunchKernelGGL(gemvt_partial_kernel<float>, grid, dim3(256), 0, s, (const float*)M, rows,
                         cols, ld, t, part);
      break;
    default:
      hipLaunchKernelGGL(gemvt_partial_kernel<bf16_t>, grid, dim3(256), 0, s, (const bf16_t*)M,
                         rows, cols, ld, t, part);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gemvt_finish_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s,
                     part, nblk, cols, cin, gamma, out);
  return hipGetLastError();
}

// v_c = u - 1/2 with u the Philox uniform of counter (c, 0, 0, dom 2)
__global__ __launch_bounds__(256) void start_vector_kernel(double* __restrict__ v, int64_t n,
                                                           uint64_t seed) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    v[c] = draw_uniform(seed, (uint64_t)c, 0u, 0u, 2u) - 0.5;
}

// dst = src * (1 / s[0])  (s on the device: the norm just computed)
__global__ __launch_bounds__(256) void scale_kernel(double* __restrict__ dst,
                                                    const double* __restrict__ src, int64_t n,
                                                    const double* __restrict__ s2) {
  const double inv = 1.0 / sqrt(s2[0]);
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    dst[c] = src[c] * inv;
}

}  // namespace rka

namespace rka {
int api_fail(int code, const char* fmt, ...);
int api_num_cus();
}

namespace {

// number of eigenvalues of the symmetric tridiagonal (a, b) below x
// (Sturm sequence / LDL^T pivots)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = a[i] - x - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

// the k-th smallest eigenvalue (k = 1 .. n) by bisection on [lo, hi]
double kth_eigenvalue(const std::vector<double>& a, const std::vector<double>& b, int k, double lo,
                      double hi) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, mid) >= k)
      hi = mid;
    else
      lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

#define SHIP(call)                                                                           \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return rka::api_fail(e_ == hipErrorOutOfMemory ? RKA_ENOMEM : RKA_EDEVICE, "%s: %s",   \
                           #call, hipGetErrorString(e_));                                    \
  } while (0)

extern "C" int rka_gemv_t(const void* M, int dtype, int64_t rows, int64_t cols, int64_t ld,
                          const double* t, const double* c, double gamma, double* out,
                          void* stream) {
  if (!M || !t || !out) return rka::api_fail(RKA_EINVAL, "M, t and out must be non-null");
  if (dtype != RKA_F64 && dtype != RKA_F32 && dtype != RKA_BF16)
    return rka::api_fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (rows < 1 || cols < 1 || ld < cols) return rka::api_fail(RKA_EINVAL, "need rows, cols >= 1, ld >= cols");
  if ((rows + rka::kTRows - 1) / rka::kTRows > 65535)
    return rka::api_fail(RKA_EINVAL, "rows must be < 65535 * %d", rka::kTRows);
  if (!isfinite(gamma)) return rka::api_fail(RKA_EINVAL, "gamma must be finite");
  if (rka::api_num_cus() <= 0) return rka::api_fail(RKA_EDEVICE, "no HIP device available");
  hipStream_t s = (hipStream_t)stream;
  double* part = nullptr;
  SHIP(hipMallocAsync((void**)&part, (size_t)rka::gemvt_part_len(rows, cols) * sizeof(double), s));
  hipError_t e = rka::launch_gemvt(M, dtype, rows, cols, ld, t, c, gamma, out, part, s);
  (void)hipFreeAsync(part, s);
  SHIP(e);
  return RKA_OK;
}

// Lanczos on the smaller Gram matrix: side 0 is A^T A (vectors of length
// n), side 1 is A A^T (length m); both have the squared singular values of A
// as their nonzero eigenvalues.
static int spectral_core(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         int32_t steps, uint64_t seed, hipStream_t s, double* lam_min,
                         double* lam_max, double* fro2) {
  const int side = m < n ? 1 : 0;
  const int64_t N = side ? m : n, O = side ? n : m;  // Lanczos length, other length
  const int k = (int)(steps < N ? steps : N);
  const bool vec_ok = ((uintptr_t)A % 16 == 0) &&
                      ((lda * (dtype == 0 ? 8 : dtype == 1 ? 4 : 2)) % 16 == 0) &&
                      (n % (dtype == 0 ? 2 : dtype == 1 ? 4 : 8) == 0);
  struct Bufs {
    hipStream_t s;
    std::vector<void*> p;
    ~Bufs() {
      for (size_t i = p.size(); i-- > 0;) (void)hipFreeAsync(p[i], s);
    }
  } bufs{s, {}};
  auto get = [&](double** out, size_t count) {
    void* q = nullptr;
    hipError_t e = hipMallocAsync(&q, (count > 0 ? count : 1) * sizeof(double), s);
    if (e == hipSuccess) {
      bufs.p.push_back(q);
      *out = (double*)q;
    }
    return e;
  };
  double *V, *w, *t, *h, *part, *tpart, *scal;
  SHIP(get(&V, (size_t)(k + 1) * N));
  SHIP(get(&w, (size_t)N));
  SHIP(get(&t, (size_t)O));
  SHIP(get(&h, (size_t)(k + 1)));
  SHIP(get(&part, (size_t)rka::sumsq_part_len()));
  SHIP(get(&tpart, (size_t)std::max<int64_t>(rka::gemvt_part_len(m, n),
                                             rka::gemvt_part_len(k + 1, N))));
  SHIP(get(&scal, 2));
  if (fro2) {  // ||A||_F^2 from the squared row norms (Eq. (4) denominator)
    double* wn;
    SHIP(get(&wn, (size_t)m));
    SHIP(rka::launch_row_norms(A, dtype, m, n, lda, vec_ok, wn, s));
    std::vector<double> hw(m);
    SHIP(hipMemcpyAsync(hw.data(), wn, m * sizeof(double), hipMemcpyDeviceToHost, s));
    SHIP(hipStreamSynchronize(s));
    double f = 0.0;
    for (int64_t i = 0; i < m; ++i) f += hw[i];
    *fro2 = f;
  }
  hipLaunchKernelGGL(rka::start_vector_kernel, dim3(64), dim3(256), 0, s, w, N, seed);
  SHIP(hipGetLastError());
  SHIP(rka::launch_sumsq(w, nullptr, N, part, scal, s));
  hipLaunchKernelGGL(rka::scale_kernel, dim3(64), dim3(256), 0, s, V, w, N, scal);
  SHIP(hipGetLastError());
  std::vector<double> al, be;
  for (int j = 0; j < k; ++j) {
    double* vj = V + (size_t)j * N;
    if (side == 0) {  // w = A^T (A v_j)
      SHIP(rka::launch_gemv(A, dtype, m, n, lda, vec_ok, vj, nullptr, 1.0, t, s));
      SHIP(rka::launch_gemvt(A, dtype, m, n, lda, t, nullptr, 1.0, w, tpart, s));
    } else {  // w = A (A^T v_j)
      SHIP(rka::launch_gemvt(A, dtype, m, n, lda, vj, nullptr, 1.0, t, tpart, s));
      SHIP(rka::launch_gemv(A, dtype, m, n, lda, vec_ok, t, nullptr, 1.0, w, s));
    }
    // full reorthogonalisation against v_0 .. v_j, twice: h = V w, w -= V^T h
    double aj = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      SHIP(rka::launch_gemv(V, RKA_F64, j + 1, N, N, N % 2 == 0, w, nullptr, 1.0, h, s));
      if (pass == 0) SHIP(hipMemcpyAsync(&aj, h + j, sizeof aj, hipMemcpyDeviceToHost, s));
      SHIP(rka::launch_gemvt(V, RKA_F64, j + 1, N, N, h, w, -1.0, w, tpart, s));
    }
    SHIP(rka::launch_sumsq(w, nullptr, N, part, scal, s));
    double b2 = 0.0;
    SHIP(hipMemcpyAsync(&b2, scal, sizeof b2, hipMemcpyDeviceToHost, s));
    SHIP(hipStreamSynchronize(s));
    al.push_back(aj);
    const double bj = sqrt(b2);
    if (j + 1 == k || !(bj > 1e-12 * fabs(aj)) || !isfinite(bj)) break;
    be.push_back(bj);
    hipLaunchKernelGGL(rka::scale_kernel, dim3(64), dim3(256), 0, s, V + (size_t)(j + 1) * N, w, N,
                       scal);
    SHIP(hipGetLastError());
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  double lo = INFINITY, hi = -INFINITY;  // Gershgorin interval, then bisection
  for (size_t i = 0; i < al.size(); ++i) {
    const double r = (i > 0 ? fabs(be[i - 1]) : 0.0) + (i < be.size() ? fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  *lam_min = kth_eigenvalue(al, be, 1, lo, hi);
  *lam_max = kth_eigenvalue(al, be, (int)al.size(), lo, hi);
  SHIP(hipStreamSynchronize(s));
  return RKA_OK;
}

static int spectral_args(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                         int32_t steps) {
  if (!A) return rka::api_fail(RKA_EINVAL, "A must be non-null");
  if (dtype != RKA_F64 && dtype != RKA_F32 && dtype != RKA_BF16)
    return rka::api_fail(RKA_EINVAL, "dtype %d is not an rka_dtype", dtype);
  if (m < 1 || n < 1 || lda < n) return rka::api_fail(RKA_EINVAL, "need m, n >= 1 and lda >= n");
  if ((m + rka::kTRows - 1) / rka::kTRows > 65535)
    return rka::api_fail(RKA_EINVAL, "m must be < 65535 * %d", rka::kTRows);
  if (steps < 1 || steps > 4096) return rka::api_fail(RKA_EINVAL, "steps must be in [1, 4096]");
  if (rka::api_num_cus() <= 0) return rka::api_fail(RKA_EDEVICE, "no HIP device available");
  return RKA_OK;
}

extern "C" int rka_spectral_bounds(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                                   int32_t steps, uint64_t seed, void* stream, double* lam_min,
                                   double* lam_max, double* fro2) {
  if (!lam_min || !lam_max) return rka::api_fail(RKA_EINVAL, "lam_min and lam_max must be non-null");
  const int v = spectral_args(A, dtype, m, n, lda, steps);
  if (v != RKA_OK) return v;
  return spectral_core(A, dtype, m, n, lda, steps, seed, (hipStream_t)stream, lam_min, lam_max,
                       fro2);
}

namespace rka {
// Eq. (6): the uniform weight minimising the worst contraction factor over
// s = sigma^2 / ||A||_F^2 in [s_min, s_max]; q = 1 always takes the first case
double alpha_star_eq6(double s_min, double s_max, int q) {
  if (q == 1 || s_max - s_min <= 1.0 / (q - 1)) return q / (1.0 + (q - 1) * s_min);
  return 2.0 * q / (1.0 + (q - 1) * (s_min + s_max));
}
}  // namespace rka

extern "C" int rka_partial_alpha(const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                                 int32_t q, int32_t steps, uint64_t seed, void* stream,
                                 double* alpha_out) {
  if (!alpha_out) return rka::api_fail(RKA_EINVAL, "alpha_out must be non-null");
  const int v = spectral_args(A, dtype, m, n, lda, steps);
  if (v != RKA_OK) return v;
  if (q < 1 || q > m) return rka::api_fail(RKA_EINVAL, "need 1 <= q <= m");
  const int es = dtype == RKA_F64 ? 8 : dtype == RKA_F32 ? 4 : 2;
  for (int w = 0; w < q; ++w) {
    const int64_t lo = (int64_t)w * m / q, hi = ((int64_t)w + 1) * m / q;
    double lmin = 0.0, lmax = 0.0, f = 0.0;
    const int rc = spectral_core((const char*)A + lo * lda * es, dtype, hi - lo, n, lda, steps,
                                 seed + (uint64_t)w, (hipStream_t)stream, &lmin, &lmax, &f);
    if (rc != RKA_OK) return rc;
    if (!(f > 0.0)) return rka::api_fail(RKA_EZERONORM, "worker %d's row block has zero weight", w);
    alpha_out[w] = rka::alpha_star_eq6(lmin / f, lmax / f, q);
  }
  return RKA_OK;
}
