// Small row-wise helper kernels around the fused FFT kernels: per-row
// intensity statistics, normalisation and scaling of rows, zero fill (used
// instead of memset so the launches stay graph-capturable), and the per-row
// result record.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "aux.hpp"

namespace tmk {

static __device__ __forceinline__ float bf16f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

template <int WG>
static __device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < WG / 64; ++i) s += red[i];
  return s;
}

// rowsum[p] = sum_k I[p][k] (FP64 accumulation), rowmean = rowsum / len.
__global__ void __launch_bounds__(256) k_row_isum(const void* I, int bf16, int64_t len, int P,
                                                   double* rowsum, float* rowmean) {
  __shared__ double red[4];
  int p = blockIdx.x;
  if (p >= P) return;
  double s = 0;
  if (bf16) {
    const uint16_t* src = (const uint16_t*)I + (size_t)p * len;
    for (int64_t i = threadIdx.x; i < len; i += 256) s += (double)bf16f(src[i]);
  } else {
    const float* src = (const float*)I + (size_t)p * len;
    for (int64_t i = threadIdx.x; i < len; i += 256) s += (double)src[i];
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) {
    if (rowsum) rowsum[p] = s;
    if (rowmean) rowmean[p] = (float)(s / (double)len);
  }
}

// t[p] *= scale_p where scale_p = 1/||t_p|| (mode 0) or
// sqrt(rowsum[p] / denom) / ||t_p|| (mode 1).
__global__ void __launch_bounds__(256) k_row_rescale(float2* t, int N, int P, int mode,
                                                      const double* rowsum, double denom) {
  __shared__ double red[4];
  int p = blockIdx.x;
  if (p >= P) return;
  float2* r = t + (size_t)p * N;
  double s = 0;
  for (int i = threadIdx.x; i < N; i += 256) {
    float2 v = r[i];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  s = block_sum<256>(s, red);
  double sc = (s > 0) ? 1.0 / sqrt(s) : 1.0;
  if (mode == 1) sc *= sqrt(fmax(rowsum[p], 0.0) / denom);
  float f = (float)sc;
  for (int i = threadIdx.x; i < N; i += 256) {
    float2 v = r[i];
    r[i] = make_float2(v.x * f, v.y * f);
  }
}

__global__ void __launch_bounds__(256) k_fill_zero(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) p[i] = 0u;
}

template <typename V>
__global__ void __launch_bounds__(256) k_copy(V* dst, const V* src, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_fill_hash(float* p, int64_t n, uint32_t seed, float lo, float hi) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) {
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    p[i] = lo + (hi - lo) * ((h >> 8) * (1.0f / 16777216.0f));
  }
}

// Per-row result record (layout of tm_row_stats).
struct RowStats {
  double rho;
  float f;
  float amp_res;
  int32_t iters;
  int32_t flags;
};

__global__ void __launch_bounds__(256) k_finalize(RowStats* st, int P, const double* sums64,
                                                   const float* sums, int nsum, int f_idx,
                                                   int amp_idx, int iters, double rho_flag) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  double sr = sums64[2 * p], si = sums64[2 * p + 1];
  double rho = (si > 0) ? sr / si : (sr > 0 ? INFINITY : 0.0);
  RowStats r;
  r.rho = rho;
  r.f = (sums && f_idx >= 0) ? sums[(size_t)p * nsum + f_idx] : (float)sr;
  r.amp_res = (sums && amp_idx >= 0) ? sums[(size_t)p * nsum + amp_idx] : 0.f;
  r.iters = iters;
  int flags = 0;
  if (!(rho <= rho_flag)) flags |= 1;
  if (!isfinite(rho)) flags |= 2;
  r.flags = flags;
  st[p] = r;
}

// ------------------------------------------------------------------ launchers
int launch_row_isum(const void* I, int bf16, int64_t len, int P, double* rowsum, float* rowmean,
                    void* s) {
  if (P <= 0) return 0;
  k_row_isum<<<P, 256, 0, (hipStream_t)s>>>(I, bf16, len, P, rowsum, rowmean);
  return (int)hipGetLastError();
}
int launch_row_rescale(void* t, int N, int P, int mode, const double* rowsum, double denom,
                       void* s) {
  if (P <= 0) return 0;
  k_row_rescale<<<P, 256, 0, (hipStream_t)s>>>((float2*)t, N, P, mode, rowsum, denom);
  return (int)hipGetLastError();
}
int launch_fill_zero(void* p, int64_t bytes, void* s) {
  int64_t n = bytes / 4;
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_zero<<<(int)blocks, 256, 0, (hipStream_t)s>>>((uint32_t*)p, n);
  return (int)hipGetLastError();
}
int launch_copy(void* dst, const void* src, int64_t bytes, void* s) {
  if (bytes <= 0) return 0;
  const uintptr_t al = (uintptr_t)dst | (uintptr_t)src | (uintptr_t)bytes;
  if (al & 7) return (int)hipErrorInvalidValue;
  const int w = (al & 15) ? 8 : 16;
  int64_t n = bytes / w;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (w == 16) k_copy<uint4><<<(int)blocks, 256, 0, (hipStream_t)s>>>((uint4*)dst, (const uint4*)src, n);
  else k_copy<uint2><<<(int)blocks, 256, 0, (hipStream_t)s>>>((uint2*)dst, (const uint2*)src, n);
  return (int)hipGetLastError();
}
int launch_fill_hash(float* p, int64_t n, uint32_t seed, float lo, float hi, void* s) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_hash<<<(int)blocks, 256, 0, (hipStream_t)s>>>(p, n, seed, lo, hi);
  return (int)hipGetLastError();
}
int launch_finalize(void* st, int P, const double* sums64, const float* sums, int nsum, int f_idx,
                    int amp_idx, int iters, double rho_flag, void* s) {
  if (P <= 0) return 0;
  k_finalize<<<(P + 255) / 256, 256, 0, (hipStream_t)s>>>((RowStats*)st, P, sums64, sums, nsum,
                                                           f_idx, amp_idx, iters, rho_flag);
  return (int)hipGetLastError();
}


// ---------------------------------------------------------------- Lanczos start
namespace {

// number of eigenvalues below x of the symmetric tridiagonal (al, be[i] coupling i - 1 and i)
__device__ int sturm_below(const double* al, const double* be, int k, double x) {
  int c = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    q = (al[i] - x) - (i ? be[i] * be[i] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++c;
  }
  return c;
}

__global__ void __launch_bounds__(64) k_lz_ritz(const float* hist, int k, int P, double* y) {
  const int p = blockIdx.x * 64 + threadIdx.x;
  if (p >= P) return;
  double al[LZ_MAX], be[LZ_MAX], cp[LZ_MAX], z[LZ_MAX];
  for (int i = 0; i < k; ++i) {
    al[i] = (double)hist[((size_t)i * P + p) * 2];
    be[i] = i ? (double)hist[((size_t)(i - 1) * P + p) * 2 + 1] : 0.0;
  }
  // Gershgorin interval, then bisection for the largest eigenvalue (count below hi == k)
  double lo = al[0], hi = al[0];
  for (int i = 0; i < k; ++i) {
    const double r = fabs(be[i]) + (i + 1 < k ? fabs(be[i + 1]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  const double mag = fmax(fabs(lo), fabs(hi));
  if (!(mag > 1e-290)) {  // T = 0 (a zero row): any unit vector; take the seed
    for (int i = 0; i < k; ++i) y[(size_t)p * k + i] = i == 0 ? 1.0 : 0.0;
    return;
  }
  const double span = hi - lo;
  hi += 1e-12 * span + 1e-15 * mag;
  for (int it = 0; it < 200 && hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_below(al, be, k, mid) == k) hi = mid;
    else lo = mid;
  }
  // inverse iteration just above the largest eigenvalue: T - mu I is negative
  // definite, so the elimination needs no pivoting
  const double mu = hi + 1e-10 * span + 1e-12 * mag;
  for (int i = 0; i < k; ++i) z[i] = 1.0;
  for (int rep = 0; rep < 3; ++rep) {
    double m = al[0] - mu;
    cp[0] = (k > 1 ? be[1] : 0.0) / m;
    z[0] = z[0] / m;
    for (int i = 1; i < k; ++i) {
      m = (al[i] - mu) - be[i] * cp[i - 1];
      cp[i] = (i + 1 < k ? be[i + 1] : 0.0) / m;
      z[i] = (z[i] - be[i] * z[i - 1]) / m;
    }
    for (int i = k - 2; i >= 0; --i) z[i] -= cp[i] * z[i + 1];
    double n = 0.0;
    for (int i = 0; i < k; ++i) n += z[i] * z[i];
    n = n > 0.0 ? 1.0 / sqrt(n) : 0.0;
    for (int i = 0; i < k; ++i) z[i] *= n;
  }
  const double sg = z[0] < 0.0 ? -1.0 : 1.0;
  for (int i = 0; i < k; ++i) y[(size_t)p * k + i] = sg * z[i];
}

__global__ void __launch_bounds__(256) k_lz_combine(float2* t, const float2* Vw, const double* y, int k, int P,
                                                    int N) {
  const int64_t n = (int64_t)P * N;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const int64_t p = i / N;
    const double* yp = y + p * k;
    const float2 v0 = t[i];
    double ax = yp[0] * v0.x, ay = yp[0] * v0.y;
    for (int j = 1; j < k; ++j) {
      const float2 v = Vw[(size_t)(j - 1) * n + i];
      ax += yp[j] * v.x;
      ay += yp[j] * v.y;
    }
    t[i] = make_float2((float)ax, (float)ay);
  }
}

}  // namespace

int launch_lz_ritz(const float* hist, int k, int P, double* y, void* stream) {
  if (P <= 0) return 0;
  if (k < 1 || k > LZ_MAX) return (int)hipErrorInvalidValue;
  k_lz_ritz<<<(P + 63) / 64, 64, 0, (hipStream_t)stream>>>(hist, k, P, y);
  return (int)hipGetLastError();
}

int launch_lz_combine(void* t, const void* Vw, const double* y, int k, int P, int N, void* stream) {
  if (P <= 0) return 0;
  const int64_t n = (int64_t)P * N;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  k_lz_combine<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((float2*)t, (const float2*)Vw, y, k, P, N);
  return (int)hipGetLastError();
}

}  // namespace tmk
