// Small row-wise helper kernels around the fused FFT kernels: per-row
// intensity statistics, normalisation and scaling of rows, zero fill (used
// instead of memset so the launches stay graph-capturable), and the per-row
// result record.
#include <hip/hip_runtime.h>

#include <algorithm>
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

// rowsum / rowmean as k_row_isum for FP32 I with len % 4 == 0 and a 16-byte
// aligned I: 16-byte loads, eight per thread in flight, four FP64 partial sums.
__global__ void __launch_bounds__(256) k_row_isum4(const float4* I, int64_t len4, int P, double* rowsum,
                                                    float* rowmean) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  if (p >= P) return;
  const float4* src = I + (size_t)p * len4;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t i = threadIdx.x;
  for (; i + 7 * 256 < len4; i += 8 * 256) {
    float4 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = src[i + q * 256];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      s0 += (double)v[q].x;
      s1 += (double)v[q].y;
      s2 += (double)v[q].z;
      s3 += (double)v[q].w;
    }
  }
  for (; i < len4; i += 256) {
    const float4 v = src[i];
    s0 += (double)v.x;
    s1 += (double)v.y;
    s2 += (double)v.z;
    s3 += (double)v.w;
  }
  const double s = block_sum<256>((s0 + s1) + (s2 + s3), red);
  if (threadIdx.x == 0) {
    if (rowsum) rowsum[p] = s;
    if (rowmean) rowmean[p] = (float)(s / (double)(len4 * 4));
  }
}

// The same for BF16 I with len % 8 == 0 and a 16-byte aligned I: eight
// values per 16-byte load.
__global__ void __launch_bounds__(256) k_row_isum8(const uint4* I, int64_t len8, int P, double* rowsum,
                                                    float* rowmean) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  if (p >= P) return;
  const uint4* src = I + (size_t)p * len8;
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t i = threadIdx.x;
  auto add = [&](const uint4 v) {
    s0 += (double)bf16f((uint16_t)(v.x & 0xffffu)) + (double)bf16f((uint16_t)(v.x >> 16));
    s1 += (double)bf16f((uint16_t)(v.y & 0xffffu)) + (double)bf16f((uint16_t)(v.y >> 16));
    s2 += (double)bf16f((uint16_t)(v.z & 0xffffu)) + (double)bf16f((uint16_t)(v.z >> 16));
    s3 += (double)bf16f((uint16_t)(v.w & 0xffffu)) + (double)bf16f((uint16_t)(v.w >> 16));
  };
  for (; i + 3 * 256 < len8; i += 4 * 256) {
    uint4 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = src[i + q * 256];
#pragma unroll
    for (int q = 0; q < 4; ++q) add(v[q]);
  }
  for (; i < len8; i += 256) add(src[i]);
  const double s = block_sum<256>((s0 + s1) + (s2 + s3), red);
  if (threadIdx.x == 0) {
    if (rowsum) rowsum[p] = s;
    if (rowmean) rowmean[p] = (float)(s / (double)(len8 * 8));
  }
}

// Rows of at most RW_WG * RW_V * 2 complex values held in registers (one
// 16-byte load per two values): one read and one write per row.
constexpr int RW_WG = 512, RW_V = 8;

// Block sum over RW_WG threads; every thread gets the total.
static __device__ __forceinline__ double rw_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < RW_WG / 64; ++i) s += red[i];
  return s;
}

// Scale and write a register-resident row: the factor of k_row_rescale from
// the squared norm s of the FP32 values.
static __device__ __forceinline__ void rw_scale_store(float4* r, int NH, const float4* v, double s, int mode,
                                                      const double* rowsum, int p, double denom) {
  double sc = (s > 0) ? 1.0 / sqrt(s) : 1.0;
  if (mode == 1) sc *= sqrt(fmax(rowsum[p], 0.0) / denom);
  const float f = (float)sc;
#pragma unroll
  for (int q = 0; q < RW_V; ++q) {
    const int c = q * RW_WG + threadIdx.x;
    if (c < NH) r[c] = make_float4(v[q].x * f, v[q].y * f, v[q].z * f, v[q].w * f);
  }
}

__global__ void __launch_bounds__(RW_WG) k_row_rescale_reg(float4* t, int NH, int mode, const double* rowsum,
                                                           double denom) {
  __shared__ double red[RW_WG / 64];
  const int p = blockIdx.x;
  float4* r = t + (size_t)p * NH;
  float4 v[RW_V];
  double s = 0;
#pragma unroll
  for (int q = 0; q < RW_V; ++q) {
    const int c = q * RW_WG + threadIdx.x;
    v[q] = c < NH ? r[c] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int q = 0; q < RW_V; ++q)
    s += ((double)v[q].x * v[q].x + (double)v[q].y * v[q].y) + ((double)v[q].z * v[q].z + (double)v[q].w * v[q].w);
  s = rw_sum(s, red);
  rw_scale_store(r, NH, v, s, mode, rowsum, p, denom);
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
  if (!bf16 && len % 4 == 0 && (uintptr_t)I % 16 == 0)
    k_row_isum4<<<P, 256, 0, (hipStream_t)s>>>((const float4*)I, len / 4, P, rowsum, rowmean);
  else if (bf16 && len % 8 == 0 && (uintptr_t)I % 16 == 0)
    k_row_isum8<<<P, 256, 0, (hipStream_t)s>>>((const uint4*)I, len / 8, P, rowsum, rowmean);
  else
    k_row_isum<<<P, 256, 0, (hipStream_t)s>>>(I, bf16, len, P, rowsum, rowmean);
  return (int)hipGetLastError();
}
// rows that fit the register-resident kernels: even N, at most RW_WG * RW_V
// pairs, 16-byte aligned
static bool rows_in_registers(const void* t, int N) {
  return N % 2 == 0 && N / 2 <= RW_WG * RW_V && (uintptr_t)t % 16 == 0;
}
int launch_row_rescale(void* t, int N, int P, int mode, const double* rowsum, double denom,
                       void* s) {
  if (P <= 0) return 0;
  if (rows_in_registers(t, N))
    k_row_rescale_reg<<<P, RW_WG, 0, (hipStream_t)s>>>((float4*)t, N / 2, mode, rowsum, denom);
  else
    k_row_rescale<<<P, 256, 0, (hipStream_t)s>>>((float2*)t, N, P, mode, rowsum, denom);
  return (int)hipGetLastError();
}
// rows whose FP64 residual exceeds thr (or is not finite): idx[*count] = p
__global__ void __launch_bounds__(256) k_flag_rows(const RowStats* __restrict__ st, int P, double thr, int* idx,
                                                   int* count) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const double r = st[p].rho;
  if (!(r <= thr)) idx[atomicAdd(count, 1)] = p;
}

// dst row j <- src row idx[j], rows of `words` 8-byte words
__global__ void __launch_bounds__(256) k_gather_rows(uint2* __restrict__ dst, const uint2* __restrict__ src,
                                                     const int* __restrict__ idx, int64_t words) {
  const int j = blockIdx.y;
  const uint2* s = src + (size_t)idx[j] * words;
  uint2* d = dst + (size_t)j * words;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256) d[i] = s[i];
}

// row idx[j] of t and of st takes the fallback's row j where its residual is lower
__global__ void __launch_bounds__(256) k_select_rows(uint2* __restrict__ t, const uint2* __restrict__ tf,
                                                     RowStats* __restrict__ st, const RowStats* __restrict__ stf,
                                                     const int* __restrict__ idx, int64_t words) {
  const int j = blockIdx.y;
  const int p = idx[j];
  const bool take = stf[j].rho < st[p].rho || !(st[p].rho == st[p].rho);
  if (!take) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (int64_t)gridDim.x * 256)
    t[(size_t)p * words + i] = tf[(size_t)j * words + i];
  __syncthreads();  // every thread has read st[p].rho above before it is replaced
  if (blockIdx.x == 0 && threadIdx.x == 0) st[p] = stf[j];
}

int launch_flag_rows(const void* st, int P, double thr, int* idx, int* count, void* s) {
  if (P <= 0) return 0;
  k_flag_rows<<<(P + 255) / 256, 256, 0, (hipStream_t)s>>>((const RowStats*)st, P, thr, idx, count);
  return (int)hipGetLastError();
}

int launch_gather_rows(void* dst, const void* src, const int* idx, int rows, int64_t row_bytes, void* s) {
  if (rows <= 0) return 0;
  if (row_bytes % 8 || (uintptr_t)dst % 8 || (uintptr_t)src % 8) return (int)hipErrorInvalidValue;
  const int64_t words = row_bytes / 8;
  dim3 grid((unsigned)std::min<int64_t>((words + 255) / 256, 64), (unsigned)rows);
  k_gather_rows<<<grid, 256, 0, (hipStream_t)s>>>((uint2*)dst, (const uint2*)src, idx, words);
  return (int)hipGetLastError();
}

int launch_select_rows(void* t, const void* tf, void* st, const void* stf, const int* idx, int rows, int64_t row_bytes,
                       void* s) {
  if (rows <= 0) return 0;
  if (row_bytes % 8) return (int)hipErrorInvalidValue;
  const int64_t words = row_bytes / 8;
  // one workgroup per row: the residual comparison and the record update stay in one workgroup
  dim3 grid(1, (unsigned)rows);
  k_select_rows<<<grid, 256, 0, (hipStream_t)s>>>((uint2*)t, (const uint2*)tf, (RowStats*)st,
                                                  (const RowStats*)stf, idx, words);
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

// number of eigenvalues below x of the symmetric tridiagonal with diagonal al
// and squared couplings b2[i] = be[i]^2 (be[i] couples i - 1 and i)
__device__ int sturm_below(const double* al, const double* b2, int k, double x) {
  int c = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    q = (al[i] - x) - (i ? b2[i] / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++c;
  }
  return c;
}

__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// One wave per row (four rows per workgroup), T in LDS. The largest eigenvalue
// by multisection on Sturm counts: each round the 64 lanes count at 64 interior
// points of [lo, hi] and the interval shrinks to the step between the last
// point below the eigenvalue and the first above it (a factor 65 per round
// instead of 2). Then, by lane 0, inverse iteration just above it: T - mu I is
// negative definite, so the elimination needs no pivoting.
constexpr int LZR = 4;
__global__ void __launch_bounds__(64 * LZR) k_lz_ritz(const float* hist, int k, int P, double* y) {
  __shared__ double s_al[LZR][LZ_MAX], s_be[LZR][LZ_MAX], s_b2[LZR][LZ_MAX], s_cp[LZR][LZ_MAX], s_z[LZR][LZ_MAX];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int p = blockIdx.x * LZR + w;
  const bool valid = p < P;
  double* al = s_al[w];
  double* be = s_be[w];
  double* b2 = s_b2[w];
  if (valid && lane < k) {
    al[lane] = (double)hist[((size_t)lane * P + p) * 2];
    be[lane] = lane ? (double)hist[((size_t)(lane - 1) * P + p) * 2 + 1] : 0.0;
    b2[lane] = be[lane] * be[lane];
  }
  __syncthreads();
  if (!valid) return;
  // Gershgorin interval
  double glo = 1e308, ghi = -1e308;
  if (lane < k) {
    const double r = fabs(be[lane]) + (lane + 1 < k ? fabs(be[lane + 1]) : 0.0);
    glo = al[lane] - r;
    ghi = al[lane] + r;
  }
  double lo = wave_min(glo), hi = wave_max(ghi);
  const double mag = fmax(fabs(lo), fabs(hi));
  if (!(mag > 1e-290)) {  // T = 0 (a zero row): any unit vector; take the seed
    if (lane < k) y[(size_t)p * k + lane] = lane == 0 ? 1.0 : 0.0;
    return;
  }
  const double span = hi - lo;
  hi += 1e-12 * span + 1e-15 * mag;
  for (int it = 0; it < 40 && hi - lo > 4e-16 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double h = (hi - lo) / 65.0;
    const double x = lo + h * (double)(lane + 1);
    const unsigned long long above = __ballot(sturm_below(al, b2, k, x) == k);
    const int l = above ? __ffsll((long long)above) - 1 : 64;  // first point above the eigenvalue
    const double nhi = l < 64 ? lo + h * (double)(l + 1) : hi;
    const double nlo = l > 0 ? lo + h * (double)l : lo;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) {
    double* cp = s_cp[w];
    double* z = s_z[w];
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

// t = sum_j y_j v_j for even N: the grid's row y is basis row p, each thread
// takes CV pairs of values (16-byte loads, CV * 256 apart), the basis rows'
// loads go out in groups of four before their products are added (FP64 sums).
constexpr int CV = 2;
__global__ void __launch_bounds__(256) k_lz_combine2(float4* t, const float4* Vw, const double* y, int k, int NH,
                                                     int64_t nh) {
  const int c0 = blockIdx.x * (256 * CV) + threadIdx.x;
  const int p = blockIdx.y;
  const int64_t i0 = (int64_t)p * NH + c0;
  const double* yp = y + (size_t)p * k;
  bool ok[CV];
  double a[CV][4];
#pragma unroll
  for (int u = 0; u < CV; ++u) {
    ok[u] = c0 + u * 256 < NH;
    const float4 v0 = ok[u] ? t[i0 + u * 256] : make_float4(0.f, 0.f, 0.f, 0.f);
    a[u][0] = yp[0] * v0.x;
    a[u][1] = yp[0] * v0.y;
    a[u][2] = yp[0] * v0.z;
    a[u][3] = yp[0] * v0.w;
  }
  int j = 1;
  for (; j + 3 < k; j += 4) {
    float4 v[4][CV];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < CV; ++u)
        v[q][u] = ok[u] ? Vw[(size_t)(j - 1 + q) * nh + i0 + u * 256] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double w = yp[j + q];
#pragma unroll
      for (int u = 0; u < CV; ++u) {
        a[u][0] += w * v[q][u].x;
        a[u][1] += w * v[q][u].y;
        a[u][2] += w * v[q][u].z;
        a[u][3] += w * v[q][u].w;
      }
    }
  }
  for (; j < k; ++j) {
    const double w = yp[j];
#pragma unroll
    for (int u = 0; u < CV; ++u) {
      const float4 v = ok[u] ? Vw[(size_t)(j - 1) * nh + i0 + u * 256] : make_float4(0.f, 0.f, 0.f, 0.f);
      a[u][0] += w * v.x;
      a[u][1] += w * v.y;
      a[u][2] += w * v.z;
      a[u][3] += w * v.w;
    }
  }
#pragma unroll
  for (int u = 0; u < CV; ++u)
    if (ok[u]) t[i0 + u * 256] = make_float4((float)a[u][0], (float)a[u][1], (float)a[u][2], (float)a[u][3]);
}

}  // namespace

int launch_lz_ritz(const float* hist, int k, int P, double* y, void* stream) {
  if (P <= 0) return 0;
  if (k < 1 || k > LZ_MAX) return (int)hipErrorInvalidValue;
  k_lz_ritz<<<(P + LZR - 1) / LZR, 64 * LZR, 0, (hipStream_t)stream>>>(hist, k, P, y);
  return (int)hipGetLastError();
}

int launch_lz_combine_scaled(void* t, const void* Vw, const double* y, int k, int P, int N, const double* rowsum,
                             double denom, void* stream) {
  int e = launch_lz_combine(t, Vw, y, k, P, N, stream);
  if (!e) e = launch_row_rescale(t, N, P, 1, rowsum, denom, stream);
  return e;
}

int launch_lz_combine(void* t, const void* Vw, const double* y, int k, int P, int N, void* stream) {
  if (P <= 0) return 0;
  const int64_t n = (int64_t)P * N;
  if (N % 2 == 0 && P <= 65535 && (uintptr_t)t % 16 == 0 && (uintptr_t)Vw % 16 == 0) {
    // one row per grid row, two values per thread
    const dim3 grid((N / 2 + 256 * CV - 1) / (256 * CV), P);
    k_lz_combine2<<<grid, 256, 0, (hipStream_t)stream>>>((float4*)t, (const float4*)Vw, y, k, N / 2, n / 2);
    return (int)hipGetLastError();
  }
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  k_lz_combine<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((float2*)t, (const float2*)Vw, y, k, P, N);
  return (int)hipGetLastError();
}

}  // namespace tmk
