// Conjugate-phase foci of retrieved TM rows and their power ratio (Sec. 3):
// the pattern of row p is the phase of the conjugate of the retrieved row,
// the focus image is |TM_true u_p|^2 on the TM's pixels (one complex GEMM,
// done by the caller), and PR is the power in a (2w+1) x (2w+1) grid window
// around the image's peak over its total power.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "foci.hpp"

namespace tmk {

namespace {

__global__ void __launch_bounds__(256) k_conj_phase(const float2* t, float2* u, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) {
    const float2 v = t[i];
    const float m2 = v.x * v.x + v.y * v.y;
    if (m2 > 0.f) {
      const float r = rsqrtf(m2);
      u[i] = make_float2(v.x * r, -v.y * r);
    } else {
      u[i] = make_float2(1.f, 0.f);
    }
  }
}

constexpr int FWG = 256;

// one workgroup per focus image (row p of E)
__global__ void __launch_bounds__(FWG) k_foci_pr(const float2* E, int G, const int32_t* pix, int g2, int w, float* pr,
                                                int32_t* peak) {
  __shared__ float bv[FWG / 64];
  __shared__ int bq[FWG / 64];
  __shared__ double red[FWG / 64];
  __shared__ int pk;
  const int p = blockIdx.x;
  const float2* row = E + (size_t)p * G;
  // brightest pixel, ties to the smaller raster index; and the total power
  float best = -1.f;
  int bestq = 0x7fffffff;
  double tot = 0.0;
  for (int q = threadIdx.x; q < G; q += FWG) {
    const float2 v = row[q];
    const float I = v.x * v.x + v.y * v.y;
    const int r = pix[q];
    tot += (double)I;
    if (I > best || (I == best && r < bestq)) {
      best = I;
      bestq = r;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(best, off, 64);
    const int oq = __shfl_xor(bestq, off, 64);
    if (ov > best || (ov == best && oq < bestq)) {
      best = ov;
      bestq = oq;
    }
    tot += __shfl_xor(tot, off, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    bv[wv] = best;
    bq[wv] = bestq;
    red[wv] = tot;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float b = bv[0];
    int bqq = bq[0];
    double t = red[0];
    for (int i = 1; i < FWG / 64; ++i) {
      if (bv[i] > b || (bv[i] == b && bq[i] < bqq)) {
        b = bv[i];
        bqq = bq[i];
      }
      t += red[i];
    }
    pk = bqq;
    red[0] = t;
  }
  __syncthreads();
  const double total = red[0];
  const int py = pk / g2, px = pk - (pk / g2) * g2;
  __syncthreads();
  double sig = 0.0;
  for (int q = threadIdx.x; q < G; q += FWG) {
    const int r = pix[q];
    const int y = r / g2, x = r - (r / g2) * g2;
    if (abs(y - py) <= w && abs(x - px) <= w) {
      const float2 v = row[q];
      sig += (double)(v.x * v.x + v.y * v.y);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) sig += __shfl_xor(sig, off, 64);
  if ((threadIdx.x & 63) == 0) red[wv] = sig;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < FWG / 64; ++i) s += red[i];
    const bool lit = total > 0.0;
    pr[p] = lit ? (float)(s / total) : 0.f;
    peak[p] = lit ? pk : -1;
  }
}

}  // namespace

int launch_conj_phase(const void* tm_est, void* u, int64_t n, void* stream) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_conj_phase<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((const float2*)tm_est, (float2*)u, n);
  return (int)hipGetLastError();
}

int launch_foci_pr(const void* E, int Pf, int G, const int32_t* pix, int g1, int g2, int w, float* pr, int32_t* peak,
                   void* stream) {
  (void)g1;
  if (Pf <= 0) return 0;
  k_foci_pr<<<Pf, FWG, 0, (hipStream_t)stream>>>((const float2*)E, G, pix, g2, w, pr, peak);
  return (int)hipGetLastError();
}

}  // namespace tmk

namespace tmk {
namespace {

// one workgroup per row p: w = -4 conj(y (I - |y|^2)), f_p = sum (I - |y|^2)^2 (FP64 accumulation)
__global__ void __launch_bounds__(256) k_dense_pointwise(float2* Y, const float* I, int64_t M, float* f) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  float2* y = Y + (size_t)p * M;
  const float* ip = I + (size_t)p * M;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < M; i += 256) {
    const float2 v = y[i];
    const float r = ip[i] - (v.x * v.x + v.y * v.y);
    s += (double)r * (double)r;
    y[i] = make_float2(-4.f * r * v.x, 4.f * r * v.y);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0 && f) f[p] = (float)((red[0] + red[1]) + (red[2] + red[3]));
}

__global__ void __launch_bounds__(256) k_conj(float2* x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) x[i].y = -x[i].y;
}

}  // namespace

int launch_dense_pointwise(void* Y, const float* I, int P, int64_t M, float* f, void* stream) {
  if (P <= 0) return 0;
  k_dense_pointwise<<<P, 256, 0, (hipStream_t)stream>>>((float2*)Y, I, M, f);
  return (int)hipGetLastError();
}

int launch_conj_inplace(void* x, int64_t n, void* stream) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_conj<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((float2*)x, n);
  return (int)hipGetLastError();
}

}  // namespace tmk

// ------------------------------------------------------------ propagated TM
namespace tmk {
namespace {

constexpr int TT = 32;  // transpose tiles of 32 x 32 complex values, 256 threads (8 rows per pass)

// X[n][pix[p]] = tm[p][n]: tiles of 32 rows p x 32 columns n
__global__ void __launch_bounds__(256) k_cols_to_grid(const float2* tm, int P, int N, const int32_t* pix, int G,
                                                     float2* X) {
  __shared__ float2 tile[TT][TT + 1];
  const int n0 = blockIdx.x * TT, p0 = blockIdx.y * TT;
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;
  for (int r = ty; r < TT; r += 256 / TT) {
    const int p = p0 + r, n = n0 + tx;
    tile[r][tx] = (p < P && n < N) ? tm[(size_t)p * N + n] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int r = ty; r < TT; r += 256 / TT) {
    const int n = n0 + r, p = p0 + tx;
    if (n < N && p < P) X[(size_t)n * G + pix[p]] = tile[tx][r];
  }
}

// out[q][n] = X[n][q]
__global__ void __launch_bounds__(256) k_grid_to_rows(const float2* X, int N, int G, float2* out) {
  __shared__ float2 tile[TT][TT + 1];
  const int q0 = blockIdx.x * TT, n0 = blockIdx.y * TT;
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;
  for (int r = ty; r < TT; r += 256 / TT) {
    const int n = n0 + r, q = q0 + tx;
    tile[r][tx] = (n < N && q < G) ? X[(size_t)n * G + q] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  for (int r = ty; r < TT; r += 256 / TT) {
    const int q = q0 + r, n = n0 + tx;
    if (q < G && n < N) out[(size_t)q * N + n] = tile[tx][r];
  }
}

__device__ __forceinline__ double sfreq(int k, int n, double ps) {
  const int s = (k < (n + 1) / 2) ? k : k - n;
  return (double)s / ((double)n * ps);
}

// H[k1 g2 + k2] = exp(j 2 pi / lambda sqrt(1 - lambda^2 (u^2 + v^2)) z) inside the pupil, 0 outside
__global__ void __launch_bounds__(256) k_prop_filter(float2* H, int g1, int g2, double lam, double ps, double NA,
                                                    double z) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= g1 * g2) return;
  const int k1 = i / g2, k2 = i - (i / g2) * g2;
  const double u = sfreq(k1, g1, ps), v = sfreq(k2, g2, ps);
  const double rho2 = (lam * u) * (lam * u) + (lam * v) * (lam * v);
  float2 h = make_float2(0.f, 0.f);
  if (sqrt(rho2) <= NA) {
    const double ph = 2.0 * M_PI / lam * sqrt(1.0 - rho2) * z;
    h = make_float2((float)cos(ph), (float)sin(ph));
  }
  H[i] = h;
}

__global__ void __launch_bounds__(256) k_fill_c32(float2* x, int64_t n, float re, float im) {
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (; i < n; i += stride) x[i] = make_float2(re, im);
}

}  // namespace

int launch_cols_to_grid(const void* tm, int P, int N, const int32_t* pix, int G, void* X, void* stream) {
  if (P <= 0 || N <= 0) return 0;
  dim3 g((N + TT - 1) / TT, (P + TT - 1) / TT);
  k_cols_to_grid<<<g, 256, 0, (hipStream_t)stream>>>((const float2*)tm, P, N, pix, G, (float2*)X);
  return (int)hipGetLastError();
}

int launch_grid_to_rows(const void* X, int N, int G, void* out, void* stream) {
  if (N <= 0 || G <= 0) return 0;
  dim3 g((G + TT - 1) / TT, (N + TT - 1) / TT);
  k_grid_to_rows<<<g, 256, 0, (hipStream_t)stream>>>((const float2*)X, N, G, (float2*)out);
  return (int)hipGetLastError();
}

int launch_make_prop_filter(void* H, int g1, int g2, double lam, double ps, double NA, double z, void* stream) {
  k_prop_filter<<<(g1 * g2 + 255) / 256, 256, 0, (hipStream_t)stream>>>((float2*)H, g1, g2, lam, ps, NA, z);
  return (int)hipGetLastError();
}

int launch_fill_c32(void* x, int64_t n, float re, float im, void* stream) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_c32<<<(int)blocks, 256, 0, (hipStream_t)stream>>>((float2*)x, n, re, im);
  return (int)hipGetLastError();
}

}  // namespace tmk
