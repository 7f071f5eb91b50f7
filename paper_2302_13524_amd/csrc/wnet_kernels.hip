// Learned weighting of the spectral start: helper kernels of its network and
// of the training loss (not part of the paper; its start is
// Eq. backpropagation).
//
// The network maps features of a normalised intensity x = I / mean(I_p) to
// the weight T(x) of the spectral matrix A^H diag(T(x)) A (Sec. 2.2,
// Eq. probingmatrix). It is evaluated once on the NT points of a uniform
// table over [0, xmax]; the row kernels interpolate that table. Training
// runs k normalised power steps u <- M u / ||M u|| from seeds v0 and
// minimises minus the mean fidelity to the true rows; the gradient goes
// back through the k steps (fused row-kernel modes M_WAPPLY and M_WBACK)
// and lands on the table points, then on the network weights through its
// GEMMs (mlp_kernels.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "wnet.hpp"

namespace tmk {

namespace {

constexpr int WB = 256;

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Block sum of NS doubles; the totals land in every thread.
template <int NS>
__device__ __forceinline__ void block_sum(double* v, double* red) {
#pragma unroll
  for (int q = 0; q < NS; ++q)
    for (int off = 32; off >= 1; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) red[(threadIdx.x >> 6) * NS + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double s = 0.0;
    for (int w = 0; w < WB / 64; ++w) s += red[w * NS + q];
    v[q] = s;
  }
}

// Features of table point b (x = b xmax / (nt - 1)): the same 64 functions
// as the FP64 reference table_features, in that order.
__global__ void __launch_bounds__(WB) k_features(int nt, float xmax, uint16_t* X) {
  const int b = blockIdx.x * WB + threadIdx.x;
  if (b >= nt) return;
  const double x = (double)b * ((double)xmax / (double)(nt - 1));
  const double u = x / (double)xmax;
  const double pi = 3.14159265358979323846;
  double f[WNET_FEATURES];
  f[0] = u;
  f[1] = sqrt(u);
  f[2] = u * u;
  f[3] = log1p(x) / log1p((double)xmax);
  f[4] = exp(-x);
  f[5] = exp(-x / 4.0);
  f[6] = 1.0 / (1.0 + x);
  f[7] = x / (1.0 + x);
  f[8] = tanh(x - 1.0);
  f[9] = tanh((x - 3.0) / 2.0);
  f[10] = fmin(x, 1.0);
  f[11] = fmin(x, 2.0) / 2.0;
  f[12] = fmin(x, 3.0) / 3.0;
  f[13] = fmin(x, 5.0) / 5.0;
  f[14] = 1.0;
  f[15] = exp(-x * x);
  for (int q = 1; q <= 24; ++q) {
    f[14 + 2 * q] = sin(pi * q * u);
    f[15 + 2 * q] = cos(pi * q * u);
  }
  for (int i = 0; i < WNET_FEATURES; ++i) X[(size_t)b * WNET_FEATURES + i] = to_bf16((float)f[i]);
}

// network output O [nt] -> table pairs (T_b, T_{b+1} - T_b); the last slope is 0
__global__ void __launch_bounds__(WB) k_pairs(const float* __restrict__ O, int nt, float* tab) {
  const int b = blockIdx.x * WB + threadIdx.x;
  if (b >= nt) return;
  const float v = O[b];
  tab[2 * b] = v;
  tab[2 * b + 1] = (b + 1 < nt) ? O[b + 1] - v : 0.f;
}

// u = y / ||y|| per row, ||y||^2 given (sums[p * nsum]); n[p] = ||y||
__global__ void __launch_bounds__(WB) k_normalise(const float2* __restrict__ y, const float* __restrict__ sums,
                                                   int nsum, int N, float2* u, float* n) {
  const int p = blockIdx.x;
  const float nn = sqrtf(fmaxf(sums[(size_t)p * nsum], 0.f));
  const float inv = nn > 0.f ? 1.f / nn : 0.f;
  for (int i = threadIdx.x; i < N; i += WB) {
    float2 v = y[(size_t)p * N + i];
    u[(size_t)p * N + i] = make_float2(v.x * inv, v.y * inv);
  }
  if (threadIdx.x == 0) n[p] = nn;
}

// per row: c = t^H u, fidelity |c|^2 / (||t||^2 ||u||^2), loss -fidelity, and
// the packed gradient of the mean loss over B rows with respect to u:
// G = -(2 c t / (tt uu) - 2 |c|^2 u / (tt uu^2)) / B
__global__ void __launch_bounds__(WB) k_loss(const float2* __restrict__ u, const float2* __restrict__ t, int N,
                                              float inv_b, float2* G, float* fid) {
  __shared__ double red[(WB / 64) * 4];
  const int p = blockIdx.x;
  const float2* ur = u + (size_t)p * N;
  const float2* tr = t + (size_t)p * N;
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // Re c, Im c, ||t||^2, ||u||^2
  for (int i = threadIdx.x; i < N; i += WB) {
    const float2 a = tr[i], b = ur[i];
    v[0] += (double)a.x * b.x + (double)a.y * b.y;
    v[1] += (double)a.x * b.y - (double)a.y * b.x;
    v[2] += (double)a.x * a.x + (double)a.y * a.y;
    v[3] += (double)b.x * b.x + (double)b.y * b.y;
  }
  block_sum<4>(v, red);
  const double tt = v[2] > 0.0 ? v[2] : 1.0, uu = v[3] > 0.0 ? v[3] : 1.0;
  const double c2 = v[0] * v[0] + v[1] * v[1];
  const double f1 = 2.0 / (tt * uu) * inv_b, f2 = 2.0 * c2 / (tt * uu * uu) * inv_b;
  for (int i = threadIdx.x; i < N; i += WB) {
    const float2 a = tr[i], b = ur[i];
    // c t = (cr + j ci)(ax + j ay)
    const double ctr = v[0] * a.x - v[1] * a.y, cti = v[0] * a.y + v[1] * a.x;
    G[(size_t)p * N + i] = make_float2((float)(-(f1 * ctr - f2 * b.x)), (float)(-(f1 * cti - f2 * b.y)));
  }
  if (threadIdx.x == 0) fid[p] = (float)(c2 / (tt * uu));
}

// G_y = (G_u - Re(u^H G_u) u) / n
__global__ void __launch_bounds__(WB) k_normback(const float2* __restrict__ Gu, const float2* __restrict__ u,
                                                  const float* __restrict__ n, int N, float2* Gy) {
  __shared__ double red[WB / 64];
  const int p = blockIdx.x;
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < N; i += WB) {
    const float2 a = u[(size_t)p * N + i], g = Gu[(size_t)p * N + i];
    v[0] += (double)a.x * g.x + (double)a.y * g.y;
  }
  block_sum<1>(v, red);
  const float d = (float)v[0];
  const float inv = n[p] > 0.f ? 1.f / n[p] : 0.f;
  for (int i = threadIdx.x; i < N; i += WB) {
    const float2 a = u[(size_t)p * N + i], g = Gu[(size_t)p * N + i];
    Gy[(size_t)p * N + i] = make_float2((g.x - d * a.x) * inv, (g.y - d * a.y) * inv);
  }
}

template <typename IT>
__device__ __forceinline__ float ld_i(const void* I, size_t i) {
  if constexpr (sizeof(IT) == 2) return __uint_as_float(((uint32_t)((const uint16_t*)I)[i]) << 16);
  else return ((const float*)I)[i];
}

// dtab[b] += sum_i gw_i * (interpolation weight of point b at x_i): the
// adjoint of the table lookup, accumulated per workgroup in LDS, then added
// to the global table gradient (one atomic per point and workgroup).
template <typename IT>
__global__ void __launch_bounds__(WB) k_hist(const float* __restrict__ gw, const void* __restrict__ I,
                                              const float* __restrict__ rowmean, int KN, int nt, float scale,
                                              float last, int chunk, float* dtab) {
  extern __shared__ float hist[];
  for (int b = threadIdx.x; b < nt; b += WB) hist[b] = 0.f;
  __syncthreads();
  const int p = blockIdx.y;
  const float m = rowmean[p];
  const float im = m > 0.f ? 1.f / m : 1.f;
  const size_t base = (size_t)p * KN;
  const int i0 = blockIdx.x * chunk, i1 = min(KN, i0 + chunk);
  for (int i = i0 + threadIdx.x; i < i1; i += WB) {
    const float x = ld_i<IT>(I, base + i) * im;
    const float s = fminf(fmaxf(x * scale, 0.f), last);
    const int b = min((int)s, (int)last - 1);
    const float f = s - (float)b;
    const float g = gw[base + i];
    atomicAdd(&hist[b], (1.f - f) * g);
    atomicAdd(&hist[b + 1], f * g);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nt; b += WB) {
    const float v = hist[b];
    if (v != 0.f) atomicAdd(&dtab[b], v);
  }
}

// W[p][i] = T(I[p][i] / mean_p) from the table pairs (the learned weights of one retrieval)
template <typename IT>
__global__ void __launch_bounds__(WB) k_weights(const void* __restrict__ I, const float* __restrict__ rowmean,
                                                 const float2* __restrict__ tab, int64_t KN, float scale, float last,
                                                 float* W) {
  const int p = blockIdx.y;
  const float m = rowmean[p];
  const float im = m > 0.f ? 1.f / m : 1.f;
  const size_t base = (size_t)p * KN;
  for (int64_t i = (int64_t)blockIdx.x * WB + threadIdx.x; i < KN; i += (int64_t)gridDim.x * WB) {
    const float x = ld_i<IT>(I, base + i) * im;
    const float s = fminf(fmaxf(x * scale, 0.f), last);
    const int b = min((int)s, (int)last - 1);
    const float2 e = tab[b];
    W[base + i] = e.x + (s - (float)b) * e.y;
  }
}

// warm start: mean over the table points of (O_b - min(x_b, tau))^2 and its gradient
__global__ void __launch_bounds__(WB) k_regress(const float* __restrict__ O, int nt, float xmax, float tau,
                                                 float* dOf, uint16_t* dOh, float* loss) {
  __shared__ double red[WB / 64];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nt; b += WB) {
    const float x = (float)b * (xmax / (float)(nt - 1));
    const float r = O[b] - fminf(x, tau);
    v[0] += (double)r * r;
    const float g = 2.f * r / (float)nt;
    dOf[b] = g;
    dOh[b] = to_bf16(g);
  }
  block_sum<1>(v, red);
  if (threadIdx.x == 0) loss[0] = (float)(v[0] / nt);
}

// dO (FP32 and BF16) from the table gradient
__global__ void __launch_bounds__(WB) k_dout(const float* __restrict__ dtab, int nt, float* dOf, uint16_t* dOh) {
  const int b = blockIdx.x * WB + threadIdx.x;
  if (b >= nt) return;
  dOf[b] = dtab[b];
  dOh[b] = to_bf16(dtab[b]);
}

// mean of the per-row fidelities, negated: the training loss
__global__ void __launch_bounds__(WB) k_mean_loss(const float* __restrict__ fid, int B, float* loss) {
  __shared__ double red[WB / 64];
  double v[1] = {0.0};
  for (int p = threadIdx.x; p < B; p += WB) v[0] += fid[p];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) loss[0] = (float)(-v[0] / B);
}

}  // namespace

int wnet_features(int nt, float xmax, uint16_t* X, void* s) {
  k_features<<<(nt + WB - 1) / WB, WB, 0, (hipStream_t)s>>>(nt, xmax, X);
  return (int)hipGetLastError();
}

int wnet_pairs(const float* O, int nt, float* tab, void* s) {
  k_pairs<<<(nt + WB - 1) / WB, WB, 0, (hipStream_t)s>>>(O, nt, tab);
  return (int)hipGetLastError();
}

int wnet_normalise(const void* y, const float* sums, int nsum, int P, int N, void* u, float* n, void* s) {
  if (P <= 0) return 0;
  k_normalise<<<P, WB, 0, (hipStream_t)s>>>((const float2*)y, sums, nsum, N, (float2*)u, n);
  return (int)hipGetLastError();
}

int wnet_loss(const void* u, const void* t, int P, int N, void* G, float* fid, float* loss, void* s) {
  if (P <= 0) return 0;
  k_loss<<<P, WB, 0, (hipStream_t)s>>>((const float2*)u, (const float2*)t, N, 1.f / (float)P, (float2*)G, fid);
  k_mean_loss<<<1, WB, 0, (hipStream_t)s>>>(fid, P, loss);
  return (int)hipGetLastError();
}

int wnet_normback(const void* Gu, const void* u, const float* n, int P, int N, void* Gy, void* s) {
  if (P <= 0) return 0;
  k_normback<<<P, WB, 0, (hipStream_t)s>>>((const float2*)Gu, (const float2*)u, n, N, (float2*)Gy);
  return (int)hipGetLastError();
}

int wnet_hist(const float* gw, const void* I, int ibf16, const float* rowmean, int P, int KN, int nt, float xmax,
              float* dtab, void* s) {
  if (P <= 0) return 0;
  const int chunk = 8192;
  dim3 grid((KN + chunk - 1) / chunk, P);
  const float scale = (float)(nt - 1) / xmax, last = (float)(nt - 1);
  const size_t lds = (size_t)nt * sizeof(float);
  if (ibf16) k_hist<uint16_t><<<grid, WB, lds, (hipStream_t)s>>>(gw, I, rowmean, KN, nt, scale, last, chunk, dtab);
  else k_hist<float><<<grid, WB, lds, (hipStream_t)s>>>(gw, I, rowmean, KN, nt, scale, last, chunk, dtab);
  return (int)hipGetLastError();
}

int wnet_weights(const void* I, int ibf16, const float* rowmean, int P, int64_t KN, const float* tab, int nt,
                 float xmax, float* W, void* s) {
  if (P <= 0) return 0;
  dim3 grid((unsigned)std::min<int64_t>((KN + WB - 1) / WB, 64), (unsigned)P);
  const float scale = (float)(nt - 1) / xmax, last = (float)(nt - 1);
  if (ibf16) k_weights<uint16_t><<<grid, WB, 0, (hipStream_t)s>>>(I, rowmean, (const float2*)tab, KN, scale, last, W);
  else k_weights<float><<<grid, WB, 0, (hipStream_t)s>>>(I, rowmean, (const float2*)tab, KN, scale, last, W);
  return (int)hipGetLastError();
}

int wnet_regress(const float* O, int nt, float xmax, float tau, float* dOf, uint16_t* dOh, float* loss, void* s) {
  k_regress<<<1, WB, 0, (hipStream_t)s>>>(O, nt, xmax, tau, dOf, dOh, loss);
  return (int)hipGetLastError();
}

int wnet_dout(const float* dtab, int nt, float* dOf, uint16_t* dOh, void* s) {
  k_dout<<<(nt + WB - 1) / WB, WB, 0, (hipStream_t)s>>>(dtab, nt, dOf, dOh);
  return (int)hipGetLastError();
}

}  // namespace tmk
