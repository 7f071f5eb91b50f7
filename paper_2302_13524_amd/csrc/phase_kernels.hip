// Phase-offset correction from defocus intensities (Sec. 2.3), FP64.
//
// Forward model per defocus input n (Eq. forwarddefocusImage):
//   field F_n = scatter(c_n * u) on the nf1 x nf2 grid, u = e^{j phi},
//   S = K1 F_n (unitary 2-D DFT), S *= h (Eq. angularspectrum with pupil),
//   zero-pad S to (2nf1) x (2nf2) keeping signed frequencies, a_n = K2^H S.
// Objective g = sum_n || I_n - |a_n|^2 ||^2 (Eq. optphase) and gradient
// dg/dphi = -4 Im(conj(u) w), w = sum_n A_n^H (a_n r_n) (Eq. phasederive).
// The 2-D transforms run one axis at a time as FP64 line FFTs in LDS, fused
// with the pointwise steps between them.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <stdint.h>

#include "phase.hpp"

namespace tmk {

namespace {

constexpr int GATHER_SLICES = 8;  // image slices of the gradient gather

struct z2 {
  double x, y;
};
__device__ __forceinline__ z2 zmul(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ z2 zmulc(z2 a, z2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// ---- c[n][p] = sum_k theta[n][k] tm[p][k]: FP32 complex inputs, exact FP64
// products, FP64 sums, on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
// Real embedding with the outputs' real and imaginary parts as alternate
// columns: D[p][2n + c] = sum over complex k and part q of A[p][(k, q)]
// B[(k, q)][2n + c] with A = (tm_r, tm_i) and
//   B[(k, 0)][2n] = th_r, B[(k, 1)][2n] = -th_i   (real part)
//   B[(k, 0)][2n+1] = th_i, B[(k, 1)][2n+1] = th_r (imaginary part),
// so one 16 x 16 x 4 product covers two complex k; a column block is 8 images.
// Workgroup: 64 p (16 per wave) x up to 64 n (NCB <= 8 column blocks), K in
// steps of 32 complex values staged in LDS (theta as its B values), the next
// step's tiles loaded into registers while the products run; K split over
// slices whose partial sums a second kernel adds in a fixed order. Operand lanes: lane l gives A[l % 16][l / 16]
// and B[l / 16][l % 16]; the result's register r of lane l is D[l / 16 + 4 r][l % 16].
constexpr int CG_P = 64, CG_N = 64, CG_K = 32;
constexpr int CG_LD = CG_K + 1;  // LDS row stride (complex values)

template <bool PAIRS>
__device__ __forceinline__ void cg_fetch(float2 (&v)[8], const float2* __restrict__ src, int row0, int nrows, int N,
                                         int kb, int k1) {
  // 64 rows x 32 complex values; thread t: rows t / 16 + 16 q, values 2 (t % 16), +1
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = (int)(threadIdx.x >> 4) + 16 * q, kk = 2 * (int)(threadIdx.x & 15);
    const int row = row0 + r, k = kb + kk;
    float2 a = make_float2(0.f, 0.f), b = a;
    if (row < nrows) {
      const float2* s = src + (size_t)row * N + k;
      if (PAIRS) {
        if (k < k1) {  // k1 - k is even
          const float4 w = *(const float4*)s;
          a = make_float2(w.x, w.y);
          b = make_float2(w.z, w.w);
        }
      } else {
        if (k < k1) a = s[0];
        if (k + 1 < k1) b = s[1];
      }
    }
    v[2 * q] = a;
    v[2 * q + 1] = b;
  }
}

__device__ __forceinline__ void cg_store(float2* lds, const float2 (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = (int)(threadIdx.x >> 4) + 16 * q, kk = 2 * (int)(threadIdx.x & 15);
    lds[r * CG_LD + kk] = v[2 * q];
    lds[r * CG_LD + kk + 1] = v[2 * q + 1];
  }
}

// theta as the B operand's four values per complex element: (th_r, -th_i, th_i, th_r)
// at index part + 2 (column parity)
__device__ __forceinline__ void cg_store_b(float4* lds, const float2 (&v)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = (int)(threadIdx.x >> 4) + 16 * q, kk = 2 * (int)(threadIdx.x & 15);
    lds[r * CG_LD + kk] = make_float4(v[2 * q].x, -v[2 * q].y, v[2 * q].y, v[2 * q].x);
    lds[r * CG_LD + kk + 1] = make_float4(v[2 * q + 1].x, -v[2 * q + 1].y, v[2 * q + 1].y, v[2 * q + 1].x);
  }
}

typedef double cg_d4 __attribute__((ext_vector_type(4)));

// NCB column blocks per workgroup (the images of the first n tile; blocks past
// the last image compute zeros from zero-filled rows)
template <bool PAIRS, int NCB>
__global__ void __launch_bounds__(256) k_cgemm_part(const float2* __restrict__ theta, const float2* __restrict__ tm,
                                                    double* __restrict__ part, int Nd, int P, int N, int kchunk) {
  __shared__ float2 sT[CG_P * CG_LD];  // tm tile [p][k]
  __shared__ float4 sH[CG_N * CG_LD];  // theta tile [n][k], four B values per element
  const int p0 = blockIdx.x * CG_P, n0 = blockIdx.y * CG_N, sl = blockIdx.z;
  const int k0 = sl * kchunk, k1 = min(N, k0 + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;  // operand row / column, and k quarter: complex k 2 s + g / 2, part g % 2
  cg_d4 acc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) acc[cb] = cg_d4{0.0, 0.0, 0.0, 0.0};
  float2 vt[8], vh[8];
  cg_fetch<PAIRS>(vt, tm, p0, P, N, k0, k1);
  cg_fetch<PAIRS>(vh, theta, n0, Nd, N, k0, k1);
  for (int kb = k0; kb < k1; kb += CG_K) {
    cg_store(sT, vt);
    cg_store_b(sH, vh);
    __syncthreads();
    if (kb + CG_K < k1) {
      cg_fetch<PAIRS>(vt, tm, p0, P, N, kb + CG_K, k1);
      cg_fetch<PAIRS>(vh, theta, n0, Nd, N, kb + CG_K, k1);
    }
    const float2* ta = sT + (wave * 16 + i) * CG_LD + (g >> 1);
    // this lane's B value of element (n, k): index part + 2 (column parity)
    const float* hb = (const float*)(sH + (i >> 1) * CG_LD + (g >> 1)) + ((g & 1) + 2 * (i & 1));
#pragma unroll 4
    for (int st = 0; st < CG_K / 2; ++st) {
      const float2 t = ta[2 * st];
      const double a = (double)((g & 1) ? t.y : t.x);
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const double b = (double)hb[(cb * 8 * CG_LD + 2 * st) * 4];
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave has read the tiles before the next store
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    const int col = cb * 16 + i, n = n0 + (col >> 1), c = col & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = p0 + wave * 16 + g + 4 * r;
      if (n < Nd && p < P) part[(((size_t)sl * Nd + n) * P + p) * 2 + c] = acc[cb][r];
    }
  }
}

template <bool PAIRS>
static void cgemm_launch(int ncb, dim3 g, hipStream_t s, const float2* th, const float2* tmv, double* part,
                         const PhaseDims& d, int kchunk) {
  switch (ncb) {
#define TM_CG(K) \
  case K: k_cgemm_part<PAIRS, K><<<g, 256, 0, s>>>(th, tmv, part, d.Nd, d.P, d.N, kchunk); break;
    TM_CG(1) TM_CG(2) TM_CG(3) TM_CG(4) TM_CG(5) TM_CG(6) TM_CG(7)
    default: k_cgemm_part<PAIRS, 8><<<g, 256, 0, s>>>(th, tmv, part, d.Nd, d.P, d.N, kchunk);
#undef TM_CG
  }
}

__global__ void __launch_bounds__(256) k_cgemm_sum(const double* __restrict__ part, double* __restrict__ c,
                                                   int64_t n, int gs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < gs; ++k) s += part[(size_t)k * n + i];
  c[i] = s;
}

__device__ __forceinline__ double freq(int k, int n, double ps) {
  int s = (k < (n + 1) / 2) ? k : k - n;
  return (double)s / ((double)n * ps);
}

__global__ void k_make_h(double* h, int nf1, int nf2, double lam, double ps, double NA, double z) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= nf1 * nf2) return;
  int a = i / nf2, b = i % nf2;
  double u = freq(a, nf1, ps), v = freq(b, nf2, ps);
  double rho2 = (lam * u) * (lam * u) + (lam * v) * (lam * v);
  z2 r{0.0, 0.0};
  if (sqrt(rho2) <= NA) {
    double ph = 2.0 * M_PI / lam * sqrt(1.0 - rho2) * z;
    r = {cos(ph), sin(ph)};
  }
  h[2 * i] = r.x;
  h[2 * i + 1] = r.y;
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// inv[g] = p for g = pix[p], -1 elsewhere (pixels are distinct and in range)
// Pixel map and its validation on the device. inv[g] = -1, then the largest
// row p with pix[p] == g; chk[0] |= 1 for an index outside the grid (chk[1] =
// the smallest such row), |= 2 for a pixel that a later row also has
// (chk[2] = the smallest such row). Any problem sets *skip, so that no
// evaluation kernel runs on the map.
__global__ void k_invmap(int32_t* inv, const int32_t* pix, int P, int G, int* chk) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i < G) inv[i] = -1;
  if (i == 0) {
    chk[0] = 0;
    chk[1] = P;
    chk[2] = P;
  }
}
__global__ void k_invmap2(int32_t* inv, const int32_t* pix, int P, int G, int* chk, int* skip) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int g = pix[p];
  if (g >= 0 && g < G) {
    atomicMax(&inv[g], p);
  } else {
    atomicOr(&chk[0], 1);
    atomicMin(&chk[1], p);
    *skip = 1;
  }
}
__global__ void k_invmap3(const int32_t* inv, const int32_t* pix, int P, int G, int* chk, int* skip) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  const int g = pix[p];
  if (g >= 0 && g < G && inv[g] != p) {
    atomicOr(&chk[0], 2);
    atomicMin(&chk[2], p);
    *skip = 1;
  }
}

// ---- separable evaluation of the forward model and its adjoint
// The 2-D transforms are done one axis at a time, each fused with the
// pointwise step that follows it, so every kernel reads one line (a row or a
// column of one image) from memory, transforms it in LDS and writes it once:
//   rows_fwd   F = scatter(c_n u) row by row, DFT along axis 2
//   cols_fwd   DFT along axis 1, times h, zero-pad axis 1, inverse DFT (2 nf1)
//   rows_mid   zero-pad axis 2, inverse DFT (2 nf2) = a_n row; residual
//              r = I - |a|^2 (objective partial sums), a r, DFT (2 nf2), crop
//              (or |a|^2 written out for the image-only forward model)
//   cols_adj   DFT along axis 1 (2 nf1), crop, times conj(h), inverse DFT (nf1)
//   rows_adj   inverse DFT along axis 2 -> A_n^H (a_n r_n) on the field grid
// Every DFT is unitary per axis. The intermediate B holds [Nd][2 nf1][nf2]
// (image rows, axis 2 still in the unpadded frequency order).
constexpr int LINE_ELEMS = 512;  // complex doubles per LDS buffer (lines per workgroup x longest line)
constexpr int LWG = 256;

// Stockham (self-sorting) DFTs of nl lines of length L = 2^l, line i at
// a + i * ls, using b as the ping-pong buffer; every thread of the
// workgroup takes part. Radix-4 steps, with one radix-2 step first when l is
// odd. A step with sub-length p maps butterfly k (i = k mod p) from inputs
// a[k + r L/R] (r < R), twiddled by W_{Rp}^{i r}, through a length-R DFT to
// b[(k - i) R + i + s p]. sign -1: forward (W = e^{-2 pi j / n}); +1: inverse.
// Returns the buffer holding the result.
// The twiddles come from an LDS copy of the table of the longest line
// length Lt (W_L^m = twl[m Lt / L]).
__device__ __forceinline__ z2* lds_fft(z2* a, z2* b, int nl, int ls, int L, int sign, const z2* twl, int Lt) {
  const int tsc = Lt / L;
  int p = 1;
  if (__builtin_ctz((unsigned)L) & 1) {  // radix-2 step
    const int half = L >> 1;
    for (int t = threadIdx.x; t < nl * half; t += LWG) {
      const int line = t / half, k = t - line * half;
      const z2* la = a + line * ls;
      z2* lb = b + line * ls;
      z2 x0 = la[k], x1 = la[k + half];
      lb[2 * k] = {x0.x + x1.x, x0.y + x1.y};
      lb[2 * k + 1] = {x0.x - x1.x, x0.y - x1.y};
    }
    __syncthreads();
    z2* t = a;
    a = b;
    b = t;
    p = 2;
  }
  const int q = L >> 2;
  for (; p < L; p <<= 2) {
    const int ts = (L / (4 * p)) * tsc;  // twiddle stride: W_{4p}^m = twl[m ts]
    for (int t = threadIdx.x; t < nl * q; t += LWG) {
      const int line = t / q, k = t - line * q;
      const z2* la = a + line * ls;
      z2* lb = b + line * ls;
      const int i = k & (p - 1);
      z2 x0 = la[k], x1 = la[k + q], x2 = la[k + 2 * q], x3 = la[k + 3 * q];
      if (p > 1) {
        z2 w1 = twl[i * ts], w2 = twl[2 * i * ts], w3 = twl[3 * i * ts];
        if (sign > 0) {
          w1.y = -w1.y;
          w2.y = -w2.y;
          w3.y = -w3.y;
        }
        x1 = zmul(x1, w1);
        x2 = zmul(x2, w2);
        x3 = zmul(x3, w3);
      }
      // length-4 DFT: the odd outputs turn x1 - x3 by -j (forward) or +j (inverse)
      const z2 s02{x0.x + x2.x, x0.y + x2.y}, d02{x0.x - x2.x, x0.y - x2.y};
      const z2 s13{x1.x + x3.x, x1.y + x3.y}, d13{x1.x - x3.x, x1.y - x3.y};
      const z2 rd = (sign < 0) ? z2{d13.y, -d13.x} : z2{-d13.y, d13.x};
      const int o = ((k - i) << 2) + i;
      lb[o] = {s02.x + s13.x, s02.y + s13.y};
      lb[o + p] = {d02.x + rd.x, d02.y + rd.y};
      lb[o + 2 * p] = {s02.x - s13.x, s02.y - s13.y};
      lb[o + 3 * p] = {d02.x - rd.x, d02.y - rd.y};
    }
    __syncthreads();
    z2* t = a;
    a = b;
    b = t;
  }
  return a;
}

// LDS copy of the twiddle table W_L^m (m < L); the caller's next barrier
// publishes it.
__device__ __forceinline__ void load_tw(z2* twl, const double* tw64, int L) {
  const z2* tw = (const z2*)tw64 + (L - 1);
  for (int t = threadIdx.x; t < L; t += LWG) twl[t] = tw[t];
}

__device__ __forceinline__ int padpos(int k, int n) {
  int s = (k < (n + 1) / 2) ? k : k - n;
  return (s + 2 * n) % (2 * n);
}

// field bin of a doubled-spectrum index (inverse of padpos), -1 if that bin is padding
__device__ __forceinline__ int unpad(int a2, int n) {
  int hp = (n + 1) / 2;
  if (a2 < hp) return a2;
  if (a2 >= n + hp) return a2 - n;
  return -1;
}

// complex entry i of an interleaved (re, im) double array
__device__ __forceinline__ z2 ldz(const double* p, size_t i) { return z2{p[2 * i], p[2 * i + 1]}; }
__device__ __forceinline__ void stz(double* p, size_t i, z2 v) {
  p[2 * i] = v.x;
  p[2 * i + 1] = v.y;
}

__device__ __forceinline__ int lines_per_wg(int Lmax) { return Lmax >= LINE_ELEMS ? 1 : LINE_ELEMS / Lmax; }

// rows of F_n: F[n][a][b] = c[n][p] e^{j phi_p} where a nf2 + b = pix[p], 0 elsewhere;
// DFT along axis 2 -> A[n][a][:]
__global__ void __launch_bounds__(LWG) k_rows_fwd(double* A, const double* c, const double* phi, const int32_t* inv,
                                                  int Nd, int P, int nf1, int nf2, const double* tw64,
                                                  const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 sa[LINE_ELEMS], sb[LINE_ELEMS], stw[LINE_ELEMS];
  const int L = nf2, nl = lines_per_wg(L), nlines = Nd * nf1;
  const int l0 = blockIdx.x * nl;
  load_tw(stw, tw64, L);
  for (int t = threadIdx.x; t < nl * L; t += LWG) {
    const int line = t / L, j = t - line * L, gl = l0 + line;
    z2 v{0.0, 0.0};
    if (gl < nlines) {
      const int n = gl / nf1, a = gl - n * nf1;
      const int p = inv[a * nf2 + j];
      if (p >= 0) {
        z2 cv{c[((size_t)n * P + p) * 2], c[((size_t)n * P + p) * 2 + 1]};
        double sn, cs;
        sincos(phi[p], &sn, &cs);
        v = zmul(cv, z2{cs, sn});
      }
    }
    sa[line * L + j] = v;
  }
  __syncthreads();
  const z2* r = lds_fft(sa, sb, nl, L, L, -1, stw, L);
  const double sc = 1.0 / sqrt((double)L);
  for (int t = threadIdx.x; t < nl * L; t += LWG) {
    const int line = t / L, gl = l0 + line;
    if (gl < nlines) {
      z2 v = r[t];
      stz(A, (size_t)gl * L + (t - line * L), z2{v.x * sc, v.y * sc});
    }
  }
}

// columns: A[n][:][b] -> DFT (nf1), times h[:][b], pad to 2 nf1, inverse DFT -> B[n][:][b]
__global__ void __launch_bounds__(LWG) k_cols_fwd(double* B, const double* A, const double* h, int Nd, int nf1,
                                                  int nf2, const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 sa[LINE_ELEMS], sb[LINE_ELEMS], stw[LINE_ELEMS];
  const int L1 = nf1, L2 = 2 * nf1, nl = lines_per_wg(L2), ncols = Nd * nf2;
  const int l0 = blockIdx.x * nl;
  load_tw(stw, tw64, L2);
  // consecutive threads read consecutive columns of one row
  for (int t = threadIdx.x; t < nl * L1; t += LWG) {
    const int a = t / nl, line = t - a * nl, gl = l0 + line;
    z2 v{0.0, 0.0};
    if (gl < ncols) {
      const int n = gl / nf2, b = gl - n * nf2;
      v = ldz(A, ((size_t)n * nf1 + a) * nf2 + b);
    }
    sa[line * L2 + a] = v;
  }
  // kernel values of this thread's padded elements, loaded before the transforms
  z2 hv[LINE_ELEMS / LWG];
#pragma unroll
  for (int k = 0; k < LINE_ELEMS / LWG; ++k) {
    const int t = threadIdx.x + k * LWG, line = t / L2, gl = l0 + line;
    const int a = unpad(t - line * L2, nf1);
    hv[k] = z2{0.0, 0.0};
    if (a >= 0 && gl < ncols) {
      const int b = gl % nf2;
      hv[k] = z2{h[2 * (a * nf2 + b)], h[2 * (a * nf2 + b) + 1]};
    }
  }
  __syncthreads();
  z2* r = lds_fft(sa, sb, nl, L2, L1, -1, stw, L2);
  z2* q = (r == sa) ? sb : sa;
  const double s1 = 1.0 / sqrt((double)L1);
#pragma unroll
  for (int k = 0; k < LINE_ELEMS / LWG; ++k) {
    const int t = threadIdx.x + k * LWG, line = t / L2, a2 = t - line * L2, gl = l0 + line;
    const int a = unpad(a2, nf1);
    z2 v{0.0, 0.0};
    if (a >= 0 && gl < ncols) {
      z2 x = r[line * L2 + a];
      v = zmul(z2{x.x * s1, x.y * s1}, hv[k]);
    }
    q[t] = v;
  }
  __syncthreads();
  const z2* o = lds_fft(q, r, nl, L2, L2, +1, stw, L2);
  const double s2 = 1.0 / sqrt((double)L2);
  for (int t = threadIdx.x; t < nl * L2; t += LWG) {
    const int a2 = t / nl, line = t - a2 * nl, gl = l0 + line;
    if (gl < ncols) {
      const int n = gl / nf2, b = gl - n * nf2;
      z2 v = o[line * L2 + a2];
      stz(B, ((size_t)n * L2 + a2) * nf2 + b, z2{v.x * s2, v.y * s2});
    }
  }
}

// image rows: B[n][a2][:] -> pad to 2 nf2, inverse DFT = a_n[a2][:].
// Id != null: r = I - |a|^2, partial sum of r^2 per workgroup into gpart,
// a r -> DFT (2 nf2) -> crop -> B[n][a2][:]. Id == null: |a|^2 -> I_out.
__global__ void __launch_bounds__(LWG) k_rows_mid(double* B, const float* Id, double* gpart, float* I_out, int Nd,
                                                  int nf1, int nf2, const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 sa[LINE_ELEMS], sb[LINE_ELEMS], stw[LINE_ELEMS];
  __shared__ double red[LWG / 64];
  const int L = 2 * nf2, nl = lines_per_wg(L), nlines = Nd * 2 * nf1;
  const int l0 = blockIdx.x * nl;
  load_tw(stw, tw64, L);
  for (int t = threadIdx.x; t < nl * L; t += LWG) {
    const int line = t / L, b2 = t - line * L, gl = l0 + line;
    const int b = unpad(b2, nf2);
    z2 v{0.0, 0.0};
    if (b >= 0 && gl < nlines) v = ldz(B, (size_t)gl * nf2 + b);
    sa[t] = v;
  }
  // the measured intensities of this thread's elements, loaded before the transforms
  float idv[LINE_ELEMS / LWG];
#pragma unroll
  for (int k = 0; k < LINE_ELEMS / LWG; ++k) {
    const int t = threadIdx.x + k * LWG, gl = l0 + t / L;
    idv[k] = (Id && gl < nlines) ? Id[(size_t)l0 * L + t] : 0.f;
  }
  __syncthreads();
  z2* r = lds_fft(sa, sb, nl, L, L, +1, stw, L);
  const double s2 = 1.0 / sqrt((double)L);
  if (!Id) {
    for (int t = threadIdx.x; t < nl * L; t += LWG) {
      const int gl = l0 + t / L;
      if (gl < nlines) {
        z2 v = r[t];
        I_out[(size_t)l0 * L + t] = (float)((v.x * v.x + v.y * v.y) * (s2 * s2));
      }
    }
    return;
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < LINE_ELEMS / LWG; ++k) {
    const int t = threadIdx.x + k * LWG, gl = l0 + t / L;
    z2 v = r[t];
    v = {v.x * s2, v.y * s2};
    double res = 0.0;
    if (gl < nlines) {
      res = (double)idv[k] - (v.x * v.x + v.y * v.y);
      acc += res * res;
    }
    r[t] = {v.x * res, v.y * res};
  }
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) gpart[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  z2* q = (r == sa) ? sb : sa;
  const z2* o = lds_fft(r, q, nl, L, L, -1, stw, L);
  for (int t = threadIdx.x; t < nl * nf2; t += LWG) {
    const int line = t / nf2, b = t - line * nf2, gl = l0 + line;
    if (gl < nlines) {
      z2 v = o[line * L + padpos(b, nf2)];
      stz(B, (size_t)gl * nf2 + b, z2{v.x * s2, v.y * s2});
    }
  }
}

// columns: B[n][:][b] -> DFT (2 nf1), crop, times conj(h[:][b]), inverse DFT (nf1) -> A[n][:][b]
__global__ void __launch_bounds__(LWG) k_cols_adj(double* A, const double* B, const double* h, int Nd, int nf1,
                                                  int nf2, const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 sa[LINE_ELEMS], sb[LINE_ELEMS], stw[LINE_ELEMS];
  const int L1 = nf1, L2 = 2 * nf1, nl = lines_per_wg(L2), ncols = Nd * nf2;
  const int l0 = blockIdx.x * nl;
  load_tw(stw, tw64, L2);
  for (int t = threadIdx.x; t < nl * L2; t += LWG) {
    const int a2 = t / nl, line = t - a2 * nl, gl = l0 + line;
    z2 v{0.0, 0.0};
    if (gl < ncols) {
      const int n = gl / nf2, b = gl - n * nf2;
      v = ldz(B, ((size_t)n * L2 + a2) * nf2 + b);
    }
    sa[line * L2 + a2] = v;
  }
  // kernel values of this thread's cropped elements, loaded before the transforms
  constexpr int NC = (LINE_ELEMS / 2 + LWG - 1) / LWG;
  z2 hv[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int t = threadIdx.x + k * LWG, line = t / L1, a = t - line * L1, gl = l0 + line;
    hv[k] = z2{0.0, 0.0};
    if (t < nl * L1 && gl < ncols) {
      const int b = gl % nf2;
      hv[k] = z2{h[2 * (a * nf2 + b)], h[2 * (a * nf2 + b) + 1]};
    }
  }
  __syncthreads();
  z2* r = lds_fft(sa, sb, nl, L2, L2, -1, stw, L2);
  z2* q = (r == sa) ? sb : sa;
  const double s2 = 1.0 / sqrt((double)L2);
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int t = threadIdx.x + k * LWG, line = t / L1, a = t - line * L1, gl = l0 + line;
    if (t < nl * L1) {
      z2 v{0.0, 0.0};
      if (gl < ncols) {
        z2 x = r[line * L2 + padpos(a, nf1)];
        v = zmulc(z2{x.x * s2, x.y * s2}, hv[k]);
      }
      q[line * L2 + a] = v;
    }
  }
  __syncthreads();
  const z2* o = lds_fft(q, r, nl, L2, L1, +1, stw, L2);
  const double s1 = 1.0 / sqrt((double)L1);
  for (int t = threadIdx.x; t < nl * L1; t += LWG) {
    const int a = t / nl, line = t - a * nl, gl = l0 + line;
    if (gl < ncols) {
      const int n = gl / nf2, b = gl - n * nf2;
      z2 v = o[line * L2 + a];
      stz(A, ((size_t)n * nf1 + a) * nf2 + b, z2{v.x * s1, v.y * s1});
    }
  }
}

// rows: A[n][a][:] -> inverse DFT along axis 2 (in place)
__global__ void __launch_bounds__(LWG) k_rows_adj(double* A, int Nd, int nf1, int nf2, const double* tw64,
                                                  const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 sa[LINE_ELEMS], sb[LINE_ELEMS], stw[LINE_ELEMS];
  const int L = nf2, nl = lines_per_wg(L), nlines = Nd * nf1;
  const int l0 = blockIdx.x * nl;
  load_tw(stw, tw64, L);
  for (int t = threadIdx.x; t < nl * L; t += LWG) {
    const int gl = l0 + t / L;
    sa[t] = (gl < nlines) ? ldz(A, (size_t)l0 * L + t) : z2{0.0, 0.0};
  }
  __syncthreads();
  const z2* r = lds_fft(sa, sb, nl, L, L, +1, stw, L);
  const double sc = 1.0 / sqrt((double)L);
  for (int t = threadIdx.x; t < nl * L; t += LWG) {
    const int gl = l0 + t / L;
    if (gl < nlines) {
      z2 v = r[t];
      stz(A, (size_t)l0 * L + t, z2{v.x * sc, v.y * sc});
    }
  }
}

// Partial w_s[p] = sum over the images n of slice s of conj(c[n][p]) A[n][pix[p]]:
// threads run over consecutive p (coalesced c reads), grid.y over image slices.
__global__ void __launch_bounds__(256) k_gather_part(double* wpart, const double* A, const double* c,
                                                      const int32_t* pix, int Nd, int P, int G, int per,
                                                      const int* skip) {
  if (skip && *skip) return;
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  int n0 = blockIdx.y * per, n1 = min(Nd, n0 + per);
  int g = pix[p];
  z2 w{0.0, 0.0};
  for (int n = n0; n < n1; ++n) {
    size_t o = ((size_t)n * G + g) * 2;
    z2 v{A[o], A[o + 1]};
    z2 cv{c[((size_t)n * P + p) * 2], c[((size_t)n * P + p) * 2 + 1]};
    z2 t = zmulc(v, cv);
    w.x += t.x;
    w.y += t.y;
  }
  wpart[((size_t)blockIdx.y * P + p) * 2] = w.x;
  wpart[((size_t)blockIdx.y * P + p) * 2 + 1] = w.y;
}

// Partial sum of dvec^T grad over the 64 pixels of this wave (wave-uniform
// call; lanes past P pass gr = 0), into dpart[pixel / 64].
__device__ __forceinline__ void dot_part(const double* dvec, double* dpart, int p, int P, double gr) {
  double x = (p < P) ? dvec[p] * gr : 0.0;
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) dpart[p >> 6] = x;
}

// grad[p] = -4 Im(conj(u_p) w[p]) with w the sum of the slices; gval = sum of
// the residual partials; with dvec, the partials of dvec^T grad
__global__ void __launch_bounds__(256) k_gather(double* grad, double* gval, const double* wpart, const double* phi,
                                                 const double* gpart, int ngp, int nslice, int P, const int* skip,
                                                 const double* dvec, double* dpart) {
  if (skip && *skip) return;
  int p = blockIdx.x * 256 + threadIdx.x;
  double gr = 0.0;
  if (p < P) {
    z2 w{0.0, 0.0};
    for (int sl = 0; sl < nslice; ++sl) {
      w.x += wpart[((size_t)sl * P + p) * 2];
      w.y += wpart[((size_t)sl * P + p) * 2 + 1];
    }
    double sn, cs;
    sincos(phi[p], &sn, &cs);
    z2 q = zmulc(w, z2{cs, sn});  // w conj(u)
    gr = -4.0 * q.y;
    grad[p] = gr;
  }
  if (dvec) dot_part(dvec, dpart, p, P, gr);
  if (blockIdx.x == 0) {  // objective: block-wide sum of the residual partials
    __shared__ double red[4];
    double s = 0;
    for (int i = threadIdx.x; i < ngp; i += 256) s += gpart[i];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gval[0] = red[0] + red[1] + red[2] + red[3];
  }
}


// ---- pupil-band evaluation
// The same model and adjoint with the transforms pruned to the box of
// spectrum bins where h can be nonzero (signed frequencies s1 in
// [s1lo, s1lo + B1), s2 in [s2lo, s2lo + B2)). Five passes, each spread over
// many workgroups (the work per evaluation is small, so the passes are
// bound by latency, not by arithmetic):
//   band_spec (image x block of field rows): DFT of the field rows at the B2
//     box frequencies, then along axis 1 at the B1 box frequencies over the
//     block's rows: partial box spectra Sp[n][chunk][i1][i2]
//   band_img (image x block of image rows x column chunk): S = sum of the
//     partials, H = S h, the column's T[i1] = sum_i2 H[i1][i2] e^{+2 pi j s2 x2 / 2nf2};
//     for each row a = sum_i1 T[i1] e^{+2 pi j s1 x1 / 2nf1}, r = I - |a|^2
//     (objective partials) and the adjoint along axis 1,
//     U[i1][x2] = sum_x1 a r e^{-2 pi j s1 x1 / 2nf1}, per row block
//   band_v (image x box row i1): sum of the row blocks, DFT along axis 2 at
//     the box frequencies, times conj(h): V[n][i1][i2]
//   band_pix (image x block of pixels): inverse DFTs back to the field
//     pixels, times conj(c_n): Wn[n][p]
//   band_gather: w_p = sum_n Wn[n][p], gradient -4 Im(conj(u_p) w_p), objective
// Unitary scales as in the separable path: 1/(2 nf1 nf2) for the forward
// chain and for the adjoint chain.
constexpr int BM = 16;           // largest box side
// Field values per workgroup of the spectrum pass (RA = SPEC_FIELD / nf2 rows)
// and blocks of 256 pixels per workgroup of the pass back to the pixels (which
// share one image's Z). Measured at 64 x 64 with 50 images: 1024 values and 3
// blocks (200 and 150 workgroups per evaluation instead of 400 and 450) left
// the pipelined step unchanged (10.23 against 10.28 ms) and made the phase
// solve alone 0.1 ms slower.
constexpr int SPEC_FIELD = 512;
constexpr int PIX_BLOCKS = 1;

__device__ __forceinline__ z2 zfma(z2 a, z2 b, z2 acc) {  // acc + a b
  return {acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ z2 zfmac(z2 a, z2 b, z2 acc) {  // acc + a conj(b)
  return {acc.x + a.x * b.x + a.y * b.y, acc.y + a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ z2 zadd(z2 a, z2 b) { return {a.x + b.x, a.y + b.y}; }

// e^{-2 pi j m / L} of the table of length L (power of two) into LDS
__device__ __forceinline__ void load_tab(z2* dst, const double* tw64, int L, int nt) {
  const z2* tw = (const z2*)tw64 + (L - 1);
  for (int t = threadIdx.x; t < L; t += nt) dst[t] = tw[t];
}

__global__ void __launch_bounds__(256) k_band_spec(double* Sp, const double* c, const double* phi,
                                                   const int32_t* inv, PhaseBand b, int P, int nf1, int nf2,
                                                   const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 F[SPEC_FIELD];
  __shared__ z2 S1[SPEC_FIELD];  // RA B2 <= (SPEC_FIELD / nf2) nf2 outputs
  __shared__ z2 tw1[256], tw2[256];
  const int ch = blockIdx.x, n = blockIdx.y, a0 = ch * b.RA;
  const int ne = b.RA * nf2;  // <= SPEC_FIELD field values
  // the block's field values: pixel rows first (loads issued together)
  constexpr int FPT = SPEC_FIELD / 256;
  int pp[FPT];
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int t = threadIdx.x + k * 256;
    pp[k] = (t < ne) ? inv[(size_t)a0 * nf2 + t] : -1;
  }
  load_tab(tw1, tw64, nf1, 256);
  load_tab(tw2, tw64, nf2, 256);
#pragma unroll
  for (int k = 0; k < FPT; ++k) {
    const int t = threadIdx.x + k * 256;
    z2 v{0.0, 0.0};
    if (pp[k] >= 0) {
      double sn, cs;
      sincos(phi[pp[k]], &sn, &cs);
      v = zmul(ldz(c, (size_t)n * P + pp[k]), z2{cs, sn});
    }
    if (t < ne) F[t] = v;
  }
  __syncthreads();
  // S1[r][i2] = sum_b F[r][b] e^{-2 pi j s2 b / nf2}; the terms of one output split over q threads
  const int nout = b.RA * b.B2;
  int q = 1;
  while (q < 16 && nout * q * 2 <= 256) q *= 2;
  for (int o0 = 0; o0 < nout; o0 += 256 / q) {  // more outputs than thread groups: several rounds
    const int o = o0 + threadIdx.x / q, part = threadIdx.x % q;
    z2 acc{0.0, 0.0};
    if (o < nout) {
      const int r = o / b.B2, j2 = o - r * b.B2;
      const int sm = (b.s2lo + j2) & (nf2 - 1);
      const z2* fr = F + r * nf2;
#pragma unroll 4
      for (int bb = part; bb < nf2; bb += q) acc = zfma(fr[bb], tw2[(sm * bb) & (nf2 - 1)], acc);
    }
    for (int off = 1; off < q; off <<= 1) {  // q consecutive lanes of one wave
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (o < nout && part == 0) S1[o] = acc;
  }
  __syncthreads();
  // partial box spectrum over this block's rows
  for (int t = threadIdx.x; t < b.B1 * b.B2; t += 256) {
    const int i1 = t / b.B2, i2 = t - i1 * b.B2;
    const int sm = (b.s1lo + i1) & (nf1 - 1);
    z2 acc{0.0, 0.0};
    for (int r = 0; r < b.RA; ++r) acc = zfma(S1[r * b.B2 + i2], tw1[(sm * (a0 + r)) & (nf1 - 1)], acc);
    stz(Sp, ((size_t)n * b.CH + ch) * (BM * BM) + i1 * BM + i2, acc);
  }
}

// cos and sin of 2 pi m / 16, m < 8
__device__ constexpr double c16(int m) {
  return m == 0 ? 1.0 : m == 1 ? 0.92387953251128674 : m == 2 ? 0.70710678118654757 : m == 3 ? 0.38268343236508978
         : m == 4 ? 0.0 : m == 5 ? -0.38268343236508978 : m == 6 ? -0.70710678118654757 : -0.92387953251128674;
}
__device__ constexpr double s16(int m) { return c16(m < 4 ? 4 - m : m - 4); }
__device__ constexpr int bitrev_n(int i, int n) {
  int r = 0;
  for (int b = 1; b < n; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

// In-register DFT of length N (4, 8 or 16): x_k <- sum_j x_j e^{SIGN 2 pi i j k / N},
// radix-2 decimation in time with compile-time indices and twiddles.
template <int N, int SIGN>
__device__ __forceinline__ void reg_dft(z2* x) {
  z2 y[N];
#pragma unroll
  for (int i = 0; i < N; ++i) y[bitrev_n(i, N)] = x[i];
#pragma unroll
  for (int half = 1; half < N; half <<= 1) {
#pragma unroll
    for (int g = 0; g < N; g += 2 * half) {
#pragma unroll
      for (int k = 0; k < half; ++k) {
        const int m = k * (16 / (2 * half));  // W_{2 half}^k = e^{SIGN 2 pi i m / 16}
        const z2 v = y[g + k + half];
        z2 t;
        if (m == 0) t = v;
        else if (m == 4) t = (SIGN > 0) ? z2{-v.y, v.x} : z2{v.y, -v.x};
        else t = zmul(v, z2{c16(m), SIGN * s16(m)});
        y[g + k + half] = z2{y[g + k].x - t.x, y[g + k].y - t.y};
        y[g + k] = z2{y[g + k].x + t.x, y[g + k].y + t.y};
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = y[i];
}

// Image pass. Rows x1 = G k + l (k < BT1) of one column belong to thread l of
// the column's G = 2nf1 / BT1 threads. With box row j at signed frequency
// s1lo + j and e^{2 pi i j x1 / 2nf1} = e^{2 pi i j k / BT1} e^{2 pi i j l / 2nf1},
//   a[G k + l] = e^{2 pi i s1lo x1 / 2nf1} A_k,
//   A = DFT+_BT1 (T[j] e^{2 pi i j l / 2nf1}),
// so |a|^2 = |A_k|^2, and the adjoint's first axis,
// sum_x1 a r e^{-2 pi i (s1lo + j) x1 / 2nf1}, is per thread
// e^{-2 pi i j l / 2nf1} DFT-_BT1 (A r)[j] (the phase factor cancels). The G
// threads of a column then add their parts: the workgroup writes whole
// columns of U. A length-BT1 DFT per BT1 pixels replaces BT1 terms per pixel.
// BT1: the box's axis-1 side padded to 4, 8 or 16 (rows beyond B1 are zero).
// At least three waves per SIMD (168 VGPRs at BT1 = 16, a few spilled): with
// 53 KiB of LDS three workgroups then fit a CU beside each other, which is what
// counts when the solve runs beside a retrieval (pipelined step 9.77 -> 9.74 ms;
// the solve alone 0.03 ms slower).
template <int BT1>
__global__ void __launch_bounds__(256, 3) k_band_img(double* Vp, double* gpart, const double* Sp, const float* Id,
                                                  const double* h, PhaseBand b, int nf1, int nf2,
                                                  const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 H[BM * BM];
  __shared__ z2 twl1[512], twl2[512];
  // box rows of the image-axis-2 transform, [j][column of the workgroup] (BT1 CPW <= BT1 / 2 * 256: G >= 2)
  __shared__ z2 TC[BT1 / 2 * 256];
  __shared__ double wred[4];
  z2* stage = TC;  // reused for the adjoint partials of half the box rows, [j][l][column], then U [j][column]
  const int L1 = 2 * nf1, L2 = 2 * nf2, G = b.G, CPW = b.CPW;
  const int n = blockIdx.y;
  const int cl = threadIdx.x % CPW, l = threadIdx.x / CPW;
  const int col = blockIdx.x * CPW + cl;
  const bool colok = col < L2;
  // this thread's measured pixels, loaded first
  float idv[BT1];
#pragma unroll
  for (int k = 0; k < BT1; ++k) idv[k] = colok ? Id[((size_t)n * L1 + G * k + l) * L2 + col] : 0.f;
  load_tab(twl1, tw64, L1, 256);
  load_tab(twl2, tw64, L2, 256);
  // box spectrum (sum of the row-block partials) times h and the forward scale
  const double sc = 1.0 / (2.0 * (double)nf1 * (double)nf2);
  for (int t = threadIdx.x; t < BT1 * BM; t += 256) {
    const int i1 = t / BM, i2 = t % BM;
    z2 v{0.0, 0.0};
    if (i1 < b.B1 && i2 < b.B2) {
      const int k1 = (b.s1lo + i1) & (nf1 - 1), k2 = (b.s2lo + i2) & (nf2 - 1);
      const z2 hv = ldz(h, (size_t)k1 * nf2 + k2);
      const double* sp = Sp + ((size_t)n * b.CH * (BM * BM) + i1 * BM + i2) * 2;
      z2 acc{0.0, 0.0};
#pragma unroll 8
      for (int k = 0; k < b.CH; ++k) acc = zadd(acc, z2{sp[(size_t)k * BM * BM * 2], sp[(size_t)k * BM * BM * 2 + 1]});
      v = zmul(acc, hv);
      v = z2{v.x * sc, v.y * sc};
    }
    H[t] = v;
  }
  __syncthreads();
  // T[j][col] = sum_i2 H[j][i2] e^{+2 pi i s2 col / L2}: the column's threads share the rows j
  for (int j = l; j < BT1; j += G) {
    z2 acc{0.0, 0.0};
    if (colok)
      for (int i2 = 0; i2 < b.B2; ++i2) {
        const int sm = (b.s2lo + i2) & (L2 - 1);
        acc = zfmac(H[j * BM + i2], twl2[(sm * col) & (L2 - 1)], acc);
      }
    TC[j * CPW + cl] = acc;
  }
  __syncthreads();
  z2 x[BT1];
#pragma unroll
  for (int j = 0; j < BT1; ++j) x[j] = zmulc(TC[j * CPW + cl], twl1[(j * l) & (L1 - 1)]);  // e^{+2 pi i j l / L1}
  reg_dft<BT1, 1>(x);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < BT1; ++k) {
    const double res = colok ? (double)idv[k] - (x[k].x * x[k].x + x[k].y * x[k].y) : 0.0;
    acc += res * res;
    x[k] = z2{x[k].x * res, x[k].y * res};
  }
  reg_dft<BT1, -1>(x);
  // objective partial of this workgroup
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = acc;
  __syncthreads();  // also: every thread has read TC
  if (threadIdx.x == 0) gpart[(size_t)n * gridDim.x + blockIdx.x] = (wred[0] + wred[1]) + (wred[2] + wred[3]);
  // the column's adjoint: its G threads' parts added, half the box rows at a
  // time through LDS (half the bytes of staging them all: two workgroups fit a
  // CU), the sums held in registers until both halves are done
  constexpr int JH = BT1 / 2;
  constexpr int RPH = JH / 2;  // outputs per thread and half: JH CPW / 256 = JH / G with G >= 2
  z2 us[2][RPH];
#pragma unroll
  for (int hf = 0; hf < 2; ++hf) {
    if (hf) __syncthreads();  // every thread has read the first half's partials
#pragma unroll
    for (int jj = 0; jj < JH; ++jj) {
      const int j = hf * JH + jj;
      stage[(jj * G + l) * CPW + cl] = zmul(x[j], twl1[(j * l) & (L1 - 1)]);  // e^{-2 pi i j l / L1}
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RPH; ++k) {
      const int o = threadIdx.x + k * 256;
      const int jj = o / CPW, c2 = o - jj * CPW;
      z2 sacc{0.0, 0.0};
      if (jj < JH && hf * JH + jj < b.B1)
        for (int q = 0; q < G; ++q) sacc = zadd(sacc, stage[(jj * G + q) * CPW + c2]);
      us[hf][k] = sacc;
    }
  }
  __syncthreads();  // every thread has read the second half's partials
  // U[j][column] at j CPW + column
#pragma unroll
  for (int hf = 0; hf < 2; ++hf)
#pragma unroll
    for (int k = 0; k < RPH; ++k) {
      const int o = threadIdx.x + k * 256;
      if (o < JH * CPW) stage[hf * JH * CPW + o] = us[hf][k];
    }
  __syncthreads();
  // adjoint along axis 2 at the box frequencies over this workgroup's columns:
  // Vp[n][block][i1][i2] = sum_col U[i1][col] e^{-2 pi i s2 col / L2} (the blocks are added by band_pix)
  for (int t = threadIdx.x; t < b.B1 * b.B2; t += 256) {
    const int i1 = t / b.B2, i2 = t - (t / b.B2) * b.B2;
    const int sm = (b.s2lo + i2) & (L2 - 1);
    z2 acc{0.0, 0.0};
    for (int c2 = 0; c2 < CPW; ++c2) {
      const int cc = blockIdx.x * CPW + c2;
      if (cc < L2) acc = zfma(stage[i1 * CPW + c2], twl2[(sm * cc) & (L2 - 1)], acc);
    }
    stz(Vp, (((size_t)n * gridDim.x + blockIdx.x) * BM + i1) * BM + i2, acc);
  }
}

// Wn[n][p] = conj(c[n][p]) sum_i1 e^{+2 pi j s1 a_p / nf1} sum_i2 V[n][i1][i2] e^{+2 pi j s2 b_p / nf2}
__global__ void __launch_bounds__(256) k_band_pix(double* Wn, const double* Vp, const double* c, const double* h,
                                                  const int32_t* pix, PhaseBand b, int P, int nf1, int nf2,
                                                  const double* tw64, const int* skip) {
  if (skip && *skip) return;
  __shared__ z2 V[BM * BM];
  __shared__ z2 tw1[256], tw2[256];
  extern __shared__ z2 Z[];  // [B1][nf2], sized at launch (fewer bytes, more workgroups per CU)
  const int n = blockIdx.y;
  // PIX_BLOCKS blocks of 256 pixels per workgroup share its V and Z (their loads issued first)
  int g[PIX_BLOCKS];
  z2 cv[PIX_BLOCKS];
#pragma unroll
  for (int k = 0; k < PIX_BLOCKS; ++k) {
    const int p = (blockIdx.x * PIX_BLOCKS + k) * 256 + threadIdx.x;
    g[k] = 0;
    cv[k] = z2{0.0, 0.0};
    if (p < P) {
      g[k] = pix[p];
      cv[k] = ldz(c, (size_t)n * P + p);
    }
  }
  // V = conj(h) sc (sum of the image pass's column-block partials)
  const double sc = 1.0 / (2.0 * (double)nf1 * (double)nf2);
  for (int t = threadIdx.x; t < b.B1 * BM; t += 256) {
    const int i1 = t / BM, i2 = t % BM;
    z2 v{0.0, 0.0};
    if (i2 < b.B2) {
      const int k1 = (b.s1lo + i1) & (nf1 - 1), k2 = (b.s2lo + i2) & (nf2 - 1);
      const z2 hv = ldz(h, (size_t)k1 * nf2 + k2);
      z2 acc{0.0, 0.0};
#pragma unroll 4
      for (int q = 0; q < b.NXB; ++q) acc = zadd(acc, ldz(Vp, ((size_t)n * b.NXB + q) * BM * BM + t));
      v = zmulc(acc, hv);
      v = z2{v.x * sc, v.y * sc};
    }
    V[t] = v;
  }
  load_tab(tw1, tw64, nf1, 256);
  load_tab(tw2, tw64, nf2, 256);
  __syncthreads();
  for (int t = threadIdx.x; t < b.B1 * nf2; t += 256) {
    const int j1 = t / nf2, bb = t & (nf2 - 1);
    z2 acc{0.0, 0.0};
    for (int j2 = 0; j2 < b.B2; ++j2) {
      const int sm = (b.s2lo + j2) & (nf2 - 1);
      acc = zfmac(V[j1 * BM + j2], tw2[(sm * bb) & (nf2 - 1)], acc);
    }
    Z[j1 * nf2 + bb] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PIX_BLOCKS; ++k) {
    const int p = (blockIdx.x * PIX_BLOCKS + k) * 256 + threadIdx.x;
    if (p < P) {
      const int a = g[k] / nf2, bb = g[k] & (nf2 - 1);
      z2 acc{0.0, 0.0};
      for (int j1 = 0; j1 < b.B1; ++j1) {
        const int sm = (b.s1lo + j1) & (nf1 - 1);
        acc = zfmac(Z[j1 * nf2 + bb], tw1[(sm * a) & (nf1 - 1)], acc);
      }
      stz(Wn, (size_t)n * P + p, zmulc(acc, cv[k]));
    }
  }
}

// grad[p] = -4 Im(conj(u_p) sum_n Wn[n][p]); gval = sum of the objective partials;
// with dvec, the partial of dvec^T grad over the workgroup's 64 pixels.
// 64 pixels x 4 slices of the images per workgroup: each thread adds its
// slice (loads issued together), the four slices meet in LDS
__global__ void __launch_bounds__(256) k_band_gather(double* grad, double* gval, const double* Wn, const double* phi,
                                                     const double* gpart, int ngp, int Nd, int P, const int* skip,
                                                     const double* dvec, double* dpart) {
  if (skip && *skip) return;
  __shared__ z2 part[4][64];
  const int pl = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + pl;
  const int per = (Nd + 3) / 4, n0 = sl * per, n1 = min(Nd, n0 + per);
  z2 w{0.0, 0.0};
  if (p < P) {
#pragma unroll 16
    for (int n = n0; n < n1; ++n) w = zadd(w, ldz(Wn, (size_t)n * P + p));
  }
  part[sl][pl] = w;
  __syncthreads();
  if (sl == 0) {  // the first wave
    double gr = 0.0;
    if (p < P) {
      w = zadd(zadd(part[0][pl], part[1][pl]), zadd(part[2][pl], part[3][pl]));
      double sn, cs;
      sincos(phi[p], &sn, &cs);
      gr = -4.0 * zmulc(w, z2{cs, sn}).y;
      grad[p] = gr;
    }
    if (dvec) dot_part(dvec, dpart, p, P, gr);
  }
  if (blockIdx.x == 0) {
    __shared__ double red[4];
    double s = 0;
    for (int i = threadIdx.x; i < ngp; i += 256) s += gpart[i];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gval[0] = red[0] + red[1] + red[2] + red[3];
  }
}

// pass geometry (depends on the dimensions only, except BT1 and G: the plan sets them)
void band_geometry(const PhaseDims& d, PhaseBand* b) {
  b->RA = std::max(1, std::min(d.nf1, SPEC_FIELD / d.nf2));
  b->CH = d.nf1 / b->RA;
}

int band_bt1(int B1) { return B1 <= 4 ? 4 : B1 <= 8 ? 8 : 16; }

int grid_of(int nlines, int Lmax) {
  const int nl = Lmax >= LINE_ELEMS ? 1 : LINE_ELEMS / Lmax;
  return (nlines + nl - 1) / nl;
}

// workgroups of the image-row kernel = objective partial sums per evaluation
int mid_groups(const PhaseDims& d) { return grid_of(d.Nd * 2 * d.nf1, 2 * d.nf2); }

// scatter + forward model up to the image rows (B holds image rows in the
// unpadded axis-2 frequency order)
int forward_to_rows(const PhaseDims& d, const double* phi, PhaseWork& w, const double* tw64, hipStream_t s) {
  k_rows_fwd<<<grid_of(d.Nd * d.nf1, d.nf2), LWG, 0, s>>>(w.A, w.c, phi, w.inv, d.Nd, d.P, d.nf1, d.nf2, tw64,
                                                          w.skip);
  k_cols_fwd<<<grid_of(d.Nd * d.nf2, 2 * d.nf1), LWG, 0, s>>>(w.B, w.A, w.h, d.Nd, d.nf1, d.nf2, tw64, w.skip);
  return (int)hipGetLastError();
}

}  // namespace

namespace {
size_t band_Sp_doubles(const PhaseDims& d) {
  PhaseBand b;
  band_geometry(d, &b);
  return (size_t)d.Nd * b.CH * BM * BM * 2;
}
// image-pass column blocks, at most: 256 / G columns per block with G <= 2 nf1 / 4
size_t band_nxb_max(const PhaseDims& d) {
  const size_t cols = (size_t)std::max(1, 256 / std::max(1, 2 * d.nf1 / 4));
  return (2 * (size_t)d.nf2 + cols - 1) / cols;
}
// image-pass workgroups: at most 2 nf2 column blocks per image
size_t gpart_doubles(const PhaseDims& d) { return std::max((size_t)mid_groups(d), (size_t)d.Nd * 2 * d.nf2); }
// one partial per wave of the gather kernels (64 pixels each, four waves per 256-pixel workgroup)
size_t dpart_doubles(const PhaseDims& d) { return 4 * (((size_t)d.P + 255) / 256); }
}  // namespace

size_t phase_work_bytes(const PhaseDims& d) {
  size_t G = (size_t)d.nf1 * d.nf2;
  size_t dbl = (size_t)d.Nd * d.P * 2 + G * 2 + (size_t)d.Nd * G * 2 + (size_t)d.Nd * 2 * G * 2 +
               gpart_doubles(d) + (size_t)GATHER_SLICES * d.P * 2 + 8 + G + 2 + band_Sp_doubles(d) +
               (size_t)d.Nd * band_nxb_max(d) * BM * BM * 2 + (size_t)d.Nd * d.P * 2 + dpart_doubles(d);
  return dbl * sizeof(double) + 14 * 256;
}

PhaseBand phase_band_plan(const PhaseDims& d, const PhaseOptics& o, int enable) {
  PhaseBand b{};
  band_geometry(d, &b);
  // signed frequencies of the bins inside the pupil (with a relative margin,
  // so that a bin the device counts in is never left out of the box)
  int lo1 = d.nf1, hi1 = -d.nf1, lo2 = d.nf2, hi2 = -d.nf2;
  for (int k1 = 0; k1 < d.nf1; ++k1) {
    const int s1 = (k1 < (d.nf1 + 1) / 2) ? k1 : k1 - d.nf1;
    const double u = (double)s1 / ((double)d.nf1 * o.ps);
    for (int k2 = 0; k2 < d.nf2; ++k2) {
      const int s2 = (k2 < (d.nf2 + 1) / 2) ? k2 : k2 - d.nf2;
      const double v = (double)s2 / ((double)d.nf2 * o.ps);
      const double rho2 = (o.lambda * u) * (o.lambda * u) + (o.lambda * v) * (o.lambda * v);
      if (std::sqrt(rho2) <= o.NA * (1.0 + 1e-9)) {
        lo1 = std::min(lo1, s1);
        hi1 = std::max(hi1, s1);
        lo2 = std::min(lo2, s2);
        hi2 = std::max(hi2, s2);
      }
    }
  }
  if (hi1 < lo1) {  // empty pupil: a one-bin box (h is zero there too)
    lo1 = hi1 = lo2 = hi2 = 0;
  }
  b.s1lo = lo1;
  b.B1 = hi1 - lo1 + 1;
  b.s2lo = lo2;
  b.B2 = hi2 - lo2 + 1;
  // (the image pass needs at least two threads per column: nf1 >= the padded box side)
  b.on = enable && b.B1 <= BM && b.B2 <= BM && d.nf1 >= band_bt1(b.B1);
  const int bt1 = band_bt1(b.B1);
  b.G = std::max(1, 2 * d.nf1 / bt1);
  b.CPW = 256 / b.G;
  b.NXB = (2 * d.nf2 + b.CPW - 1) / b.CPW;
  return b;
}

void phase_work_carve(void* base, const PhaseDims& d, PhaseWork* w) {
  size_t G = (size_t)d.nf1 * d.nf2;
  char* p = (char*)base;
  auto take = [&](size_t ndbl) {
    double* r = (double*)p;
    p += ((ndbl * sizeof(double) + 255) / 256) * 256;
    return r;
  };
  w->c = take((size_t)d.Nd * d.P * 2);
  w->h = take(G * 2);
  w->A = take((size_t)d.Nd * G * 2);
  w->B = take((size_t)d.Nd * 2 * G * 2);
  w->gpart = take(gpart_doubles(d));
  w->w = take((size_t)GATHER_SLICES * d.P * 2);
  w->gval = take(8);
  w->inv = (int32_t*)take(G);
  w->skip = (int*)take(2);
  w->chk = w->skip + 1;
  w->Sp = take(band_Sp_doubles(d));
  w->V = take((size_t)d.Nd * band_nxb_max(d) * BM * BM * 2);
  w->Wn = take((size_t)d.Nd * d.P * 2);
  w->dpart = take(dpart_doubles(d));
  w->band = PhaseBand{};
}

int phase_setup(const PhaseDims& d, const PhaseOptics& o, const void* tm_est, const void* theta,
                const int32_t* pix, PhaseWork& w, void* stream) {
  (void)tm_est;
  (void)theta;
  hipStream_t s = (hipStream_t)stream;
  int G = d.nf1 * d.nf2;
  k_make_h<<<(G + 255) / 256, 256, 0, s>>>(w.h, d.nf1, d.nf2, o.lambda, o.ps, o.NA, o.z);
  k_set_int<<<1, 1, 0, s>>>(w.skip, 0);
  k_invmap<<<(G + 255) / 256, 256, 0, s>>>(w.inv, pix, d.P, G, w.chk);
  k_invmap2<<<(d.P + 255) / 256, 256, 0, s>>>(w.inv, pix, d.P, G, w.chk, w.skip);
  k_invmap3<<<(d.P + 255) / 256, 256, 0, s>>>(w.inv, pix, d.P, G, w.chk, w.skip);
  return (int)hipGetLastError();
}

int phase_eval(const PhaseDims& d, const int32_t* pix, const float* Id, const double* phi, double* grad,
               PhaseWork& w, const double* tw64, void* stream, const double* dvec) {
  hipStream_t s = (hipStream_t)stream;
  int e;
  const int G = d.nf1 * d.nf2;
  const int per = (d.Nd + GATHER_SLICES - 1) / GATHER_SLICES;
  const int nsl = (d.Nd + per - 1) / per;
  if (w.band.on) {
    const PhaseBand& b = w.band;
    k_band_spec<<<dim3(b.CH, d.Nd), 256, 0, s>>>(w.Sp, w.c, phi, w.inv, b, d.P, d.nf1, d.nf2, tw64, w.skip);
    const dim3 gi(b.NXB, d.Nd);
    switch (band_bt1(b.B1)) {
      case 4: k_band_img<4><<<gi, 256, 0, s>>>(w.V, w.gpart, w.Sp, Id, w.h, b, d.nf1, d.nf2, tw64, w.skip); break;
      case 8: k_band_img<8><<<gi, 256, 0, s>>>(w.V, w.gpart, w.Sp, Id, w.h, b, d.nf1, d.nf2, tw64, w.skip); break;
      default: k_band_img<16><<<gi, 256, 0, s>>>(w.V, w.gpart, w.Sp, Id, w.h, b, d.nf1, d.nf2, tw64, w.skip);
    }
    k_band_pix<<<dim3((d.P + 256 * PIX_BLOCKS - 1) / (256 * PIX_BLOCKS), d.Nd), 256,
                 (size_t)b.B1 * d.nf2 * sizeof(z2), s>>>(w.Wn, w.V, w.c, w.h, pix, b, d.P, d.nf1, d.nf2, tw64,
                                                             w.skip);
    k_band_gather<<<(d.P + 63) / 64, 256, 0, s>>>(grad, w.gval, w.Wn, phi, w.gpart, d.Nd * b.NXB, d.Nd, d.P,
                                                  w.skip, dvec, w.dpart);
    return (int)hipGetLastError();
  }
  if ((e = forward_to_rows(d, phi, w, tw64, s))) return e;
  const int ngp = mid_groups(d);
  k_rows_mid<<<ngp, LWG, 0, s>>>(w.B, Id, w.gpart, nullptr, d.Nd, d.nf1, d.nf2, tw64, w.skip);
  k_cols_adj<<<grid_of(d.Nd * d.nf2, 2 * d.nf1), LWG, 0, s>>>(w.A, w.B, w.h, d.Nd, d.nf1, d.nf2, tw64, w.skip);
  k_rows_adj<<<grid_of(d.Nd * d.nf1, d.nf2), LWG, 0, s>>>(w.A, d.Nd, d.nf1, d.nf2, tw64, w.skip);
  if ((e = (int)hipGetLastError())) return e;
  k_gather_part<<<dim3((d.P + 255) / 256, nsl), 256, 0, s>>>(w.w, w.A, w.c, pix, d.Nd, d.P, G, per, w.skip);
  k_gather<<<(d.P + 255) / 256, 256, 0, s>>>(grad, w.gval, w.w, phi, w.gpart, ngp, nsl, d.P, w.skip, dvec,
                                             w.dpart);
  return (int)hipGetLastError();
}

int phase_images(const PhaseDims& d, const int32_t* pix, const double* phi, float* I_out, PhaseWork& w,
                 const double* tw64, void* stream) {
  (void)pix;
  hipStream_t s = (hipStream_t)stream;
  int e;
  if ((e = forward_to_rows(d, phi, w, tw64, s))) return e;
  k_rows_mid<<<mid_groups(d), LWG, 0, s>>>(w.B, nullptr, nullptr, I_out, d.Nd, d.nf1, d.nf2, tw64, w.skip);
  return (int)hipGetLastError();
}

// ------------------------------------------------------------ L-BFGS over phi
namespace {
constexpr int PWG = 512;
constexpr int UE = 4;  // vector elements per thread per pass step (their loads are issued together)

// Block-wide sums of several values: each wave adds its lanes' x into
// red[wave][j] (wave_put), then bsum_finish adds the waves: out[0..nv) for
// every thread. red holds (PWG / 64) * MAXV doubles.
constexpr int MAXV = 4 * 16 + 5;
__device__ __forceinline__ void wave_put(double x, int j, double* red) {
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * MAXV + j] = x;
}
__device__ void bsum_finish(int nv, double* red, double* out) {
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += PWG) {
    double s = 0;
    for (int i = 0; i < PWG / 64; ++i) s += red[i * MAXV + j];
    out[j] = s;
  }
  __syncthreads();
}

// Line search and iteration control on the device, so that iterations replay
// back-to-back without host synchronisation. State sc (doubles):
// [0] head, [1] count, [2] slope of d, [3] step a of the pending trial,
// [4] objective f at phi, [5] accepted iterations, [6] objective evaluations
// (the start point and every trial point set so far),
// [7] halvings of this direction, [8] a trial is pending, [9] converged (the
// last accepted trial lowered f by at most ftol f), [10] a best trial is kept,
// [11] its step, [12] its objective, [13] doublings of this direction; then
// the m x m matrices SY[i][j] = s_i^T y_j and YY[i][j] = y_i^T y_j over the
// history slots.
// *skip = 1 ends the solve (every later kernel returns at once).
// One iteration is k_piter followed by the objective and gradient at phit
// (with the partials of d^T g there): k_piter first decides on the pending
// trial and sets the next trial point phit = phi + a d. Line search: a trial
// that satisfies Armijo (f_t <= f + 1e-4 a slope) and is below the kept one
// is kept; while no halving has happened and the slope there is still below
// 0.9 slope (the curvature condition fails), the step doubles (at most 20
// times); otherwise, or when a trial fails after one was kept, the kept trial
// is accepted: the pair is stored and a new direction taken with a = 1. While
// nothing is kept, a failing trial halves the step (at most 40 times).
// The direction is the L-BFGS product -H g in the compact form of Byrd,
// Nocedal and Schnabel (1994): with a = S^T g, b = Y^T g over the k stored
// pairs (oldest first), R the upper triangle of S^T Y, D its diagonal and
// gamma = s^T y / y^T y of the newest pair, H g = gamma g + S p - gamma Y u
// where R u = a and R^T p = (D + gamma Y^T Y) u - gamma b. This equals the
// two-loop recursion; all its dot products, and those of the new pair with
// the stored ones, come from one pass over the vectors, and the direction
// and the trial point from a second.
constexpr int SC_HIST = 14;
constexpr double LS_C1 = 1e-4, LS_C2 = 0.9;
constexpr int LS_HALVINGS = 40, LS_DOUBLINGS = 20;

// smat (LDS, SMAT doubles): the k x k blocks of SY and YY in age order, then
// the small solve's u and p.
constexpr int SMAT = 2 * 16 * 16 + 2 * 16;

// Thread 0: coefficients of d = coef[0] g + sum_j coef[1+j] S_j + coef[1+k+j] Y_j
// over the k stored pairs (age order, slot of pair j: (head - k + j) mod m)
// from a_j = s_j^T g (dots[j]), b_j = y_j^T g (dots[k+j]) and g^T g (dots[2k]).
// Sets sc[1] = 0 (history dropped) when the product is not a descent
// direction, and sc[2] = the slope g^T d. coef[1 + 2k] = 1 if the pairs are used.
__device__ void dir_solve(int k, int head, int m, int P, double* sc, const double* dots, double* coef,
                          double* smat) {
  double* R = smat;        // R[i][j] = s_i^T y_j (age order), row stride 16
  double* W = smat + 256;  // W[i][j] = y_i^T y_j
  double* u = smat + 512;
  double* p = smat + 528;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      const int si = (head - k + i + 2 * m) % m, sj = (head - k + j + 2 * m) % m;
      R[i * 16 + j] = sc[SC_HIST + si * m + sj];
      W[i * 16 + j] = sc[SC_HIST + m * m + si * m + sj];
    }
  const double gg = dots[2 * k];
  double cg = 0.0, slope = 0.0;
  bool keep = k > 0;
  if (k > 0) {
    const double gam = R[(k - 1) * 17] / W[(k - 1) * 17];
    for (int i = k - 1; i >= 0; --i) {  // R u = a (upper triangle)
      double t = dots[i];
      for (int j = i + 1; j < k; ++j) t -= R[i * 16 + j] * u[j];
      u[i] = t / R[i * 17];
    }
    for (int i = 0; i < k; ++i) {  // R^T p = (D + gam Y^T Y) u - gam b
      double t = R[i * 17] * u[i] - gam * dots[k + i];
      for (int j = 0; j < k; ++j) t += gam * W[i * 16 + j] * u[j];
      for (int j = 0; j < i; ++j) t -= R[j * 16 + i] * p[j];
      p[i] = t / R[i * 17];
    }
    // d = -H g = -gam g - S p + gam Y u
    cg = -gam;
    slope = -gam * gg;
    for (int j = 0; j < k; ++j) {
      coef[1 + j] = -p[j];
      coef[1 + k + j] = gam * u[j];
      slope += -p[j] * dots[j] + gam * u[j] * dots[k + j];
    }
    if (!(slope < 0.0)) keep = false;  // not a descent direction: drop the history
  }
  if (!keep) {  // -sqrt(P) g / ||g||: a step of 1 moves the offsets by 1 rad RMS
    cg = gg > 0 ? -sqrt((double)P) / sqrt(gg) : 0.0;
    slope = cg * gg;
    sc[1] = 0;
  }
  coef[0] = cg;
  coef[1 + 2 * k] = keep ? 1.0 : 0.0;
  sc[2] = slope;
}

// d from the coefficients, and the trial point phit = phi + d (step 1)
// (two elements per thread and up to six pairs per pass, so that the loads of a
// pass are in flight together)
constexpr int DA_PAIRS = 6;
__device__ void dir_apply(PhaseLb& L, int P, int m, int k, int head, const double* coef) {
  const int kk = coef[1 + 2 * k] != 0.0 ? k : 0;
  for (int i0 = threadIdx.x; i0 < P; i0 += UE * PWG) {
    double d[UE], f[UE];
#pragma unroll
    for (int e = 0; e < UE; ++e) {
      const int i = i0 + e * PWG;
      d[e] = i < P ? coef[0] * L.g[i] : 0.0;
      f[e] = i < P ? L.phi[i] : 0.0;
    }
    for (int c0 = 0; c0 < kk; c0 += DA_PAIRS) {
      double sv[UE][DA_PAIRS], yv[UE][DA_PAIRS];
#pragma unroll
      for (int q = 0; q < DA_PAIRS; ++q) {
        const size_t o = (size_t)((head - k + c0 + q + 2 * m) % m) * P;
#pragma unroll
        for (int e = 0; e < UE; ++e) {
          const int i = i0 + e * PWG;
          const bool ok = c0 + q < kk && i < P;
          sv[e][q] = ok ? L.S[o + i] : 0.0;
          yv[e][q] = ok ? L.Y[o + i] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < DA_PAIRS; ++q) {
        if (c0 + q < kk) {
          const double cs = coef[1 + c0 + q], cy = coef[1 + k + c0 + q];
#pragma unroll
          for (int e = 0; e < UE; ++e) d[e] += cs * sv[e][q] + cy * yv[e][q];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < UE; ++e) {
      const int i = i0 + e * PWG;
      if (i < P) {
        L.d[i] = d[e];
        L.phit[i] = f[e] + d[e];
      }
    }
  }
}

// First direction (no trial yet): the L-BFGS product over the stored pairs,
// which after the start are none, so -sqrt(P) g / ||g||; then the trial point.
__device__ void first_direction(PhaseLb& L, int P, int m, double* red, double* sc, double* sh, double* smat) {
  const int head = (int)sc[0], k = (int)sc[1];
  for (int j = 0; j < k; ++j) {
    const int sl = (head - k + j + 2 * m) % m;
    double xa = 0.0, xb = 0.0;
    for (int i = threadIdx.x; i < P; i += PWG) {
      const double gi = L.g[i];
      xa += L.S[(size_t)sl * P + i] * gi;
      xb += L.Y[(size_t)sl * P + i] * gi;
    }
    wave_put(xa, j, red);
    wave_put(xb, k + j, red);
  }
  double xg = 0.0;
  for (int i = threadIdx.x; i < P; i += PWG) xg += L.g[i] * L.g[i];
  wave_put(xg, 2 * k, red);
  double* dots = sh;
  double* coef = sh + MAXV;
  bsum_finish(2 * k + 1, red, dots);
  if (threadIdx.x == 0) dir_solve(k, head, m, P, sc, dots, coef, smat);
  __syncthreads();
  dir_apply(L, P, m, k, head, coef);
}

// Accepted trial at step a with objective fn and gradient gsrc (the pending
// trial's or the kept one's): the pair s = a d, y = g_t - g goes into slot
// head (its dot products with the stored pairs update SY and YY), phi and g
// move to the trial, and the dot products of the next direction (with g_t)
// are taken in the same pass. Returns 1 (to every thread) when the solve ends here.
__device__ int accept(PhaseLb& L, int P, int m, int iters, double ftol, const double* gsrc, double a, double fn,
                      double* red, double* sc, double* sh, double* smat) {
  const int head = (int)sc[0], count = (int)sc[1];
  const int keep = count < m ? count : m - 1;  // stored pairs that stay (the oldest is overwritten when full)
  double* Sh = L.S + (size_t)head * P;
  double* Yh = L.Y + (size_t)head * P;
  // per stored pair j: s_j^T y, y_j^T y, s_j^T g_t, y_j^T g_t (sums 4j..4j+3); then s^T y, y^T y,
  // s^T g_t, y^T g_t, g_t^T g_t (sums 4 keep..4 keep + 4). The stored pairs go four per pass (one pass
  // for m <= 5); the last pass also writes the new pair, phi and g.
  for (int c0 = 0; c0 < (keep > 0 ? keep : 1); c0 += 4) {
    const bool last = c0 + 4 >= keep;
    double x[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q][0] = x[q][1] = x[q][2] = x[q][3] = 0.0;
    double xsy = 0.0, xyy = 0.0, xsg = 0.0, xyg = 0.0, xgg = 0.0;
    for (int i0 = threadIdx.x; i0 < P; i0 += UE * PWG) {
      // UE elements per thread, all their loads issued before the arithmetic
      double gt[UE], dd[UE], gg[UE], ph[UE], Sv[UE][4], Yv[UE][4];
#pragma unroll
      for (int e = 0; e < UE; ++e) {
        const int i = i0 + e * PWG;
        const bool ok = i < P;
        gt[e] = ok ? gsrc[i] : 0.0;
        dd[e] = ok ? L.d[i] : 0.0;
        gg[e] = ok ? L.g[i] : 0.0;
        ph[e] = (ok && last) ? L.phi[i] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          Sv[e][q] = Yv[e][q] = 0.0;
          if (ok && c0 + q < keep) {
            const size_t o = (size_t)((head - keep + c0 + q + 2 * m) % m) * P + i;
            Sv[e][q] = L.S[o];
            Yv[e][q] = L.Y[o];
          }
        }
      }
#pragma unroll
      for (int e = 0; e < UE; ++e) {
        const int i = i0 + e * PWG;
        const double gti = gt[e], si = a * dd[e], yi = gti - gg[e];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          x[q][0] += Sv[e][q] * yi;
          x[q][1] += Yv[e][q] * yi;
          x[q][2] += Sv[e][q] * gti;
          x[q][3] += Yv[e][q] * gti;
        }
        if (last) {
          xsy += si * yi;
          xyy += yi * yi;
          xsg += si * gti;
          xyg += yi * gti;
          xgg += gti * gti;
          if (i < P) {
            Sh[i] = si;
            Yh[i] = yi;
            L.phi[i] = ph[e] + si;
            L.g[i] = gti;
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (c0 + q < keep)
        for (int r = 0; r < 4; ++r) wave_put(x[q][r], 4 * (c0 + q) + r, red);
    if (last) {
      wave_put(xsy, 4 * keep, red);
      wave_put(xyy, 4 * keep + 1, red);
      wave_put(xsg, 4 * keep + 2, red);
      wave_put(xyg, 4 * keep + 3, red);
      wave_put(xgg, 4 * keep + 4, red);
    }
  }
  double* sums = smat + SMAT;  // 4 keep + 5 values
  double* dots = sh;
  double* coef = sh + MAXV;
  __shared__ int fin, kdir, hdir;
  bsum_finish(4 * keep + 5, red, sums);
  if (threadIdx.x == 0) {
    double* SY = sc + SC_HIST;
    double* YY = sc + SC_HIST + m * m;
    const double f = sc[4];
    const double sy = sums[4 * keep], yy = sums[4 * keep + 1];
    int k = keep, nh = head;
    if (sy > 0.0) {
      for (int j = 0; j < keep; ++j) {
        const int sl = (head - keep + j + 2 * m) % m;
        SY[sl * m + head] = sums[4 * j];
        YY[sl * m + head] = sums[4 * j + 1];
        YY[head * m + sl] = sums[4 * j + 1];
      }
      SY[head * m + head] = sy;
      YY[head * m + head] = yy;
      nh = (head + 1) % m;
      k = keep + 1;
    }
    sc[0] = nh;
    sc[1] = k;  // without the new pair, slot head no longer holds a stored pair
    sc[9] = (f - fn <= ftol * fabs(fn)) ? 1.0 : 0.0;
    sc[4] = fn;
    sc[5] += 1.0;
    sc[10] = 0.0;
    sc[13] = 0.0;
    fin = (sc[5] >= (double)iters || (ftol > 0.0 && sc[9] != 0.0)) ? 1 : 0;
    if (!fin) {
      // a_j, b_j of the pairs in age order: the stored ones, then the new one
      for (int j = 0; j < keep; ++j) {
        dots[j] = sums[4 * j + 2];
        dots[k + j] = sums[4 * j + 3];
      }
      if (k > keep) {
        dots[keep] = sums[4 * keep + 2];
        dots[k + keep] = sums[4 * keep + 3];
      }
      dots[2 * k] = sums[4 * keep + 4];
      dir_solve(k, nh, m, P, sc, dots, coef, smat);
      kdir = k;
      hdir = nh;
      sc[3] = 1.0;
      sc[7] = 0.0;
      if (!(sc[2] < 0.0)) fin = 1;  // zero gradient
    }
  }
  __syncthreads();
  if (fin) return 1;
  dir_apply(L, P, m, kdir, hdir, coef);
  return 0;
}

// phit = phi + as d
__device__ void trial_point(PhaseLb& L, int P, double as, bool keep_gt) {
  for (int i0 = threadIdx.x; i0 < P; i0 += UE * PWG) {
    double f[UE], e[UE], gk[UE];
#pragma unroll
    for (int u = 0; u < UE; ++u) {
      const int i = i0 + u * PWG;
      f[u] = i < P ? L.phi[i] : 0.0;
      e[u] = i < P ? L.d[i] : 0.0;
      gk[u] = (keep_gt && i < P) ? L.gt[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UE; ++u) {
      const int i = i0 + u * PWG;
      if (i < P) {
        L.phit[i] = f[u] + as * e[u];
        if (keep_gt) L.gb[i] = gk[u];
      }
    }
  }
}

// A trial point is set: the evaluation that follows is pending.
__device__ __forceinline__ void new_trial(double* sc) {
  sc[8] = 1.0;
  sc[6] += 1.0;
}

// The solve ends: flag it for every later kernel.
__device__ void end_solve(int* skip, double* sc) {
  if (threadIdx.x == 0) {
    *skip = 1;
    sc[8] = 0.0;
  }
}

// One iteration on the state sc (an LDS copy; every branch below is taken by
// the whole workgroup).
__device__ void piter_body(PhaseLb& L, int P, int m, int iters, double ftol, const double* gval, int* skip,
                           double* sc, double* red, double* sh, double* smat) {
  __shared__ int stop;
  if (threadIdx.x == 0) stop = 0;
  __syncthreads();
  if (sc[8] != 0.0) {
    const double fn = gval[0], f = sc[4], a = sc[3], slope = sc[2];
    const bool kept = sc[10] != 0.0;
    if (fn <= f + LS_C1 * a * slope && (!kept || fn < sc[12])) {
      bool take = sc[7] > 0.0 || sc[13] >= (double)LS_DOUBLINGS;
      if (!take) {  // curvature condition: the slope d^T g_t from the evaluation's partials
        double x = 0.0;
        for (int i = threadIdx.x; i < (P + 63) / 64; i += PWG) x += L.dpart[i];
        wave_put(x, 0, red);
        bsum_finish(1, red, sh);
        take = sh[0] >= LS_C2 * slope;
        __syncthreads();  // sh is reused below
      }
      if (take) {
        if (accept(L, P, m, iters, ftol, L.gt, a, fn, red, sc, sh, smat)) end_solve(skip, sc);
        else if (threadIdx.x == 0) new_trial(sc);
        return;
      }
      // keep this trial and double the step
      if (threadIdx.x == 0) {
        sc[10] = 1.0;
        sc[11] = a;
        sc[12] = fn;
        sc[13] += 1.0;
        sc[3] = 2.0 * a;
        new_trial(sc);
      }
      trial_point(L, P, 2.0 * a, true);
      return;
    }
    if (kept) {  // the doubled step is no better: take the kept trial
      if (accept(L, P, m, iters, ftol, L.gb, sc[11], sc[12], red, sc, sh, smat)) end_solve(skip, sc);
      else if (threadIdx.x == 0) new_trial(sc);
      return;
    }
    // rejected, nothing kept: halve the step along d
    __syncthreads();
    if (threadIdx.x == 0) {
      sc[7] += 1.0;
      if (sc[7] >= (double)LS_HALVINGS) {
        stop = 1;  // no sufficient decrease along d: stop
      } else {
        sc[3] *= 0.5;
        new_trial(sc);
      }
    }
    __syncthreads();
    if (stop) {
      end_solve(skip, sc);
      return;
    }
    trial_point(L, P, sc[3], false);
    return;
  }
  // no pending trial: the first direction after the start
  if (sc[5] >= (double)iters) {
    if (threadIdx.x == 0) *skip = 1;
    return;
  }
  first_direction(L, P, m, red, sc, sh, smat);
  if (threadIdx.x == 0) {
    sc[3] = 1.0;
    sc[7] = 0.0;
    sc[10] = 0.0;
    sc[13] = 0.0;
    if (!(sc[2] < 0.0)) stop = 1;  // zero gradient
  }
  __syncthreads();
  if (stop) {
    if (threadIdx.x == 0) *skip = 1;
    return;
  }
  if (threadIdx.x == 0) new_trial(sc);
}

__global__ void __launch_bounds__(PWG) k_piter(PhaseLb L, int P, int m, int iters, double ftol, const double* gval,
                                                int* skip) {
  __shared__ double red[(PWG / 64) * MAXV];
  __shared__ double sh[2 * MAXV];
  __shared__ double smat[SMAT + MAXV];
  __shared__ double scl[SC_HIST + 2 * 16 * 16];
  if (*skip) return;
  // the iteration state lives in LDS for the kernel (one parallel load, one store back)
  const int nsc = SC_HIST + 2 * m * m;
  for (int i = threadIdx.x; i < nsc; i += PWG) scl[i] = L.sc[i];
  __syncthreads();  // also: every thread has read *skip before thread 0 may set it
  piter_body(L, P, m, iters, ftol, gval, skip, scl, red, sh, smat);
  __syncthreads();
  for (int i = threadIdx.x; i < nsc; i += PWG) L.sc[i] = scl[i];
}

// start: clear the state, take f at the start point, allow the first direction
// (unless the pixel check failed, or no iteration is asked for: the solve has
// then ended at the start point)
__global__ void k_pinit(double* sc, int n, const double* gval, int* skip, const int* chk, int iters) {
  for (int i = threadIdx.x; i < n; i += 64) sc[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    sc[4] = gval[0];
    sc[6] = 1.0;  // the start point
    *skip = (chk[0] != 0 || iters <= 0) ? 1 : 0;
  }
}

// End of a batch of iterations: the current phi to the caller's buffer (unless
// the pixel check failed) and one record for the host: f, accepted
// iterations, evaluations, the solve-ended flag and the pixel check.
__global__ void __launch_bounds__(256) k_pfinish(const double* sc, const int* skip, const int* chk,
                                                 const double* phi_src, double* phi_dst, int P, double* rec) {
  const bool ok = chk[0] == 0;
  const int stride = gridDim.x * 256;
  for (int i = blockIdx.x * 256 + threadIdx.x; ok && i < P; i += stride) phi_dst[i] = phi_src[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rec[0] = sc[4];
    rec[1] = sc[5];
    rec[2] = sc[6];
    rec[3] = (double)*skip;
    rec[4] = (double)chk[0];
    rec[5] = (double)chk[1];
    rec[6] = (double)chk[2];
  }
}
}  // namespace

int phase_lb_state_doubles(int m) { return SC_HIST + 2 * m * m; }

int phase_lb_finish(const PhaseLb& L, const PhaseWork& w, int P, double* phi_out, double* rec, void* stream) {
  const int blocks = std::max(1, std::min(64, (P + 255) / 256));
  k_pfinish<<<blocks, 256, 0, (hipStream_t)stream>>>(L.sc, w.skip, w.chk, L.phi, phi_out, P, rec);
  return (int)hipGetLastError();
}

int phase_lb_init(PhaseLb& L, int P, int m, int iters, const double* gval, int* skip, const int* chk,
                  void* stream) {
  k_pinit<<<1, 64, 0, (hipStream_t)stream>>>(L.sc, phase_lb_state_doubles(m), gval, skip, chk, iters);
  return (int)hipGetLastError();
}
int phase_lb_iter(PhaseLb& L, int P, int m, int iters, double ftol, const double* gval, int* skip, void* stream) {
  k_piter<<<1, PWG, 0, (hipStream_t)stream>>>(L, P, m, iters, ftol, gval, skip);
  return (int)hipGetLastError();
}

}  // namespace tmk

namespace tmk {
// K slices: about one round of workgroups at three per CU of a 256-CU device
// (a second, partial round left most SIMDs with one wave), each slice a whole
// number of K steps; *kchunk receives the slice length.
static int cgemm_split(const PhaseDims& d, int* kchunk) {
  const int tiles = ((d.P + CG_P - 1) / CG_P) * ((d.Nd + CG_N - 1) / CG_N);
  const int steps = (d.N + CG_K - 1) / CG_K;
  const int want = std::max(1, std::min(steps, 768 / tiles));
  const int per = (steps + want - 1) / want;
  if (kchunk) *kchunk = per * CG_K;
  return (steps + per - 1) / per;
}

int phase_cgemm_slices(const PhaseDims& d) { return cgemm_split(d, nullptr); }

int phase_cgemm(const PhaseDims& d, const void* theta, const void* tm, double* part, double* c, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int kchunk = 0;
  const int gs = cgemm_split(d, &kchunk);
  dim3 g((d.P + CG_P - 1) / CG_P, (d.Nd + CG_N - 1) / CG_N, gs);
  const float2* th = (const float2*)theta;
  const float2* tmv = (const float2*)tm;
  // 16-byte pair loads need even rows; the operands are hipMalloc'd (16-byte aligned)
  const int ncb = std::min(8, (2 * std::min(d.Nd, CG_N) + 15) / 16);  // column blocks holding images
  if (d.N % 2 == 0 && (uintptr_t)th % 16 == 0 && (uintptr_t)tmv % 16 == 0)
    cgemm_launch<true>(ncb, g, s, th, tmv, part, d, kchunk);
  else
    cgemm_launch<false>(ncb, g, s, th, tmv, part, d, kchunk);
  const int64_t n = (int64_t)d.Nd * d.P * 2;
  k_cgemm_sum<<<(int)((n + 255) / 256), 256, 0, s>>>(part, c, n, gs);
  return (int)hipGetLastError();
}
}  // namespace tmk
