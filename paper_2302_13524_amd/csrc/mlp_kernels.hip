// Learned start network on MFMA: BF16 operands, FP32 accumulation.
//
// Network (not part of the paper, whose start is back-propagation): features
// x = I_p / mean(I_p) (K N values) -> Linear -> GELU -> Linear -> GELU ->
// Linear -> 2N reals read as the complex start u = o[:N] + j o[N:]. Loss per
// row ||u||^2 + ||u*||^2 - 2|u*^H u| with u* = t / s, s = sqrt(sum(I)/(K N)),
// invariant to the row's phase (Sec. 2.3, Eq. phaseoffset); packed gradient
// 2 (u - e^{j arg(u*^H u)} u*). Adam on FP32 master weights.
//
// GEMM: C[M x N] = op(A) op(B), 128 x 128 tiles, K steps of 32 staged in LDS,
// four waves each computing 64 x 64 with v_mfma_f32_32x32x16_bf16.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mlp.hpp"

namespace tmk {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  float cdf = 0.5f * (1.f + erff(x * 0.70710678118654752f));
  float pdf = 0.39894228040143268f * __expf(-0.5f * x * x);
  return cdf + x * pdf;
}

constexpr int BM = 128, BN = 128, BK = 32, LDK = BK + 8;  // LDS row stride in bf16 (80 B)

// A K step's tile of one operand, 128 rows x 32 k, staged in registers: each
// thread holds 16 bf16 (two 16-byte words). Element (r, k) of the operand is
// at p[k * ld + r] when `trans`, else at p[r * ld + k]; out-of-range elements
// are 0. `vec`: ld is a multiple of 8 and p 16-byte aligned, so a thread's 16
// consecutive elements load as two 16-byte words wherever they are in range.
struct TileRegs {
  uint4 v[2];
};

__device__ __forceinline__ void tile_fetch(TileRegs& t, const uint16_t* __restrict__ p, int ld, bool trans, bool vec,
                                           int r0, int k0, int R, int Kd) {
  const int tid = threadIdx.x;
  // not trans: row r0 + tid / 2, k0 + 16 (tid % 2) .. + 15; trans: k0 + tid / 8, rows r0 + 16 (tid % 8) .. + 15
  const int a = trans ? k0 + (tid >> 3) : r0 + (tid >> 1);     // fixed index
  const int b = trans ? r0 + (tid & 7) * 16 : k0 + (tid & 1) * 16;  // first of the 16 consecutive
  const int alim = trans ? Kd : R, blim = trans ? R : Kd;
  const uint16_t* q = p + (size_t)a * ld + b;
  if (vec && a < alim && b + 16 <= blim) {
    t.v[0] = ((const uint4*)q)[0];
    t.v[1] = ((const uint4*)q)[1];
  } else {
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint32_t lo = (a < alim && b + 2 * i < blim) ? q[2 * i] : 0u;
      const uint32_t hi = (a < alim && b + 2 * i + 1 < blim) ? q[2 * i + 1] : 0u;
      w[i] = lo | (hi << 16);
    }
    t.v[0] = make_uint4(w[0], w[1], w[2], w[3]);
    t.v[1] = make_uint4(w[4], w[5], w[6], w[7]);
  }
}

// The staged tile into LDS as [row][k] (k contiguous, row stride LDK)
__device__ __forceinline__ void tile_store(uint16_t* lds, const TileRegs& t, bool trans) {
  const int tid = threadIdx.x;
  if (!trans) {
    uint4* d = (uint4*)&lds[(tid >> 1) * LDK + (tid & 1) * 16];  // LDK * 2 B = 80 B: 16-byte aligned
    d[0] = t.v[0];
    d[1] = t.v[1];
  } else {
    const int k = tid >> 3, rh = (tid & 7) * 16;
    const uint32_t w[8] = {t.v[0].x, t.v[0].y, t.v[0].z, t.v[0].w, t.v[1].x, t.v[1].y, t.v[1].z, t.v[1].w};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      lds[(rh + 2 * i) * LDK + k] = (uint16_t)(w[i] & 0xffffu);
      lds[(rh + 2 * i + 1) * LDK + k] = (uint16_t)(w[i] >> 16);
    }
  }
}

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;  // bf16
  int lda;
  int ta;             // A stored [K][M] if set, else [M][K]
  const uint16_t* B;  // bf16
  int ldb;
  int tb;             // B stored [N][K] if set, else [K][N]
  int epi;            // MlpEpi
  const float* bias;  // [N]
  const float* aux;   // [M][N] pre-activation for the GELU derivative
  float* outf;        // [M][N] FP32 output (may be null)
  uint16_t* outh;     // [M][N] BF16 output (may be null)
  float* outf2;       // [M][N] second FP32 output (pre-activation)
  float beta;         // outf = beta * outf + result (accumulate across calls), 0 or 1
  int veca, vecb;     // 16-byte tile loads allowed (leading dimension a multiple of 8, aligned base)
};

// Epilogue of one wave's 64 x 64 block: lane holds column n = lane % 32 of
// each 32 x 32 tile, rows 8 q + 4 (lane / 32) + r for acc element 4 q + r.
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& g, const f32x16 (&acc)[2][2], int mb, int nb, int lane) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int q = e >> 2, r = e & 3;
        const int m = mb + i * 32 + 8 * q + 4 * (lane >> 5) + r;
        const int n = nb + j * 32 + (lane & 31);
        const float a = acc[i][j][e];
        if (m < g.M && n < g.N) {
          const size_t o = (size_t)m * g.N + n;
          float v = a;
          if constexpr (EPI == MLP_EPI_BIAS_GELU) {
            v += g.bias[n];
            if (g.outf2) g.outf2[o] = v;
            const float h = gelu(v);
            if (g.outh) g.outh[o] = f2bf(h);
            if (g.outf) g.outf[o] = h;
          } else if constexpr (EPI == MLP_EPI_BIAS) {
            v += g.bias[n];
            if (g.outf) g.outf[o] = v;
            if (g.outh) g.outh[o] = f2bf(v);
          } else if constexpr (EPI == MLP_EPI_GELU_BWD) {
            v *= gelu_grad(g.aux[o]);
            if (g.outf) g.outf[o] = v;
            if (g.outh) g.outh[o] = f2bf(v);
          } else {
            if (g.outf) g.outf[o] = (g.beta != 0.f ? g.outf[o] : 0.f) + v;
            if (g.outh) g.outh[o] = f2bf(v);
          }
        }
      }
}

// K steps double-buffered: the next step's tiles are loaded into registers
// while the MFMAs run on the current one; one barrier per K step.
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  __shared__ uint16_t sA[2][BM * LDK];
  __shared__ uint16_t sB[2][BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const bool ta = g.ta != 0, tb = g.tb == 0;  // B as [n][k]: "trans" when stored [K][N]
  TileRegs ra, rb;
  tile_fetch(ra, g.A, g.lda, ta, g.veca != 0, m0, 0, g.M, g.K);
  tile_fetch(rb, g.B, g.ldb, tb, g.vecb != 0, n0, 0, g.N, g.K);
  const int nk = (g.K + BK - 1) / BK;
  for (int ks = 0; ks < nk; ++ks) {
    uint16_t* sa = sA[ks & 1];
    uint16_t* sb = sB[ks & 1];
    // this buffer's last readers (step ks - 2) passed the barrier of step ks - 1
    tile_store(sa, ra, ta);
    tile_store(sb, rb, tb);
    __syncthreads();
    if (ks + 1 < nk) {
      tile_fetch(ra, g.A, g.lda, ta, g.veca != 0, m0, (ks + 1) * BK, g.M, g.K);
      tile_fetch(rb, g.B, g.ldb, tb, g.vecb != 0, n0, (ks + 1) * BK, g.N, g.K);
    }
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf16x8 av[2], bv[2];
      const int kofs = kk + (lane >> 5) * 8;
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = *(const bf16x8*)&sa[(wm + i * 32 + (lane & 31)) * LDK + kofs];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = *(const bf16x8*)&sb[(wn + j * 32 + (lane & 31)) * LDK + kofs];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  switch (g.epi) {  // one unrolled epilogue per kind, so the accumulators stay in registers
    case MLP_EPI_BIAS_GELU: gemm_epilogue<MLP_EPI_BIAS_GELU>(g, acc, m0 + wm, n0 + wn, lane); break;
    case MLP_EPI_BIAS: gemm_epilogue<MLP_EPI_BIAS>(g, acc, m0 + wm, n0 + wn, lane); break;
    case MLP_EPI_GELU_BWD: gemm_epilogue<MLP_EPI_GELU_BWD>(g, acc, m0 + wm, n0 + wn, lane); break;
    default: gemm_epilogue<MLP_EPI_STORE>(g, acc, m0 + wm, n0 + wn, lane); break;
  }
}

// features: X[b][i] = bf16(I[b][i] / mean_b), s[b] = sqrt(sum_b / (K N))
__global__ void __launch_bounds__(256) k_features(const float* __restrict__ I, int len, int B, uint16_t* X,
                                                   float* s, float kn) {
  __shared__ double red[4];
  int b = blockIdx.x;
  if (b >= B) return;
  const float* r = I + (size_t)b * len;
  double acc = 0;
  for (int i = threadIdx.x; i < len; i += 256) acc += r[i];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double tot = red[0] + red[1] + red[2] + red[3];
  float inv = tot > 0 ? (float)(len / tot) : 1.f;
  for (int i = threadIdx.x; i < len; i += 256) X[(size_t)b * len + i] = f2bf(r[i] * inv);
  if (threadIdx.x == 0) s[b] = (float)sqrt(fmax(tot, 0.0) / (double)kn);
}

// per-row phase-invariant loss and its gradient w.r.t. the outputs
__global__ void __launch_bounds__(256) k_loss(const float* __restrict__ O, const float2* __restrict__ t,
                                               const float* __restrict__ s, int B, int N, uint16_t* dOh,
                                               float* dOf, float* loss, float inv_batch) {
  __shared__ double red[3][4];
  int b = blockIdx.x;
  if (b >= B) return;
  const float* o = O + (size_t)b * 2 * N;
  const float2* tr = t + (size_t)b * N;
  float sc = s[b] > 0 ? 1.f / s[b] : 0.f;
  double cr = 0, ci = 0, uu = 0, tt = 0;
  for (int i = threadIdx.x; i < N; i += 256) {
    float ur = o[i], ui = o[N + i];
    float2 tv = tr[i];
    float ar = tv.x * sc, ai = tv.y * sc;
    cr += (double)ar * ur + (double)ai * ui;   // conj(u*) u
    ci += (double)ar * ui - (double)ai * ur;
    uu += (double)ur * ur + (double)ui * ui;
    tt += (double)ar * ar + (double)ai * ai;
  }
  double v[4] = {cr, ci, uu, tt};
  double tot[4];
  for (int q = 0; q < 4; ++q) {
    double x = v[q];
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) ((double*)red)[threadIdx.x >> 6] = x;
    __syncthreads();
    tot[q] = ((double*)red)[0] + ((double*)red)[1] + ((double*)red)[2] + ((double*)red)[3];
  }
  double cabs = sqrt(tot[0] * tot[0] + tot[1] * tot[1]);
  double pr = cabs > 0 ? tot[0] / cabs : 1.0, pi = cabs > 0 ? tot[1] / cabs : 0.0;
  if (threadIdx.x == 0 && loss) loss[b] = (float)(tot[2] + tot[3] - 2.0 * cabs);
  for (int i = threadIdx.x; i < N; i += 256) {
    float ur = o[i], ui = o[N + i];
    float2 tv = tr[i];
    float ar = tv.x * sc, ai = tv.y * sc;
    // 2 (u - e^{j arg c} u*) / B
    float gr = 2.f * (ur - (float)(pr * ar - pi * ai)) * inv_batch;
    float gi = 2.f * (ui - (float)(pr * ai + pi * ar)) * inv_batch;
    size_t q = (size_t)b * 2 * N;
    if (dOh) {
      dOh[q + i] = f2bf(gr);
      dOh[q + N + i] = f2bf(gi);
    }
    if (dOf) {
      dOf[q + i] = gr;
      dOf[q + N + i] = gi;
    }
  }
}

// db[n] = sum_b D[b][n]
__global__ void k_colsum(const float* __restrict__ D, int B, int Nc, float* db) {
  int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= Nc) return;
  float s = 0.f, c = 0.f;
  for (int b = 0; b < B; ++b) {
    float v = D[(size_t)b * Nc + n];
    float t = s + v, bp = t - s;
    c += (s - (t - bp)) + (v - bp);
    s = t;
  }
  db[n] = s + c;
}

__global__ void k_adam(float* w, float* m, float* v, const float* g, uint16_t* wh, size_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t st = (size_t)gridDim.x * 256;
  for (; i < n; i += st) {
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wh) wh[i] = f2bf(wi);
  }
}

// start rows: t0 = u / ||u|| * s
__global__ void __launch_bounds__(256) k_start(const float* __restrict__ O, const float* __restrict__ s, int P, int N,
                                                float2* t0) {
  __shared__ double red[4];
  int p = blockIdx.x;
  if (p >= P) return;
  const float* o = O + (size_t)p * 2 * N;
  double acc = 0;
  for (int i = threadIdx.x; i < N; i += 256) acc += (double)o[i] * o[i] + (double)o[N + i] * o[N + i];
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  double tot = red[0] + red[1] + red[2] + red[3];
  float f = tot > 0 ? (float)(s[p] / sqrt(tot)) : 0.f;
  for (int i = threadIdx.x; i < N; i += 256) t0[(size_t)p * N + i] = make_float2(o[i] * f, o[N + i] * f);
}

__global__ void k_to_bf16(const float* x, uint16_t* y, size_t n) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

int gemm(const GemmArgs& g0, hipStream_t s) {
  GemmArgs g = g0;
  g.veca = g.lda % 8 == 0 && (uintptr_t)g.A % 16 == 0;
  g.vecb = g.ldb % 8 == 0 && (uintptr_t)g.B % 16 == 0;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM);
  k_gemm<<<grid, 256, 0, s>>>(g);
  return (int)hipGetLastError();
}

GemmArgs ga(int M, int N, int K, const uint16_t* A, int lda, int ta, const uint16_t* B, int ldb, int tb, int epi) {
  GemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.ta = ta;
  g.B = B;
  g.ldb = ldb;
  g.tb = tb;
  g.epi = epi;
  g.bias = nullptr;
  g.aux = nullptr;
  g.outf = nullptr;
  g.outh = nullptr;
  g.outf2 = nullptr;
  g.beta = 0.f;
  return g;
}

}  // namespace

size_t mlp_work_bytes(const MlpShape& sh, int B) {
  size_t a = 0;
  auto add = [&](size_t bytes) { a += (bytes + 255) / 256 * 256; };
  add((size_t)B * sh.n_in * 2);       // X
  add((size_t)B * 4);                 // s
  add((size_t)B * sh.hidden * 4 * 2); // A1, A2 (FP32 pre-activations)
  add((size_t)B * sh.hidden * 2 * 2); // H1, H2 (BF16)
  add((size_t)B * sh.n_out * 4);      // O
  add((size_t)B * sh.n_out * 2);      // dO (BF16)
  add((size_t)B * sh.n_out * 4);      // dO (FP32)
  add((size_t)B * sh.hidden * 2 * 2); // dA2, dA1 (BF16)
  add((size_t)B * sh.hidden * 4 * 2); // dA2, dA1 (FP32)
  add((size_t)B * 4);                 // loss
  return a;
}

void mlp_work_carve(void* base, const MlpShape& sh, int B, MlpWork* w) {
  char* p = (char*)base;
  auto take = [&](size_t bytes) {
    void* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  w->X = (uint16_t*)take((size_t)B * sh.n_in * 2);
  w->s = (float*)take((size_t)B * 4);
  w->A1 = (float*)take((size_t)B * sh.hidden * 4);
  w->A2 = (float*)take((size_t)B * sh.hidden * 4);
  w->H1 = (uint16_t*)take((size_t)B * sh.hidden * 2);
  w->H2 = (uint16_t*)take((size_t)B * sh.hidden * 2);
  w->O = (float*)take((size_t)B * sh.n_out * 4);
  w->dOh = (uint16_t*)take((size_t)B * sh.n_out * 2);
  w->dOf = (float*)take((size_t)B * sh.n_out * 4);
  w->dA2h = (uint16_t*)take((size_t)B * sh.hidden * 2);
  w->dA1h = (uint16_t*)take((size_t)B * sh.hidden * 2);
  w->dA2f = (float*)take((size_t)B * sh.hidden * 4);
  w->dA1f = (float*)take((size_t)B * sh.hidden * 4);
  w->loss = (float*)take((size_t)B * 4);
}

int mlp_forward(const MlpShape& sh, const MlpParams& P, const float* I, int B, int KN, MlpWork& w, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  k_features<<<B, 256, 0, s>>>(I, sh.n_in, B, w.X, w.s, (float)KN);
  int e = (int)hipGetLastError();
  if (e) return e;
  return mlp_forward_x(sh, P, B, w, stream);
}

int mlp_forward_x(const MlpShape& sh, const MlpParams& P, int B, MlpWork& w, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int e = 0;
  GemmArgs g1 = ga(B, sh.hidden, sh.n_in, w.X, sh.n_in, 0, P.Wh[0], sh.hidden, 0, MLP_EPI_BIAS_GELU);
  g1.bias = P.b[0];
  g1.outf2 = w.A1;
  g1.outh = w.H1;
  if ((e = gemm(g1, s))) return e;
  GemmArgs g2 = ga(B, sh.hidden, sh.hidden, w.H1, sh.hidden, 0, P.Wh[1], sh.hidden, 0, MLP_EPI_BIAS_GELU);
  g2.bias = P.b[1];
  g2.outf2 = w.A2;
  g2.outh = w.H2;
  if ((e = gemm(g2, s))) return e;
  GemmArgs g3 = ga(B, sh.n_out, sh.hidden, w.H2, sh.hidden, 0, P.Wh[2], sh.n_out, 0, MLP_EPI_BIAS);
  g3.bias = P.b[2];
  g3.outf = w.O;
  return gemm(g3, s);
}

int mlp_start(const MlpWork& w, int P, int N, void* t0, void* stream) {
  k_start<<<P, 256, 0, (hipStream_t)stream>>>(w.O, w.s, P, N, (float2*)t0);
  return (int)hipGetLastError();
}

int mlp_backward(const MlpShape& sh, const MlpParams& P, const void* t, int B, MlpWork& w, MlpGrads& G,
                 void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int N = sh.n_out / 2;
  k_loss<<<B, 256, 0, s>>>(w.O, (const float2*)t, w.s, B, N, w.dOh, w.dOf, w.loss, 1.f / (float)B);
  int e = (int)hipGetLastError();
  if (e) return e;
  return mlp_backward_dout(sh, P, B, w, G, stream);
}

int mlp_backward_dout(const MlpShape& sh, const MlpParams& P, int B, MlpWork& w, MlpGrads& G, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  int e = 0;
  // layer 3: dW3 = H2^T dO, db3 = colsum(dO), dA2 = (dO W3^T) * gelu'(A2)
  GemmArgs d3 = ga(sh.hidden, sh.n_out, B, w.H2, sh.hidden, 1, w.dOh, sh.n_out, 0, MLP_EPI_STORE);
  d3.outf = G.dW[2];
  if ((e = gemm(d3, s))) return e;
  k_colsum<<<(sh.n_out + 255) / 256, 256, 0, s>>>(w.dOf, B, sh.n_out, G.db[2]);
  GemmArgs x2 = ga(B, sh.hidden, sh.n_out, w.dOh, sh.n_out, 0, P.Wh[2], sh.n_out, 1, MLP_EPI_GELU_BWD);
  x2.aux = w.A2;
  x2.outh = w.dA2h;
  x2.outf = w.dA2f;
  if ((e = gemm(x2, s))) return e;
  // layer 2
  GemmArgs d2 = ga(sh.hidden, sh.hidden, B, w.H1, sh.hidden, 1, w.dA2h, sh.hidden, 0, MLP_EPI_STORE);
  d2.outf = G.dW[1];
  if ((e = gemm(d2, s))) return e;
  k_colsum<<<(sh.hidden + 255) / 256, 256, 0, s>>>(w.dA2f, B, sh.hidden, G.db[1]);
  GemmArgs x1 = ga(B, sh.hidden, sh.hidden, w.dA2h, sh.hidden, 0, P.Wh[1], sh.hidden, 1, MLP_EPI_GELU_BWD);
  x1.aux = w.A1;
  x1.outh = w.dA1h;
  x1.outf = w.dA1f;
  if ((e = gemm(x1, s))) return e;
  // layer 1
  GemmArgs d1 = ga(sh.n_in, sh.hidden, B, w.X, sh.n_in, 1, w.dA1h, sh.hidden, 0, MLP_EPI_STORE);
  d1.outf = G.dW[0];
  if ((e = gemm(d1, s))) return e;
  k_colsum<<<(sh.hidden + 255) / 256, 256, 0, s>>>(w.dA1f, B, sh.hidden, G.db[0]);
  return (int)hipGetLastError();
}

int mlp_adam(const MlpShape& sh, MlpParams& P, const MlpGrads& G, MlpAdam& A, float lr, int step, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  size_t nw[3] = {(size_t)sh.n_in * sh.hidden, (size_t)sh.hidden * sh.hidden, (size_t)sh.hidden * sh.n_out};
  size_t nb[3] = {(size_t)sh.hidden, (size_t)sh.hidden, (size_t)sh.n_out};
  for (int l = 0; l < 3; ++l) {
    unsigned gw = (unsigned)((nw[l] + 255) / 256 > 8192 ? 8192 : (nw[l] + 255) / 256);
    k_adam<<<gw, 256, 0, s>>>(P.W[l], A.mW[l], A.vW[l], G.dW[l], P.Wh[l], nw[l], lr, b1, b2, eps, c1, c2);
    unsigned gb = (unsigned)((nb[l] + 255) / 256);
    k_adam<<<gb, 256, 0, s>>>(P.b[l], A.mb[l], A.vb[l], G.db[l], nullptr, nb[l], lr, b1, b2, eps, c1, c2);
  }
  return (int)hipGetLastError();
}

int mlp_weights_to_bf16(const MlpShape& sh, MlpParams& P, void* stream) {
  size_t nw[3] = {(size_t)sh.n_in * sh.hidden, (size_t)sh.hidden * sh.hidden, (size_t)sh.hidden * sh.n_out};
  for (int l = 0; l < 3; ++l) {
    k_to_bf16<<<(unsigned)((nw[l] + 255) / 256), 256, 0, (hipStream_t)stream>>>(P.W[l], P.Wh[l], nw[l]);
  }
  return (int)hipGetLastError();
}

int gemm_bf16(int M, int N, int K, const uint16_t* A, int ta, const uint16_t* B, int tb, float* C, void* stream) {
  GemmArgs g = ga(M, N, K, A, ta ? M : K, ta, B, tb ? K : N, tb, MLP_EPI_STORE);
  g.outf = C;
  return gemm(g, (hipStream_t)stream);
}

}  // namespace tmk
