// Complex FP32 GEMM on the FP32 matrix cores (v_mfma_f32_32x32x2_f32):
//   C[m][n] = sum_k A[m][k] op(B)[k][n]   (complex64, row-major)
// A is [M][K] (k contiguous); B is [N][K] (k contiguous, trans_b) or [K][N]
// (n contiguous). Used by the foci (patterns times the true TM, Sec. 3) and
// the dense-probing comparator (a random-phase Q in place of the FFTs).
//
// Real embedding of the complex product: for one complex k the MFMA's two
// real k are (real part, imaginary part), so that
//   C_r += [a_r a_i] . [b_r, -b_i],   C_i += [a_r a_i] . [b_i, b_r]:
// one 32x32x2 MFMA each, lanes 0-31 carrying the real parts of A (and of the
// first B operand), lanes 32-63 the imaginary parts. 128 x 128 output tiles,
// 256 threads (four waves of 64 x 64), K in steps of 16 complex values staged
// in LDS k-major ([k][row]: the 32 lanes of a half-wave read 32 consecutive
// rows), double-buffered through registers: the next step's tiles load while
// the MFMAs run on the current one.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmk {

namespace {

typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int TM = 128, TN = 128, TK = 16;  // tile rows, columns, complex k per step
constexpr int VPT = TK * TM / 256;           // complex values of a tile per thread and operand

struct CgemmArgs {
  int M, N, K;
  const float2* A;
  int64_t lda;
  const float2* B;
  int64_t ldb;
  int trans_b;  // B stored [N][K]
  float2* C;
  int64_t ldc;
  int conj_c;   // store conj(C)
  int veca, vecb;  // 16-byte loads of two complex values allowed
};

// A tile's 128 x TK complex values in registers, VPT per thread. k-contiguous
// source (A, or B with trans_b): row r0 + t / 2, k k0 + VPT (t % 2) .. + VPT - 1;
// n-contiguous source (B): k k0 + t / (TM / VPT), n r0 + VPT (t % (TM / VPT)) ...
struct Stage {
  float2 v[VPT];
};

__device__ __forceinline__ void fetch(Stage& s, const float2* __restrict__ p, int64_t ld, bool kcontig, bool vec,
                                      int r0, int k0, int R, int K) {
  const int t = threadIdx.x;
  constexpr int NT = TM / VPT;  // threads along a k-major tile row
  const int a = kcontig ? r0 + (t >> 1) : k0 + t / NT;                  // fixed index (row, or k)
  const int b = kcontig ? k0 + VPT * (t & 1) : r0 + VPT * (t % NT);     // first of VPT consecutive
  const int alim = kcontig ? R : K, blim = kcontig ? K : R;
  const float2* q = p + (int64_t)a * ld + b;
  if (vec && a < alim && b + VPT <= blim) {
#pragma unroll
    for (int i = 0; i < VPT / 2; ++i) {
      const float4 u = ((const float4*)q)[i];
      s.v[2 * i] = make_float2(u.x, u.y);
      s.v[2 * i + 1] = make_float2(u.z, u.w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < VPT; ++i) s.v[i] = (a < alim && b + i < blim) ? q[i] : make_float2(0.f, 0.f);
  }
}

// into LDS as [k][row] (row stride TM complex values)
__device__ __forceinline__ void stage_store(float2* lds, const Stage& s, bool kcontig) {
  const int t = threadIdx.x;
  if (kcontig) {
    const int r = t >> 1, kb = VPT * (t & 1);
#pragma unroll
    for (int i = 0; i < VPT; ++i) lds[(kb + i) * TM + r] = s.v[i];
  } else {
    constexpr int NT = TM / VPT;
    const int k = t / NT, nb = VPT * (t % NT);
    float4* d = (float4*)&lds[k * TM + nb];
#pragma unroll
    for (int i = 0; i < VPT / 2; ++i) d[i] = make_float4(s.v[2 * i].x, s.v[2 * i].y, s.v[2 * i + 1].x, s.v[2 * i + 1].y);
  }
}

__global__ void __launch_bounds__(256, 2) k_cgemm_mfma(CgemmArgs g) {
  __shared__ float2 sA[2][TK * TM];
  __shared__ float2 sB[2][TK * TN];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const bool hi = lane >= 32;
  f32x16 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) cr[i][j][e] = ci[i][j][e] = 0.f;

  const bool bk = g.trans_b != 0;
  Stage ra, rb;
  fetch(ra, g.A, g.lda, true, g.veca != 0, m0, 0, g.M, g.K);
  fetch(rb, g.B, g.ldb, bk, g.vecb != 0, n0, 0, g.N, g.K);
  const int nk = (g.K + TK - 1) / TK;
  for (int ks = 0; ks < nk; ++ks) {
    float2* a_s = sA[ks & 1];
    float2* b_s = sB[ks & 1];
    // this buffer's last readers (step ks - 2) passed the barrier of step ks - 1
    stage_store(a_s, ra, true);
    stage_store(b_s, rb, bk);
    __syncthreads();
    if (ks + 1 < nk) {
      fetch(ra, g.A, g.lda, true, g.veca != 0, m0, (ks + 1) * TK, g.M, g.K);
      fetch(rb, g.B, g.ldb, bk, g.vecb != 0, n0, (ks + 1) * TK, g.N, g.K);
    }
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      float av[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float2 a = a_s[kk * TM + wm + 32 * i + (lane & 31)];
        av[i] = hi ? a.y : a.x;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const float2 b = b_s[kk * TN + wn + 32 * j + (lane & 31)];
        br[j] = hi ? -b.y : b.x;
        bi[j] = hi ? b.x : b.y;
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bi[j], ci[i][j], 0, 0, 0);
        }
    }
  }
  // lane holds column n = lane % 32 of each 32 x 32 block, rows 8 q + 4 (lane / 32) + r for element 4 q + r
  const float sgn = g.conj_c ? -1.f : 1.f;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int m = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int n = n0 + wn + 32 * j + (lane & 31);
        const float x = cr[i][j][e], y = ci[i][j][e];
        if (m < g.M && n < g.N) g.C[(int64_t)m * g.ldc + n] = make_float2(x, sgn * y);
      }
}

}  // namespace

int launch_cgemm(int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb, int trans_b, void* C,
                 int64_t ldc, int conj_c, void* stream) {
  if (M <= 0 || N <= 0) return 0;
  if (K <= 0 || !A || !B || !C || lda < K || (trans_b ? ldb < K : ldb < N) || ldc < N)
    return (int)hipErrorInvalidValue;
  if ((int64_t)(M + TM - 1) / TM > 65535) return (int)hipErrorInvalidValue;
  CgemmArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = (const float2*)A;
  g.lda = lda;
  g.B = (const float2*)B;
  g.ldb = ldb;
  g.trans_b = trans_b;
  g.C = (float2*)C;
  g.ldc = ldc;
  g.conj_c = conj_c;
  g.veca = lda % 2 == 0 && (uintptr_t)A % 16 == 0;
  g.vecb = ldb % 2 == 0 && (uintptr_t)B % 16 == 0;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  k_cgemm_mfma<<<grid, 256, 0, (hipStream_t)stream>>>(g);
  return (int)hipGetLastError();
}

}  // namespace tmk
