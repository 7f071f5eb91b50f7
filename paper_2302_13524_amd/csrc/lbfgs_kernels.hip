// Device L-BFGS for every row at once (Sec. 2.2, Alg. 1; two-loop recursion
// of Nocedal & Wright Alg. 7.4 over R^{2N} with <a, b> = Re(a^H b)).
//
// Per iteration: [direction] finalise the pending (s, y) pair, coefficients
// of the L-BFGS product (compact form), descent check; [line sums] fused FFT
// kernel M_LS forms d from them and gives the six sums of the quartic
// f(t + a d); [step] exact minimiser a > 0 in FP64, t += a d, s = a d kept as
// the pending pair; [gradient] fused FFT kernel M_GRAD.
//
// The amplitude cost (the Poisson-noise variant of the Discussion) runs the
// same loop with M_AGRAD for the gradient and M_ALS for the line: the cost at
// the trial steps 1/8 .. 16, the smallest wins if it is below the cost at t,
// otherwise the step is 0 and the row's history is dropped. With no history
// the direction is -g / (2 K N), whose unit step is an error-reduction step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbfgs.hpp"
#include "row_kernels.hpp"

namespace tmk {

namespace {

constexpr int LWG = 256;

struct LbArgs {
  int P, N, m;
  const float2* g;   // gradient at current t
  const float2* gp;  // gradient at previous t
  float2* d;
  float2* S;
  float2* Y;
  double* sc;
  const float* sums;
  float2* t;
  int first;         // no pending pair
  float h0;          // inverse-Hessian scale with no stored pairs
  int unit_first;    // with no stored pairs use -g/||g|| instead of -h0 g
  double* dots;      // [P][dir_split(N, DEPT)][NDOT] partial dot products of the direction
};

__device__ __forceinline__ void ts_add(float& s, float& c, float v) {
  float t = s + v;
  float bp = t - s;
  c += (s - (t - bp)) + (v - bp);
  s = t;
}

// Merge of two compensated values (TwoSum: t + err is exactly a + b).
__device__ __forceinline__ void ts_merge(float& s, float& c, float s2, float c2) {
  const float t = s + s2, bp = t - s;
  c = (c + c2) + ((s - (t - bp)) + (s2 - bp));
  s = t;
}

// Block-wide compensated sums of NS values over WG threads; thread i < nout
// writes the i-th total to out[i]. Within a wave, lane bits 5 and 4 first
// scatter the values: v_permlane32_swap / v_permlane16_swap exchange the upper
// half of one value's lanes with the lower half of another's, so after one
// swap and one add each lane holds half of the values, summed over its partner
// lane (no per-lane selects); the values left are then added over lane bits
// 3 .. 0 by shuffles. A wave thus exchanges about NS / 2 + 2 NS / 4 ... values
// instead of 6 NS. The waves' totals meet in FP64 in wave order.
template <int NS, int WG = LWG>
__device__ __forceinline__ void block_sums(const float* s, const float* c, float* red, double* out, int nout) {
  constexpr int LB = NS <= 1 ? 0 : NS <= 2 ? 1 : NS <= 4 ? 2 : NS <= 8 ? 3 : NS <= 16 ? 4 : 5;
  constexpr int NP = 1 << LB;
  constexpr int SW = LB < 2 ? LB : 2;  // swap steps (lane bits 5, then 4)
  constexpr int NR = NP >> SW;         // values a lane holds after them
  static_assert(NS <= 32, "at most 32 sums");
  float vs[NP], vc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    vs[i] = i < NS ? s[i] : 0.f;
    vc[i] = i < NS ? c[i] : 0.f;
  }
  if constexpr (SW >= 1) {
    // lanes 0-31 keep value i and add lane l + 32's; lanes 32-63 keep value i + NP/2 and add lane l - 32's
#pragma unroll
    for (int i = 0; i < NP / 2; ++i) {
      auto ps = __builtin_amdgcn_permlane32_swap(__float_as_uint(vs[i]), __float_as_uint(vs[i + NP / 2]), false, false);
      auto pc = __builtin_amdgcn_permlane32_swap(__float_as_uint(vc[i]), __float_as_uint(vc[i + NP / 2]), false, false);
      vs[i] = __uint_as_float(ps[0]);
      vc[i] = __uint_as_float(pc[0]);
      ts_merge(vs[i], vc[i], __uint_as_float(ps[1]), __uint_as_float(pc[1]));
    }
  }
  if constexpr (SW >= 2) {
    // the same over lane bit 4 (rows of 16 lanes)
#pragma unroll
    for (int i = 0; i < NP / 4; ++i) {
      auto ps = __builtin_amdgcn_permlane16_swap(__float_as_uint(vs[i]), __float_as_uint(vs[i + NP / 4]), false, false);
      auto pc = __builtin_amdgcn_permlane16_swap(__float_as_uint(vc[i]), __float_as_uint(vc[i + NP / 4]), false, false);
      vs[i] = __uint_as_float(ps[0]);
      vc[i] = __uint_as_float(pc[0]);
      ts_merge(vs[i], vc[i], __uint_as_float(ps[1]), __uint_as_float(pc[1]));
    }
  }
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 32 >> SW; off >= 1; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NR; ++i) ts_merge(vs[i], vc[i], __shfl_xor(vs[i], off, 64), __shfl_xor(vc[i], off, 64));
  }
  // lane bits 5 .. 6 - SW name the block of NR values a lane holds
  const int w = threadIdx.x >> 6, blk = lane >> (6 - SW);
  __syncthreads();  // the previous call's readers are done with red
  if ((lane & ((64 >> SW) - 1)) == 0) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int idx = blk * NR + i;
      if (idx < NS) {
        red[(w * NS + idx) * 2] = vs[i];
        red[(w * NS + idx) * 2 + 1] = vc[i];
      }
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < nout) {
    const int i = threadIdx.x;
    double acc = 0.0;
    for (int k = 0; k < WG / 64; ++k) acc += (double)red[(k * NS + i) * 2] + (double)red[(k * NS + i) * 2 + 1];
    out[i] = acc;
  }
}

// Direction from the compact representation of the L-BFGS matrix (Byrd,
// Nocedal & Schnabel 1994): with the stored pairs in age order, S^T g, Y^T g,
// R = upper triangle of S^T Y, D = diag(S^T Y) and Y^T Y,
//   H g = gam g + S p - gam Y u,  R u = S^T g,  R^T p = (D + gam Y^T Y) u - gam Y^T g,
// the same product as the two-loop recursion of Nocedal & Wright Alg. 7.4,
// but with every dot product against g and the pending pair's y known after
// one pass over the history. Two kernels, the first with each row split over
// several workgroups so that its pass streams at full occupancy:
//   k_dir_dots:  partial dot products of each row slice (the pending pair's y
//                is formed and stored here);
//   k_dir_solve: per row, the slices' partials summed in a fixed order, the
//                pending pair accepted or skipped (S^T Y, Y^T Y updated over the
//                ring slots), the small triangular solves, the descent check;
//                writes the coefficients of d = cg g + sum_j cs_j s_j + cy_j y_j.
// The second pass over the history, d itself, is the prologue of the line
// search's row kernel (M_LS / M_ALS), where its loads overlap other rows'
// transforms instead of taking a launch of its own.
constexpr int MMAX = 16;
constexpr int NDOT = 5 + 4 * MMAX;  // partial sums per slice: pending pair, g^T g, 4 per stored pair
constexpr int DEPT = 4;    // values per thread in the split kernels

__host__ __device__ constexpr int dir_split(int N, int ept) { return N > LWG * ept ? N / (LWG * ept) : 1; }
__device__ __forceinline__ double* lb_coef(double* sc, int m) { return sc + 4 + 2 * LB_SLOTS(m) * LB_SLOTS(m); }

// dots[(p * split + q) * NDOT + k]: 0..3 s^T y, y^T y, s^T g, y^T g of the pending pair,
// 4 g^T g, 5 + 4 j + {0..3} s_j^T g, y_j^T g, s_j^T y_new, y_j^T y_new (age order j).
// Up to CFIX stored pairs a body specialised on their count issues every load
// of the slice before the sums and reduces all 5 + 4 C sums at once; beyond
// that, pairs go in groups of DG with one block reduction per group.
constexpr int DG = 4;
constexpr int CFIX = 6;  // 5 + 4 CFIX sums fit one block reduction

// ring slot of stored pair j (age order) given the newest's successor head
__device__ __forceinline__ size_t pair_base(int p, int R, int head, int count, int j, int N, int q, int L) {
  return ((size_t)p * R + (head - count + j + 2 * R) % R) * N + (size_t)q * L;
}

template <int C>
__device__ __forceinline__ void dots_fixed(const LbArgs& a, float* red, double* out, const float2* gv,
                                           const bool* act, bool pending, size_t rb, size_t hb, int p, int R,
                                           int head, int q, int L) {
  constexpr int NS = 5 + 4 * C, CC = C > 0 ? C : 1;
  const int tid = threadIdx.x;
  float2 gp[DEPT], sh[DEPT], sv[CC][DEPT], yy[CC][DEPT];
#pragma unroll
  for (int i = 0; i < DEPT; ++i) {
    gp[i] = sh[i] = make_float2(0.f, 0.f);
    if (act[i] && pending) {
      gp[i] = a.gp[rb + tid + i * LWG];
      sh[i] = a.S[hb + tid + i * LWG];
    }
  }
#pragma unroll
  for (int j = 0; j < C; ++j) {
    const size_t sb = pair_base(p, R, head, C, j, a.N, q, L);
#pragma unroll
    for (int i = 0; i < DEPT; ++i) {
      sv[j][i] = yy[j][i] = make_float2(0.f, 0.f);
      if (act[i]) {
        sv[j][i] = a.S[sb + tid + i * LWG];
        yy[j][i] = a.Y[sb + tid + i * LWG];
      }
    }
  }
  float s[NS], c[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) s[k] = c[k] = 0.f;
#pragma unroll
  for (int i = 0; i < DEPT; ++i) {
    if (!act[i]) continue;
    const float2 g = gv[i];
    float2 y = make_float2(0.f, 0.f);
    ts_add(s[4], c[4], g.x * g.x + g.y * g.y);
    if (pending) {
      y = make_float2(g.x - gp[i].x, g.y - gp[i].y);
      a.Y[hb + tid + i * LWG] = y;
      ts_add(s[0], c[0], sh[i].x * y.x + sh[i].y * y.y);
      ts_add(s[1], c[1], y.x * y.x + y.y * y.y);
      ts_add(s[2], c[2], sh[i].x * g.x + sh[i].y * g.y);
      ts_add(s[3], c[3], y.x * g.x + y.y * g.y);
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const float2 sj = sv[j][i], yj = yy[j][i];
      ts_add(s[5 + 4 * j + 0], c[5 + 4 * j + 0], sj.x * g.x + sj.y * g.y);
      ts_add(s[5 + 4 * j + 1], c[5 + 4 * j + 1], yj.x * g.x + yj.y * g.y);
      ts_add(s[5 + 4 * j + 2], c[5 + 4 * j + 2], sj.x * y.x + sj.y * y.y);
      ts_add(s[5 + 4 * j + 3], c[5 + 4 * j + 3], yj.x * y.x + yj.y * y.y);
    }
  }
  block_sums<NS>(s, c, red, out, NS);
}

__global__ void __launch_bounds__(LWG) k_dir_dots(LbArgs a, double* dots) {
  __shared__ float red[(LWG / 64) * 2 * (5 + 4 * CFIX)];
  const int p = blockIdx.y, q = blockIdx.x, split = gridDim.x;
  const int tid = threadIdx.x;
  const int N = a.N, m = a.m, R = m + 1;
  const int L = N / split;
  const size_t rb = (size_t)p * N + (size_t)q * L;
  const double* sc = a.sc + (size_t)p * LB_SCALARS(m);
  const int head = (int)sc[0], count = (int)sc[1];
  const bool pending = !a.first && sc[3] != 0.0;
  double* out = dots + ((size_t)p * split + q) * NDOT;
  float2 gv[DEPT], yv[DEPT];
  bool act[DEPT];
#pragma unroll
  for (int i = 0; i < DEPT; ++i) {
    const int e = tid + i * LWG;
    act[i] = e < L;
    gv[i] = act[i] ? a.g[rb + e] : make_float2(0.f, 0.f);
    yv[i] = make_float2(0.f, 0.f);
  }
  const size_t hb0 = ((size_t)p * R + head) * N + (size_t)q * L;
  switch (count) {  // uniform over the workgroup (one row)
    case 0: return dots_fixed<0>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 1: return dots_fixed<1>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 2: return dots_fixed<2>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 3: return dots_fixed<3>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 4: return dots_fixed<4>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 5: return dots_fixed<5>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    case 6: return dots_fixed<6>(a, red, out, gv, act, pending, rb, hb0, p, R, head, q, L);
    default: break;
  }
  {
    float s5[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, c5[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    const size_t hb = ((size_t)p * R + head) * N + (size_t)q * L;
#pragma unroll
    for (int i = 0; i < DEPT; ++i) {
      if (!act[i]) continue;
      const int e = tid + i * LWG;
      ts_add(s5[4], c5[4], gv[i].x * gv[i].x + gv[i].y * gv[i].y);
      if (pending) {
        const float2 gp = a.gp[rb + e];
        const float2 y = make_float2(gv[i].x - gp.x, gv[i].y - gp.y);
        const float2 sv = a.S[hb + e];
        a.Y[hb + e] = y;
        yv[i] = y;
        ts_add(s5[0], c5[0], sv.x * y.x + sv.y * y.y);
        ts_add(s5[1], c5[1], y.x * y.x + y.y * y.y);
        ts_add(s5[2], c5[2], sv.x * gv[i].x + sv.y * gv[i].y);
        ts_add(s5[3], c5[3], y.x * gv[i].x + y.y * gv[i].y);
      }
    }
    block_sums<5>(s5, c5, red, out, 5);
  }
  for (int j0 = 0; j0 < count; j0 += DG) {
    float s4[4 * DG], c4[4 * DG];
#pragma unroll
    for (int k = 0; k < 4 * DG; ++k) s4[k] = c4[k] = 0.f;
#pragma unroll
    for (int u = 0; u < DG; ++u) {
      const int j = j0 + u;
      if (j >= count) break;
      const size_t sb = pair_base(p, R, head, count, j, N, q, L);
#pragma unroll
      for (int i = 0; i < DEPT; ++i) {
        if (!act[i]) continue;
        const int e = tid + i * LWG;
        const float2 sv = a.S[sb + e], y = a.Y[sb + e];
        ts_add(s4[4 * u + 0], c4[4 * u + 0], sv.x * gv[i].x + sv.y * gv[i].y);
        ts_add(s4[4 * u + 1], c4[4 * u + 1], y.x * gv[i].x + y.y * gv[i].y);
        ts_add(s4[4 * u + 2], c4[4 * u + 2], sv.x * yv[i].x + sv.y * yv[i].y);
        ts_add(s4[4 * u + 3], c4[4 * u + 3], y.x * yv[i].x + y.y * yv[i].y);
      }
    }
    block_sums<4 * DG>(s4, c4, red, out + 5 + 4 * j0, min(4 * DG, 4 * (count - j0)));
  }
}

// One wave per row: sums of the slices' partials (fixed order), then lane 0
// accepts the pending pair, solves, and writes head, count and the coefficients.
__global__ void __launch_bounds__(64) k_dir_solve(LbArgs a, const double* dots, int split) {
  __shared__ double tot[NDOT];
  __shared__ double Rm[MMAX * MMAX], Wm[MMAX * MMAX];
  const int p = blockIdx.x, lane = threadIdx.x;
  const int m = a.m, R = m + 1;
  double* sc = a.sc + (size_t)p * LB_SCALARS(m);
  const int count0 = (int)sc[1];
  const int nd = 5 + 4 * count0;
  for (int k = lane; k < nd; k += 64) {
    double acc = 0.0;
    for (int q = 0; q < split; ++q) acc += dots[((size_t)p * split + q) * NDOT + k];
    tot[k] = acc;
  }
  __syncthreads();
  if (lane != 0) return;
  double* STY = sc + 4;          // [R][R] s_i^T y_j over ring slots
  double* YTY = sc + 4 + R * R;  // [R][R] y_i^T y_j
  double* coef = lb_coef(sc, m);  // cg, cs[R], cy[R]
  const int head0 = (int)sc[0];
  const bool pending = !a.first && sc[3] != 0.0;
  const double* nw = tot;  // s^T y, y^T y, s^T g, y^T g, g^T g of the pending pair
  double sg[MMAX], yg[MMAX], sy[MMAX], yy[MMAX];
  for (int j = 0; j < count0; ++j) {
    sg[j] = tot[5 + 4 * j];
    yg[j] = tot[6 + 4 * j];
    sy[j] = tot[7 + 4 * j];
    yy[j] = tot[8 + 4 * j];
  }
  // accept the pending pair if s^T y > 0: it becomes the newest stored pair
  // (with m pairs stored, the oldest drops out of the ring)
  const bool acc = pending && nw[0] > 0.0 && isfinite(nw[0]) && nw[1] > 0.0;
  const int drop = (acc && count0 == m) ? 1 : 0;
  const int keep = count0 - drop;
  const int k = keep + (acc ? 1 : 0);
  auto oslot = [&](int j) { return (head0 - count0 + j + 2 * R) % R; };
  for (int i = 0; i < keep; ++i) {
    for (int j = 0; j < keep; ++j) {
      Rm[i * MMAX + j] = STY[oslot(drop + i) * R + oslot(drop + j)];
      Wm[i * MMAX + j] = YTY[oslot(drop + i) * R + oslot(drop + j)];
    }
    sg[i] = sg[drop + i];
    yg[i] = yg[drop + i];
    sy[i] = sy[drop + i];
    yy[i] = yy[drop + i];
  }
  int head = head0;
  if (acc) {
    for (int i = 0; i < keep; ++i) {
      Rm[i * MMAX + keep] = sy[i];
      Wm[i * MMAX + keep] = Wm[keep * MMAX + i] = yy[i];
      const int si = oslot(drop + i);
      STY[si * R + head0] = sy[i];
      YTY[si * R + head0] = YTY[head0 * R + si] = yy[i];
    }
    Rm[keep * (MMAX + 1)] = nw[0];
    Wm[keep * (MMAX + 1)] = nw[1];
    STY[head0 * R + head0] = nw[0];
    YTY[head0 * R + head0] = nw[1];
    sg[keep] = nw[2];
    yg[keep] = nw[3];
    head = (head0 + 1) % R;
  }
  // d = -H g = -gam g - S p + gam Y u with R u = S^T g, R^T p = (D + gam Y^T Y) u - gam Y^T g
  const double gg = nw[4];
  double cg = 0.0;
  double u[MMAX], pv[MMAX];
  bool use = k > 0;
  if (use) {
    const double gam = Rm[(k - 1) * (MMAX + 1)] / Wm[(k - 1) * (MMAX + 1)];
    for (int i = k - 1; i >= 0; --i) {
      double t = sg[i];
      for (int j = i + 1; j < k; ++j) t -= Rm[i * MMAX + j] * u[j];
      u[i] = t / Rm[i * (MMAX + 1)];
    }
    for (int i = 0; i < k; ++i) {
      double t = Rm[i * (MMAX + 1)] * u[i] - gam * yg[i];
      for (int j = 0; j < k; ++j) t += gam * Wm[i * MMAX + j] * u[j];
      for (int j = 0; j < i; ++j) t -= Rm[j * MMAX + i] * pv[j];
      pv[i] = t / Rm[i * (MMAX + 1)];
    }
    double slope = -gam * gg;
    for (int j = 0; j < k; ++j) slope += -pv[j] * sg[j] + gam * u[j] * yg[j];
    cg = -gam;
    for (int j = 0; j < k; ++j) {
      coef[1 + j] = -pv[j];
      coef[1 + R + j] = gam * u[j];
    }
    if (!(slope < 0.0) || !isfinite(slope)) use = false;  // not a descent direction: drop the history
  }
  if (!use) {
    // the negative gradient; normalised (unit_first) for the exact line search,
    // whose new iterate does not depend on the direction's scale and whose
    // quartic coefficients grow as ||d||^4 (-g itself can overflow their FP32 sums)
    cg = a.unit_first ? (gg > 0.0 ? -1.0 / sqrt(gg) : 0.0) : -(double)a.h0;
  }
  coef[0] = cg;
  sc[0] = head;
  sc[1] = use ? k : 0;
}

// phi(a) = c1 a + c2 a^2 + c3 a^3 + c4 a^4
__device__ __forceinline__ double quart(double c1, double c2, double c3, double c4, double x) {
  return x * (c1 + x * (c2 + x * (c3 + x * c4)));
}

// Exact minimiser over a > 0 among the real roots of phi'(a) = 0 (smallest
// value, ties to the smaller a); 0 when there is none.
__device__ double exact_step(double c1, double c2, double c3, double c4) {
  if (!(c4 > 0.0)) {
    if (c2 > 0.0 && c1 < 0.0) return -c1 / (2.0 * c2);
    return 0.0;
  }
  // 4c4 a^3 + 3c3 a^2 + 2c2 a + c1 = 0  ->  a^3 + B a^2 + C a + D = 0
  double B = 3.0 * c3 / (4.0 * c4), C = 2.0 * c2 / (4.0 * c4), D = c1 / (4.0 * c4);
  double p = C - B * B / 3.0;
  double q = 2.0 * B * B * B / 27.0 - B * C / 3.0 + D;
  double roots[3];
  int nr = 0;
  double disc = q * q / 4.0 + p * p * p / 27.0;
  if (disc > 0.0) {
    double sd = sqrt(disc);
    double u = cbrt(-q / 2.0 + sd), v = cbrt(-q / 2.0 - sd);
    roots[nr++] = u + v - B / 3.0;
  } else if (p < 0.0) {
    double r = 2.0 * sqrt(-p / 3.0);
    double arg = (3.0 * q / (2.0 * p)) * sqrt(-3.0 / p);
    arg = fmin(1.0, fmax(-1.0, arg));
    double th = acos(arg) / 3.0;
    for (int k = 0; k < 3; ++k) roots[nr++] = r * cos(th - 2.0 * M_PI * k / 3.0) - B / 3.0;
  } else {
    roots[nr++] = -B / 3.0;  // triple root
  }
  double best = 0.0, bestv = 0.0;
  bool have = false;
  for (int k = 0; k < nr; ++k) {
    double x = roots[k];
    for (int it = 0; it < 2; ++it) {  // Newton polish on the cubic
      double f = ((4.0 * c4 * x + 3.0 * c3) * x + 2.0 * c2) * x + c1;
      double fp = (12.0 * c4 * x + 6.0 * c3) * x + 2.0 * c2;
      if (fp != 0.0) x -= f / fp;
    }
    if (!(x > 0.0) || !isfinite(x)) continue;
    double v = quart(c1, c2, c3, c4, x);
    if (!have || v < bestv || (v == bestv && x < best)) {
      best = x;
      bestv = v;
      have = true;
    }
  }
  return have ? best : 0.0;
}

template <int EPT>
__global__ void __launch_bounds__(LWG) k_step(LbArgs a) {
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, m = a.m;
  const size_t rb = (size_t)p * N;
  double* sc = a.sc + (size_t)p * LB_SCALARS(m);
  const float* s = a.sums + (size_t)p * NSUM;
  // f(a) = sum (r - 2ab - a^2 c)^2 with sums {r^2, rb, b^2, rc, bc, c^2}
  double c1 = -4.0 * (double)s[1];
  double c2 = 4.0 * (double)s[2] - 2.0 * (double)s[3];
  double c3 = 4.0 * (double)s[4];
  double c4 = (double)s[5];
  double al = exact_step(c1, c2, c3, c4);
  int head = (int)sc[0];
  float af = (float)al;
  float2* Sh = a.S + ((size_t)p * (m + 1) + head) * N;  // pending slot
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int e = tid + i * LWG;
    if (e >= N) continue;
    float2 dv = a.d[rb + e];
    float2 st = make_float2(af * dv.x, af * dv.y);
    float2 tv = a.t[rb + e];
    a.t[rb + e] = make_float2(tv.x + st.x, tv.y + st.y);
    Sh[e] = st;
  }
  if (tid == 0) {
    sc[2] = al;
    sc[3] = (al > 0.0) ? 1.0 : 0.0;  // pending pair exists
  }
}

// Amplitude line search: sums {f_a(t), f_a(t + a_j d)} with a_j = 2^(j-3).
template <int EPT>
__global__ void __launch_bounds__(LWG) k_step_amp(LbArgs a) {
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, m = a.m;
  const size_t rb = (size_t)p * N;
  double* sc = a.sc + (size_t)p * LB_SCALARS(m);
  const float* s = a.sums + (size_t)p * NSUM;
  int jb = 0;
  for (int j = 1; j < AMP_TRIALS; ++j)
    if (s[1 + j] < s[1 + jb]) jb = j;  // first minimum: the smaller step on ties
  const double al = (s[1 + jb] < s[0]) ? ldexp(1.0, jb - 3) : 0.0;
  int head = (int)sc[0];
  const float af = (float)al;
  float2* Sh = a.S + ((size_t)p * (m + 1) + head) * N;  // pending slot
  if (al > 0.0) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      int e = tid + i * LWG;
      if (e >= N) continue;
      float2 dv = a.d[rb + e];
      float2 st = make_float2(af * dv.x, af * dv.y);
      float2 tv = a.t[rb + e];
      a.t[rb + e] = make_float2(tv.x + st.x, tv.y + st.y);
      Sh[e] = st;
    }
  }
  if (tid == 0) {
    sc[2] = al;
    sc[3] = (al > 0.0) ? 1.0 : 0.0;  // pending pair exists
    if (al == 0.0) sc[1] = 0.0;      // no decrease: drop the history
  }
}

__global__ void k_lb_init(double* sc, int P, int m) {
  int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  double* r = sc + (size_t)p * LB_SCALARS(m);
  for (int i = 0; i < LB_SCALARS(m); ++i) r[i] = 0.0;
}

template <int EPT>
int launch_dir_step(int what, const LbArgs& a, hipStream_t s) {
  if (what == 1) k_step<EPT><<<a.P, LWG, 0, s>>>(a);
  else k_step_amp<EPT><<<a.P, LWG, 0, s>>>(a);
  return (int)hipGetLastError();
}

// what: 0 direction, 1 exact quartic step, 2 amplitude trial step
int dispatch(int what, const LbArgs& a, hipStream_t s) {
  if (what == 0) {
    const int split = dir_split(a.N, DEPT);
    if (a.N % split || a.N / split > LWG * DEPT || a.m > MMAX) return (int)hipErrorInvalidValue;
    k_dir_dots<<<dim3(split, a.P), LWG, 0, s>>>(a, a.dots);
    k_dir_solve<<<a.P, 64, 0, s>>>(a, a.dots, split);
    return (int)hipGetLastError();
  }
  int ept = (a.N + LWG - 1) / LWG;
  switch (ept) {
    case 1: return launch_dir_step<1>(what, a, s);
    case 2: return launch_dir_step<2>(what, a, s);
    case 4: return launch_dir_step<4>(what, a, s);
    case 8: return launch_dir_step<8>(what, a, s);
    case 16: return launch_dir_step<16>(what, a, s);
    case 32: return launch_dir_step<32>(what, a, s);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace

int run_lbfgs(row_launcher fn, const RowArgs& base, int ibf16, int N, int iters, int m, void* t,
              LbfgsBuffers& b, void* stream, int amplitude) {
  const int gmode = amplitude ? M_AGRAD : M_GRAD, lmode = amplitude ? M_ALS : M_LS;
  hipStream_t s = (hipStream_t)stream;
  const int P = base.P;
  k_lb_init<<<(P + 255) / 256, 256, 0, s>>>((double*)b.sc, P, m);
  int e = (int)hipGetLastError();
  if (e) return e;
  void* gcur = b.g;
  void* gprev = b.gp;
  RowArgs ga = base;
  ga.tin = (const cx<float>*)t;
  ga.tout = (cx<float>*)gcur;
  ga.sums = (iters == 0) ? b.sums : nullptr;  // f is reported for the final point only
  if ((e = fn(gmode, ibf16, ga, stream))) return e;
  for (int it = 0; it < iters; ++it) {
    LbArgs la;
    la.P = P;
    la.N = N;
    la.m = m;
    la.g = (const float2*)gcur;
    la.gp = (const float2*)gprev;
    la.d = (float2*)b.d;
    la.S = (float2*)b.S;
    la.Y = (float2*)b.Y;
    la.sc = (double*)b.sc;
    la.sums = b.sums;
    la.t = (float2*)t;
    la.first = (it == 0);
    la.h0 = amplitude ? 1.f / (2.f * (float)base.K * (float)N) : 1.f;
    la.unit_first = !amplitude;
    la.dots = (double*)b.dots;
    if (b.hook_begin) b.hook_begin(b.hook_user, 20, stream);
    e = dispatch(0, la, s);
    if (b.hook_end) b.hook_end(b.hook_user, 20, stream);
    if (e) return e;
    RowArgs ls = base;  // forms d from the coefficients, then the line sums
    ls.tin = (const cx<float>*)t;
    ls.din = nullptr;
    ls.lb_g = (const cx<float>*)gcur;
    ls.lb_S = (const cx<float>*)b.S;
    ls.lb_Y = (const cx<float>*)b.Y;
    ls.lb_sc = (const double*)b.sc;
    ls.lb_d = (cx<float>*)b.d;
    ls.lb_m = m;
    ls.sums = b.sums;
    if ((e = fn(lmode, ibf16, ls, stream))) return e;
    if (b.hook_begin) b.hook_begin(b.hook_user, 21, stream);
    e = dispatch(amplitude ? 2 : 1, la, s);
    if (b.hook_end) b.hook_end(b.hook_user, 21, stream);
    if (e) return e;
    // gradient at the new t into the other buffer
    void* tmp = gprev;
    gprev = gcur;
    gcur = tmp;
    ga.tout = (cx<float>*)gcur;
    ga.sums = (it == iters - 1) ? b.sums : nullptr;
    if ((e = fn(gmode, ibf16, ga, stream))) return e;
  }
  return 0;
}

}  // namespace tmk
