// Device L-BFGS for every row at once (Sec. 2.2, Alg. 1; two-loop recursion
// of Nocedal & Wright Alg. 7.4 over R^{2N} with <a, b> = Re(a^H b)).
//
// Per iteration: [direction] finalise the pending (s, y) pair, two-loop ->
// d, descent check; [line sums] fused FFT kernel M_LS gives the six sums of
// the quartic f(t + a d); [step] exact minimiser a > 0 in FP64, t += a d,
// s = a d kept as the pending pair; [gradient] fused FFT kernel M_GRAD.
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
};

__device__ __forceinline__ void ts_add(float& s, float& c, float v) {
  float t = s + v;
  float bp = t - s;
  c += (s - (t - bp)) + (v - bp);
  s = t;
}

// Block-wide compensated sum of NS values; returns the totals in every thread.
template <int NS>
__device__ __forceinline__ void block_sums(float* s, float* c, float* red, double* out) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      float s2 = __shfl_xor(s[i], off, 64), c2 = __shfl_xor(c[i], off, 64);
      float t = s[i] + s2, bp = t - s[i];
      c[i] += c2 + (s[i] - (t - bp)) + (s2 - bp);
      s[i] = t;
    }
  }
  int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      red[(w * NS + i) * 2] = s[i];
      red[(w * NS + i) * 2 + 1] = c[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double acc = 0.0;
    for (int k = 0; k < LWG / 64; ++k) acc += (double)red[(k * NS + i) * 2] + (double)red[(k * NS + i) * 2 + 1];
    out[i] = acc;
  }
}

template <int EPT>
__global__ void __launch_bounds__(LWG) k_direction(LbArgs a) {
  __shared__ float red[(LWG / 64) * 2 * 2];
  const int p = blockIdx.x;
  const int tid = threadIdx.x;
  const int N = a.N, m = a.m;
  const size_t rb = (size_t)p * N;
  double* sc = a.sc + (size_t)p * LB_SCALARS(m);
  int head = (int)sc[0], count = (int)sc[1];
  const int R = m + 1;  // ring slots: m stored pairs + the pending one
  double* sy = sc + 4;
  double* yy = sc + 4 + R;
  float2 q[EPT];
  bool act[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int e = tid + i * LWG;
    act[i] = e < N;
    q[i] = act[i] ? a.g[rb + e] : make_float2(0.f, 0.f);
  }
  // finalise the pending pair (slot head, outside the m stored pairs):
  // y = g - g_prev, accept if s^T y > 0
  if (!a.first && sc[3] != 0.0) {
    float2* Sh = a.S + ((size_t)p * R + head) * N;
    float2* Yh = a.Y + ((size_t)p * R + head) * N;
    float s2[2] = {0.f, 0.f}, c2[2] = {0.f, 0.f};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (!act[i]) continue;
      int e = tid + i * LWG;
      float2 gp = a.gp[rb + e];
      float2 y = make_float2(q[i].x - gp.x, q[i].y - gp.y);
      float2 s = Sh[e];
      Yh[e] = y;
      ts_add(s2[0], c2[0], s.x * y.x + s.y * y.y);
      ts_add(s2[1], c2[1], y.x * y.x + y.y * y.y);
    }
    double o[2];
    block_sums<2>(s2, c2, red, o);
    if (o[0] > 0.0 && isfinite(o[0]) && o[1] > 0.0) {
      sy[head] = o[0];
      yy[head] = o[1];
      head = (head + 1) % R;  // with count == m this drops the oldest pair
      count = count < m ? count + 1 : m;
    }
  }
  // two-loop recursion
  double al[16];
  for (int j = 0; j < count; ++j) {
    int idx = (head - 1 - j + 2 * R) % R;
    const float2* Si = a.S + ((size_t)p * R + idx) * N;
    const float2* Yi = a.Y + ((size_t)p * R + idx) * N;
    float s1[1] = {0.f}, c1[1] = {0.f};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (!act[i]) continue;
      float2 s = Si[tid + i * LWG];
      ts_add(s1[0], c1[0], s.x * q[i].x + s.y * q[i].y);
    }
    double o[1];
    block_sums<1>(s1, c1, red, o);
    double aj = o[0] / sy[idx];
    al[j] = aj;
    float af = (float)aj;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (!act[i]) continue;
      float2 y = Yi[tid + i * LWG];
      q[i].x -= af * y.x;
      q[i].y -= af * y.y;
    }
  }
  {
    float gam = a.h0;
    if (count > 0) {
      int nw = (head - 1 + R) % R;
      gam = (float)(sy[nw] / yy[nw]);
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      q[i].x *= gam;
      q[i].y *= gam;
    }
  }
  for (int j = count - 1; j >= 0; --j) {
    int idx = (head - 1 - j + 2 * R) % R;
    const float2* Si = a.S + ((size_t)p * R + idx) * N;
    const float2* Yi = a.Y + ((size_t)p * R + idx) * N;
    float s1[1] = {0.f}, c1[1] = {0.f};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (!act[i]) continue;
      float2 y = Yi[tid + i * LWG];
      ts_add(s1[0], c1[0], y.x * q[i].x + y.y * q[i].y);
    }
    double o[1];
    block_sums<1>(s1, c1, red, o);
    float cf = (float)(al[j] - o[0] / sy[idx]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (!act[i]) continue;
      float2 s = Si[tid + i * LWG];
      q[i].x += cf * s.x;
      q[i].y += cf * s.y;
    }
  }
  // d = -q; if not a descent direction, drop the history and use the
  // negative gradient. For the exact line search the scale of d does not
  // change the new iterate (the step scales inversely), so with no stored
  // pairs the gradient direction is normalised (unit_first): the quartic's
  // coefficients grow as ||d||^4 and -g itself can overflow their FP32 sums.
  float s1[2] = {0.f, 0.f}, c1[2] = {0.f, 0.f};
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    if (!act[i]) continue;
    float2 g = a.g[rb + tid + i * LWG];
    ts_add(s1[0], c1[0], -(g.x * q[i].x + g.y * q[i].y));
    ts_add(s1[1], c1[1], g.x * g.x + g.y * g.y);
  }
  double sl[2];
  block_sums<2>(s1, c1, red, sl);
  bool reset = !(sl[0] < 0.0);
  const bool plain = reset || count == 0;
  const float gs = (a.unit_first && plain) ? (sl[1] > 0.0 ? (float)(1.0 / sqrt(sl[1])) : 0.f) : a.h0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    if (!act[i]) continue;
    int e = tid + i * LWG;
    float2 v = plain ? make_float2(gs * a.g[rb + e].x, gs * a.g[rb + e].y) : q[i];
    a.d[rb + e] = make_float2(-v.x, -v.y);
  }
  if (tid == 0) {
    sc[0] = head;
    sc[1] = reset ? 0 : count;
  }
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
  if (what == 0) k_direction<EPT><<<a.P, LWG, 0, s>>>(a);
  else if (what == 1) k_step<EPT><<<a.P, LWG, 0, s>>>(a);
  else k_step_amp<EPT><<<a.P, LWG, 0, s>>>(a);
  return (int)hipGetLastError();
}

// what: 0 direction, 1 exact quartic step, 2 amplitude trial step
int dispatch(int what, const LbArgs& a, hipStream_t s) {
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
    if ((e = dispatch(0, la, s))) return e;
    RowArgs ls = base;
    ls.tin = (const cx<float>*)t;
    ls.din = (const cx<float>*)b.d;
    ls.sums = b.sums;
    if ((e = fn(lmode, ibf16, ls, stream))) return e;
    if ((e = dispatch(amplitude ? 2 : 1, la, s))) return e;
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
