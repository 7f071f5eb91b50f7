// Fused per-row kernels: mask multiply + 2-D FFT + pointwise measurement
// step + inverse 2-D FFT + conj-mask accumulation, one row per thread group,
// rows independent (the per-pixel decomposition of Sec. 2.2).
#pragma once
#include "fft_core.hpp"
#include "lbfgs.hpp"

namespace tmk {

enum Mode : int {
  M_FWD_FIELD = 0,   // y = A t                                     -> yout c32 [P][K][N]
  M_FWD_INT = 1,     // I = |A t|^2                                 -> yout float/bf16 [P][K][N]
  M_ADJ = 2,         // x = A^H y                                   -> tout
  M_ER = 3,          // t <- A^H(sqrt(I) y/|y|)/(K N)               -> tout, sums {amp_res, f}
  M_GRAD = 4,        // g = -4 A^H(y (I - |y|^2))                   -> tout, sums {f}
  M_SPEC = 5,        // heavy-ball power step on A^H diag(w) A      -> tout (v), vscale
  M_LS = 6,          // quartic line-search sums for y = A t, z = A d -> sums[6]
  M_RES64 = 7,       // FP64 residual: sums64 {sum r^2, sum I^2}
  M_BACKPROP = 8,    // x = A^H sqrt(I) / (K N)                     -> tout
  M_AGRAD = 9,       // g = -2 A^H((sqrt(I) - |y|) y/|y|)           -> tout, sums {f_a}
  M_ALS = 10,        // amplitude cost at t + a_j d, a_j = 2^(j-3), j < 8 -> sums {f_a(t), f_a(t + a_j d)}
  M_FILT = 11,       // x = A^H(H .* A t) / (K N), H = yin [N] in natural frequency order -> tout
  M_ERC = 12,        // for m = 1..K: t <- conj(psi_m) F^H(sqrt(I_m) y/|y|)/N, y = F(psi_m t) -> tout, sums
  M_LANCZOS = 13,    // Lanczos step on A^H diag(w) A: v_next = (M v - alpha v - beta v_prev)/||.|| -> tout, lz_out
  // learned weighting of the spectral start: w = T(I / mean(I_p)) from the table wtab
  M_LANCZOS_T = 14,  // M_LANCZOS with the weights read from I (the learned weights, FP32 [P][K][N])
  M_WAPPLY = 15,     // y = A^H diag(w) A t with the learned weights      -> tout, sums {||y||^2}
  M_WBACK = 16       // gw = Re(conj(A d) (A t)) -> yout float [P][K][N]; x = A^H diag(w) A d -> tout
};

// Modes that weight by the learned table (the row kernels look it up per measurement).
constexpr bool learned_mode(int m) { return m == M_WAPPLY || m == M_WBACK; }

constexpr int NSUM = 9;
constexpr int AMP_TRIALS = 8;  // M_ALS trial steps 1/8 .. 16

struct RowArgs {
  int P, K;
  const cx<float>* masks;  // [K][N]
  const cx<float>* tin;    // [P][N]
  const cx<float>* din;    // [P][N]  (M_LS: direction d; M_SPEC: previous v / vscale; M_ER: t_prev)
  const void* I;           // [P][K][N] float or bf16
  const cx<float>* yin;    // [P][K][N] (M_ADJ)
  cx<float>* tout;         // [P][N]
  float* vscale;           // [P] M_SPEC: scale of din (read), of the new previous iterate tin (written)
  void* yout;              // [P][K][N] (M_FWD_*)
  float* sums;             // [P][NSUM]
  double* sums64;          // [P][2] (M_RES64)
  const float* rowmean;    // [P] mean of I per row (M_SPEC)
  float tau;               // M_SPEC truncation
  float momentum;          // M_SPEC heavy-ball factor c
  float spec_lower;        // M_SPEC lower end l of the rest of the spectrum (fraction of lambda)
  float er_beta;           // M_ER Nesterov factor b: iterate from z = tin + b (tin - din), din = t_prev
  const float* lz_bprev;   // M_LANCZOS: previous step's [P][2] (alpha, beta); beta is this step's beta, or null
  float* lz_out;           // M_LANCZOS: [P][2] (alpha, ||x||) of this step
  // M_LANCZOS with lz_sum != null (the first step): the prologue forms each
  // row's intensity sum (FP64, into lz_sum [P]) and mean (into lz_mean [P],
  // used in place of rowmean), and scales the seed in tin to unit norm (FP64
  // norm), writing it back over tin
  double* lz_sum;
  float* lz_mean;
  const float* wtab;       // learned weights: [nt][2] (T(x_b), T(x_b+1) - T(x_b)), x_b = b / wtab_scale
  float wtab_scale;        // (nt - 1) / xmax
  float wtab_last;         // nt - 1
  int out_bf16;            // M_FWD_INT output type
  const cx<float>* tw32;   // twiddle tables, table of length L at offset L-1
  const cx<double>* tw64;
  // M_ERC with lz_k > 0: the row is the Ritz vector sum_j y_j v_j of a Lanczos
  // start, formed in the prologue (v_1 = tin, v_j = lz_basis + (j - 2) lz_rs
  // for j >= 2, y = lz_y [P][lz_k]); the projection does not depend on its scale
  const cx<float>* lz_basis;
  const double* lz_y;
  int lz_k;
  int64_t lz_rs;
  // M_LS / M_ALS with lb_sc != null: the L-BFGS direction is formed in the
  // prologue from the compact-form coefficients of the direction solve,
  //   d = cg g + sum_j (cs_j s_j + cy_j y_j)  over the row's stored pairs,
  // written to lb_d (and read back from there by the mask loop; din unused).
  // lb_S, lb_Y: [P][LB_SLOTS(lb_m)][N] rings; lb_sc: [P][LB_SCALARS(lb_m)]
  // with head, count at 0, 1 and the coefficients from 4 + 2 LB_SLOTS^2 on.
  const cx<float>* lb_g;
  const cx<float>* lb_S;
  const cx<float>* lb_Y;
  const double* lb_sc;
  cx<float>* lb_d;
  int lb_m;
};

__device__ __forceinline__ float bf16_to_f(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}



// Accesses through global-address-space pointers (complex values as 8-byte
// vectors; complex buffers are 8-byte aligned).
#define TM_GLOBAL __attribute__((address_space(1)))
typedef float tm_v2f __attribute__((ext_vector_type(2)));
template <typename V>
__device__ __forceinline__ const TM_GLOBAL V* gc(const V* p) { return (const TM_GLOBAL V*)p; }
template <typename V>
__device__ __forceinline__ TM_GLOBAL V* gw(V* p) { return (TM_GLOBAL V*)p; }
__device__ __forceinline__ cx<float> gload(const cx<float>* p) {
  tm_v2f v = *(const TM_GLOBAL tm_v2f*)p;
  return cx<float>{v.x, v.y};
}
__device__ __forceinline__ void gstore(cx<float>* p, cx<float> v) {
  *(TM_GLOBAL tm_v2f*)p = tm_v2f{v.x, v.y};
}

template <typename IT>
__device__ __forceinline__ float load_I(const void* I, size_t idx) {
  if constexpr (sizeof(IT) == 2) return bf16_to_f(gc((const uint16_t*)I)[idx]);
  else return gc((const float*)I)[idx];
}

// Compensated (TwoSum) accumulation in FP32.
struct KSum {
  float s, c;
  __device__ __forceinline__ void add(float v) {
    float t = s + v;
    float bp = t - s;
    float e = (s - (t - bp)) + (v - bp);
    s = t;
    c += e;
  }
  __device__ __forceinline__ void merge(float s2, float c2) {
    float t = s + s2;
    float bp = t - s;
    float e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c += c2 + e;
  }
};

// Reduce NS compensated sums over the T threads of a row group. `red` is LDS
// scratch of at least (WG/64) * NS * 2 floats. Result valid in every thread.
template <int T, int WG, int NS>
__device__ __forceinline__ void row_reduce(KSum* acc, float* red, int tid, float* out) {
  if constexpr (T <= 64) {
#pragma unroll
    for (int off = T / 2; off >= 1; off >>= 1) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        float s2 = __shfl_xor(acc[i].s, off, 64);
        float c2 = __shfl_xor(acc[i].c, off, 64);
        acc[i].merge(s2, c2);
      }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) out[i] = acc[i].s + acc[i].c;
  } else {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        float s2 = __shfl_xor(acc[i].s, off, 64);
        float c2 = __shfl_xor(acc[i].c, off, 64);
        acc[i].merge(s2, c2);
      }
    }
    constexpr int WPR = T / 64;  // waves per row
    int wave = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        red[(wave * NS + i) * 2 + 0] = acc[i].s;
        red[(wave * NS + i) * 2 + 1] = acc[i].c;
      }
    }
    __syncthreads();
    int w0 = (wave / WPR) * WPR;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      KSum a{red[(w0 * NS + i) * 2], red[(w0 * NS + i) * 2 + 1]};
      for (int w = 1; w < WPR; ++w) a.merge(red[((w0 + w) * NS + i) * 2], red[((w0 + w) * NS + i) * 2 + 1]);
      out[i] = a.s + a.c;
    }
  }
}

// Two FP64 sums over the T threads of a row group, through the float scratch
// of row_reduce (each double as two 32-bit halves). Result in every thread.
template <int T, int WG>
__device__ __forceinline__ void row_reduce64x2(double& u, double& v, float* red, int tid) {
  const int n = (T <= 64) ? T / 2 : 32;
#pragma unroll
  for (int off = n; off >= 1; off >>= 1) {
    u += __shfl_xor(u, off, 64);
    v += __shfl_xor(v, off, 64);
  }
  if constexpr (T > 64) {
    constexpr int WPR = T / 64;
    const int wave = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) {
      const uint64_t bu = (uint64_t)__double_as_longlong(u), bv = (uint64_t)__double_as_longlong(v);
      red[wave * 4 + 0] = __uint_as_float((uint32_t)bu);
      red[wave * 4 + 1] = __uint_as_float((uint32_t)(bu >> 32));
      red[wave * 4 + 2] = __uint_as_float((uint32_t)bv);
      red[wave * 4 + 3] = __uint_as_float((uint32_t)(bv >> 32));
    }
    __syncthreads();
    const int w0 = (wave / WPR) * WPR;
    double su = 0.0, sv = 0.0;
    for (int w = 0; w < WPR; ++w) {
      const float* q = red + (w0 + w) * 4;
      su += __longlong_as_double((long long)(((uint64_t)__float_as_uint(q[1]) << 32) | __float_as_uint(q[0])));
      sv += __longlong_as_double((long long)(((uint64_t)__float_as_uint(q[3]) << 32) | __float_as_uint(q[2])));
    }
    u = su;
    v = sv;
  }
}

template <int T, int WG>
__device__ __forceinline__ double row_reduce64(double v, double* red, int tid) {
  if constexpr (T <= 64) {
#pragma unroll
    for (int off = T / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  } else {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    constexpr int WPR = T / 64;
    int wave = tid >> 6;
    __syncthreads();
    if ((tid & 63) == 0) red[wave] = v;
    __syncthreads();
    int w0 = (wave / WPR) * WPR;
    double s = 0;
    for (int w = 0; w < WPR; ++w) s += red[w0 + w];
    return s;
  }
}

// Shape of one workgroup of WGT threads (default: one row of T threads, at
// least 256 threads).
template <class PL, int WGT = ((PL::T >= 256) ? PL::T : 256)>
struct Launch {
  static constexpr int WG = WGT;
  static constexpr int RPW = WG / PL::T;  // rows per workgroup
  // double-buffered LDS exchange when two copies of the rows fit in 160 KiB
  static constexpr bool DB = 2 * RPW * PL::LDS_ROW * 8 <= 160 * 1024 - 4096;
  static constexpr int LDS_ELEMS = (DB ? 2 : 1) * RPW * PL::LDS_ROW;
  static constexpr int RED_FLOATS = (WG / 64 + 1) * NSUM * 2;
};

// ---------------------------------------------------------------- FP32 kernel
// Hardware square root and reciprocal square root (about 1 ulp), without the
// range-scaling and refinement sequences of the IEEE-exact library calls.
__device__ __forceinline__ float hw_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hw_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Learned weight T(x) by linear interpolation in the table (x clamped to the
// table's range; NaN reads the first point).
__device__ __forceinline__ float wtab_eval(const RowArgs& a, float x) {
  const float s = fminf(fmaxf(x * a.wtab_scale, 0.f), a.wtab_last);
  const int i0 = min((int)s, (int)a.wtab_last - 1);
  const tm_v2f e = gc((const tm_v2f*)a.wtab)[i0];
  return e.x + (s - (float)i0) * e.y;
}

// SUMS: accumulate the per-row monitoring sums (compensated) and write them;
// without it the kernel skips that work (used on iterations whose sums are
// not read).
#ifndef TM_MINW
#define TM_MINW 1
#endif

// Body of the fused kernel for the rows [blk * RPW, (blk + 1) * RPW) of one
// problem, run by a workgroup of WGT threads with LDS at lds_all (at least
// Launch<PL, WGT>::LDS_ELEMS elements) and red (RED_FLOATS floats).
// OOL: the body is called out of line (the uneven batch). The cyclic ER step
// then issues each mask's values and intensities together before their first
// use: there the compiler otherwise loaded and waited for them one at a time
// (batch sweep over 12 problems 2.60 -> 1.65 ms), while in the inlined kernel
// the same order costs 5 % (its own schedule overlaps them already).
template <class PL, int MODE, typename IT, bool SUMS, int WGT, bool OOL = false>
__device__ __forceinline__ void row_body(const RowArgs& args, int blk, cx<float>* lds_all, float* red) {
  // Every buffer is in device global memory: the accesses below go through
  // global-address-space pointers, so that where this body is not inlined into
  // a kernel they stay global (not flat) loads and stores, which do not share
  // a wait counter with the LDS exchanges.
  const RowArgs a = args;
  using T = float;
  using C = cx<T>;
  using LC = Launch<PL, WGT>;
  constexpr int E = PL::E, N = PL::N, WG = LC::WG, RPW = LC::RPW;
  constexpr int NBUF = LC::DB ? 2 : 1;

  const int tid = threadIdx.x;
  const int rloc = tid / PL::T;
  const int ltid = tid % PL::T;
  const int row = blk * RPW + rloc;
  const bool valid = row < a.P;
  const size_t prow = valid ? (size_t)row : 0;
  Xbuf<T> xb{lds_all + rloc * PL::LDS_ROW, (NBUF == 2) ? RPW * PL::LDS_ROW : 0, 0};
  Tw<T> tw{a.tw32 + (PL::N1 - 1), a.tw32 + (PL::N2 - 1)};

  using L0 = Layout0<PL>;
  using LL = LayoutL<PL>;
  int b0[L0::NB];  // pass-0 butterfly bases (natural element index)
#pragma unroll
  for (int j = 0; j < L0::NB; ++j) b0[j] = L0::base(ltid, j);
  int kb[LL::NB];  // last-pass butterfly spectrum bases
#pragma unroll
  for (int j = 0; j < LL::NB; ++j) kb[j] = LL::kbase(ltid, j);
#define E0(i) (b0[(i) / L0::R] + ((i) % L0::R) * L0::HS)
#define KL(i) (kb[(i) / LL::R] + ((i) % LL::R) * LL::KS)

  // The row t is held in registers across the mask loop (re-reading it per
  // mask from cache measured slower); d (M_LS) is re-read per mask.
  C g[E], x[E];
  const C* trow = a.tin + prow * N;
  const C* drow = a.din + prow * N;
  C treg[E];
  if constexpr (MODE != M_ADJ && MODE != M_BACKPROP) {
#pragma unroll
    for (int i = 0; i < E; ++i) treg[i] = gload(trow + E0(i));
  }
  float lz_mean0 = 1.f;  // the row's mean intensity when this (first Lanczos) step forms it
  if constexpr (MODE == M_LANCZOS) {
    if (a.lz_sum) {
      // seed norm and intensity sum in FP64; the intensities read along the
      // row (consecutive threads, consecutive values), mask by mask
      double sn = 0.0, si = 0.0;
#pragma unroll
      for (int i = 0; i < E; ++i)
        sn += fmadd((double)treg[i].x, (double)treg[i].x, (double)treg[i].y * (double)treg[i].y);
      const size_t ib = prow * (size_t)a.K * N;
      for (int m = 0; m < a.K; ++m) {
        float iv[E];
#pragma unroll
        for (int i = 0; i < E; ++i) iv[i] = load_I<IT>(a.I, ib + (size_t)m * N + i * PL::T + ltid);
#pragma unroll
        for (int i = 0; i < E; ++i) si += (double)iv[i];
      }
      row_reduce64x2<PL::T, WG>(sn, si, red, tid);
      const float f = (float)((sn > 0.0) ? 1.0 / sqrt(sn) : 1.0);
#pragma unroll
      for (int i = 0; i < E; ++i) treg[i] = scl(treg[i], f);
      lz_mean0 = (float)(si / (double)((size_t)a.K * N));
      if (valid) {
        C* t1 = const_cast<C*>(trow);
#pragma unroll
        for (int i = 0; i < E; ++i) gstore(t1 + E0(i), treg[i]);
        if (ltid == 0) {
          gw(a.lz_sum)[prow] = si;
          gw(a.lz_mean)[prow] = lz_mean0;
        }
      }
    }
  }
  if constexpr (MODE == M_LS || MODE == M_ALS) {
    if (a.lb_sc) {
      // the L-BFGS direction at this thread's values, two stored pairs' loads in
      // flight at a time; each thread later reads back only what it wrote here
      const int R = LB_SLOTS(a.lb_m);
      const double* sc = a.lb_sc + prow * (size_t)LB_SCALARS(a.lb_m);
      const int head = (int)sc[0], count = (int)sc[1];
      const double* coef = sc + 4 + 2 * R * R;
      const float cg = (float)coef[0];
      C dv[E];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const C gv = gload(a.lb_g + prow * N + E0(i));
        dv[i] = C{cg * gv.x, cg * gv.y};
      }
      for (int j = 0; j < count; j += 2) {
        const bool two = j + 1 < count;
        const size_t s0 = ((size_t)prow * R + (head - count + j + 2 * R) % R) * N;
        const size_t s1 = ((size_t)prow * R + (head - count + j + 1 + 2 * R) % R) * N;
        C sv0[E], yv0[E], sv1[E], yv1[E];
#pragma unroll
        for (int i = 0; i < E; ++i) {
          sv0[i] = gload(a.lb_S + s0 + E0(i));
          yv0[i] = gload(a.lb_Y + s0 + E0(i));
          sv1[i] = two ? gload(a.lb_S + s1 + E0(i)) : C{0.f, 0.f};
          yv1[i] = two ? gload(a.lb_Y + s1 + E0(i)) : C{0.f, 0.f};
        }
        const float cs0 = (float)coef[1 + j], cy0 = (float)coef[1 + R + j];
        const float cs1 = two ? (float)coef[2 + j] : 0.f, cy1 = two ? (float)coef[2 + R + j] : 0.f;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          dv[i].x = fmadd(cy0, yv0[i].x, fmadd(cs0, sv0[i].x, dv[i].x));
          dv[i].y = fmadd(cy0, yv0[i].y, fmadd(cs0, sv0[i].y, dv[i].y));
          if (two) {
            dv[i].x = fmadd(cy1, yv1[i].x, fmadd(cs1, sv1[i].x, dv[i].x));
            dv[i].y = fmadd(cy1, yv1[i].y, fmadd(cs1, sv1[i].y, dv[i].y));
          }
        }
      }
      C* dout = a.lb_d + prow * N;
      if (valid) {
#pragma unroll
        for (int i = 0; i < E; ++i) gstore(dout + E0(i), dv[i]);
      }
      drow = dout;
    }
  }
  if constexpr (MODE == M_ER) {
    if (a.er_beta != 0.f) {
      // Nesterov extrapolation from the previous iterate. The caller swaps the
      // two buffers every iteration (tout = din), so t is never copied, and no
      // store precedes the FFTs (the twiddle tables stay scalar loads).
      const float b = a.er_beta;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        C tp = gload(drow + E0(i));
        treg[i] = C{treg[i].x + b * (treg[i].x - tp.x), treg[i].y + b * (treg[i].y - tp.y)};
      }
    }
  }
  if constexpr (MODE == M_ERC) {
    if (a.lz_k > 0) {
      // t = sum_j y_j v_j with FP64 sums in basis order (the same sums as the
      // separate combination kernel), v_1 already in registers
      const double* yp = a.lz_y + prow * a.lz_k;
      double ax[E], ay[E];
      const double w0 = yp[0];
#pragma unroll
      for (int i = 0; i < E; ++i) {
        ax[i] = w0 * treg[i].x;
        ay[i] = w0 * treg[i].y;
      }
      // one basis row at a time (groups of rows in flight measured no faster: one
      // workgroup per CU, so these loads do not overlap the transforms either way)
      for (int j = 1; j < a.lz_k; ++j) {
        const C* vr = a.lz_basis + (size_t)(j - 1) * a.lz_rs + prow * N;
        const double w = yp[j];
        C v[E];
#pragma unroll
        for (int i = 0; i < E; ++i) v[i] = gload(vr + E0(i));
#pragma unroll
        for (int i = 0; i < E; ++i) {
          ax[i] += w * v[i].x;
          ay[i] += w * v[i].y;
        }
      }
#pragma unroll
      for (int i = 0; i < E; ++i) treg[i] = C{(float)ax[i], (float)ay[i]};
    }
  }
#define TROW(i) treg[i]
#pragma unroll
  for (int i = 0; i < E; ++i) g[i] = C{0.f, 0.f};

  KSum acc[NSUM];
#pragma unroll
  for (int i = 0; i < NSUM; ++i) acc[i] = KSum{0.f, 0.f};

  float inv_mean = 0.f;
  if constexpr (MODE == M_SPEC || MODE == M_LANCZOS || learned_mode(MODE)) {
    float m = 1.f;
    if (MODE == M_LANCZOS && a.lz_sum) m = lz_mean0;
    else if (valid) m = gc(a.rowmean)[prow];
    inv_mean = (m > 0.f) ? 1.f / m : 1.f;
  }

  // Global-load latency in the spectral and Lanczos steps: the next mask's
  // values are loaded during the last radix pass of the inverse transform (the
  // first mask's before the loop) and kept for the conjugate multiply, and each
  // mask's intensity loads are issued before its forward transform, so that
  // they are in flight during it (Lanczos step 0.394 -> 0.360 ms at
  // 2286 x 8192). The ER and gradient steps load the mask twice and the
  // intensities after the transform: the same changes measured slower there
  // (cyclic ER 0.357 -> 0.376 and 0.413 ms).
  constexpr bool PF = MODE == M_SPEC || MODE == M_LANCZOS || MODE == M_LANCZOS_T || MODE == M_WAPPLY;
  float icur[PF ? E : 1];
  C mv[PF ? E : 1];     // the mask's values, kept for the conjugate multiply
  C mnext[PF ? E : 1];  // the next mask's values, loaded during the last inverse pass
  if constexpr (PF) {
#pragma unroll
    for (int i = 0; i < E; ++i) mnext[i] = gload(a.masks + E0(i));
  }
  for (int m = 0; m < a.K; ++m) {
    const C* mk = a.masks + (size_t)m * N;
    const size_t mbase = (prow * a.K + m) * (size_t)N;
    if constexpr (MODE == M_ADJ || MODE == M_BACKPROP) {
      // spectrum arrives in natural order; place it at the digit-reversed slots
#pragma unroll
      for (int i = 0; i < E; ++i) {
        int k = KL(i);
        if constexpr (MODE == M_ADJ) x[i] = gload(a.yin + mbase + k);
        else x[i] = C{sqrtf(fmaxf(load_I<IT>(a.I, mbase + k), 0.f)), 0.f};
      }
    } else {
      if constexpr (PF) {
        // the intensity loads go out after the (earlier) mask loads, so the
        // wait for the mask values leaves them in flight under the forward
        // transform; the scheduling barriers keep that order
#pragma unroll
        for (int i = 0; i < E; ++i) mv[i] = mnext[i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < E; ++i) icur[i] = load_I<IT>(a.I, mbase + KL(i));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = cmul(TROW(i), mv[i]);
      } else if constexpr (MODE == M_ERC && OOL) {
        C mvals[E];
#pragma unroll
        for (int i = 0; i < E; ++i) mvals[i] = gload(mk + E0(i));
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = cmul(TROW(i), mvals[i]);
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = cmul(TROW(i), gload(mk + E0(i)));
      }
      fft_forward<PL, T>(x, xb, ltid, tw);
    }

    if constexpr (MODE == M_FWD_FIELD || MODE == M_FWD_INT) {
      if (valid) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          int k = KL(i);
          if constexpr (MODE == M_FWD_FIELD) gstore((C*)a.yout + mbase + k, x[i]);
          else {
            float v = norm2(x[i]);
            if (a.out_bf16) gw((uint16_t*)a.yout)[mbase + k] = f_to_bf16(v);
            else gw((float*)a.yout)[mbase + k] = v;
          }
        }
      }
      continue;
    } else if constexpr (MODE == M_ALS) {
      // f_a(t + a d) = sum (sqrt(I) - |y + a z|)^2 at a = 0 and the trial steps
      C y[E];
#pragma unroll
      for (int i = 0; i < E; ++i) y[i] = x[i];
#pragma unroll
      for (int i = 0; i < E; ++i) x[i] = cmul(gload(drow + E0(i)), gload(mk + E0(i)));
      fft_forward<PL, T>(x, xb, ltid, tw);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        int k = KL(i);
        const float amp = hw_sqrt(fmaxf(load_I<IT>(a.I, mbase + k), 0.f));
        const float r0 = amp - hw_sqrt(norm2(y[i]));
        acc[0].add(r0 * r0);
#pragma unroll
        for (int j = 0; j < AMP_TRIALS; ++j) {
          const float st = ldexpf(1.f, j - 3);
          const C w = C{y[i].x + st * x[i].x, y[i].y + st * x[i].y};
          const float r = amp - hw_sqrt(norm2(w));
          acc[1 + j].add(r * r);
        }
      }
      continue;
    } else if constexpr (MODE == M_LS) {
      C y[E];
#pragma unroll
      for (int i = 0; i < E; ++i) y[i] = x[i];
#pragma unroll
      for (int i = 0; i < E; ++i) x[i] = cmul(gload(drow + E0(i)), gload(mk + E0(i)));
      fft_forward<PL, T>(x, xb, ltid, tw);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        int k = KL(i);
        float iv = load_I<IT>(a.I, mbase + k);
        float r = iv - norm2(y[i]);
        float b = y[i].x * x[i].x + y[i].y * x[i].y;
        float c = norm2(x[i]);
        acc[0].add(r * r);
        acc[1].add(r * b);
        acc[2].add(b * b);
        acc[3].add(r * c);
        acc[4].add(b * c);
        acc[5].add(c * c);
      }
      continue;
    } else {
      if constexpr (MODE == M_FILT) {
        // multiply the spectrum by the filter (read at each slot's natural frequency)
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = cmul(x[i], gload(a.yin + KL(i)));
      }
      if constexpr (MODE == M_WBACK) {
        // second transform z = A d of this mask; gw = Re(conj(z) y) at each
        // measurement (natural order); then the weighted z goes back
        C y[E];
#pragma unroll
        for (int i = 0; i < E; ++i) y[i] = x[i];
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = cmul(gload(drow + E0(i)), gload(mk + E0(i)));
        fft_forward<PL, T>(x, xb, ltid, tw);
#pragma unroll
        for (int i = 0; i < E; ++i) {
          const int k = KL(i);
          const float w = wtab_eval(a, load_I<IT>(a.I, mbase + k) * inv_mean);
          if (valid) gw((float*)a.yout)[mbase + k] = y[i].x * x[i].x + y[i].y * x[i].y;
          x[i] = scl(x[i], w);
        }
      }
      if constexpr (MODE == M_ER || MODE == M_ERC || MODE == M_GRAD || MODE == M_SPEC || MODE == M_LANCZOS ||
                    MODE == M_AGRAD || MODE == M_LANCZOS_T || MODE == M_WAPPLY) {
        float ierc[MODE == M_ERC && OOL ? E : 1];  // the intensities loaded together (OOL)
        if constexpr (MODE == M_ERC && OOL) {
#pragma unroll
          for (int i = 0; i < E; ++i) ierc[i] = load_I<IT>(a.I, mbase + KL(i));
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = 0; i < E; ++i) {
          float iv;
          if constexpr (PF) iv = icur[i];
          else if constexpr (MODE == M_ERC && OOL) iv = ierc[i];
          else iv = load_I<IT>(a.I, mbase + KL(i));
          float n = norm2(x[i]);
          if constexpr (MODE == M_ER || MODE == M_ERC) {
            // keep the measured amplitude, keep the phase (y/|y| := 1 at y = 0)
            float amp = hw_sqrt(fmaxf(iv, 0.f));
            float rs = hw_rsq(n);
            bool nz = n > 0.f;
            float sc = nz ? amp * rs : 0.f;
            C w = scl(x[i], sc);
            if constexpr (SUMS) {
              float mag = n * rs;
              float dr = amp - (nz ? mag : 0.f), ri = iv - n;
              acc[0].add(dr * dr);
              acc[1].add(ri * ri);
            }
            x[i] = nz ? w : C{amp, 0.f};
          } else if constexpr (MODE == M_GRAD) {
            float r = iv - n;
            if constexpr (SUMS) acc[0].add(r * r);
            x[i] = scl(x[i], r);
          } else if constexpr (MODE == M_AGRAD) {
            // -2 (sqrt(I) - |y|) y/|y|, with y/|y| := 1 at y = 0
            float amp = hw_sqrt(fmaxf(iv, 0.f));
            float rs = hw_rsq(n);
            bool nz = n > 0.f;
            float r = amp - (nz ? n * rs : 0.f);
            if constexpr (SUMS) acc[0].add(r * r);
            x[i] = nz ? scl(x[i], -2.f * r * rs) : C{-2.f * r, 0.f};
          } else if constexpr (learned_mode(MODE)) {
            x[i] = scl(x[i], wtab_eval(a, iv * inv_mean));
          } else if constexpr (MODE == M_LANCZOS_T) {
            x[i] = scl(x[i], iv);  // the weight itself, evaluated once per retrieval
          } else {
            float w = fminf(iv * inv_mean, a.tau);
            x[i] = scl(x[i], w);
          }
        }
      }
      if constexpr (PF) {
        const C* mk1 = mk + N;
        const bool more = m + 1 < a.K;
        fft_inverse<PL, T>(x, xb, ltid, tw, [&]() {
          if (more) {
#pragma unroll
            for (int i = 0; i < E; ++i) mnext[i] = gload(mk1 + E0(i));
          }
        });
      } else {
        fft_inverse<PL, T>(x, xb, ltid, tw);
      }
      if constexpr (MODE == M_ERC) {
        // this mask's projection replaces the row before the next mask
        const float inv_n = 1.f / (float)N;
        if constexpr (OOL) {
#pragma unroll
          for (int i = 0; i < E; ++i) g[i] = gload(mk + E0(i));  // g is free in this mode: the mask values
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int i = 0; i < E; ++i) treg[i] = scl(cmulc(x[i], g[i]), inv_n);
        } else {
#pragma unroll
          for (int i = 0; i < E; ++i) treg[i] = scl(cmulc(x[i], gload(mk + E0(i))), inv_n);
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          if constexpr (PF) g[i] = g[i] + cmulc(x[i], mv[i]);
          else g[i] = g[i] + cmulc(x[i], gload(mk + E0(i)));
        }
      }
    }
  }

  if constexpr (MODE == M_FWD_FIELD || MODE == M_FWD_INT) {
    return;
  } else if constexpr (MODE == M_LS || MODE == M_ALS) {
    constexpr int NS = (MODE == M_LS) ? 6 : 1 + AMP_TRIALS;
    float out[NS];
    row_reduce<PL::T, WG, NS>(acc, red, tid, out);
    if (valid && ltid == 0) {
#pragma unroll
      for (int i = 0; i < NS; ++i) gw(a.sums)[prow * NSUM + i] = out[i];
    }
  } else if constexpr (MODE == M_LANCZOS || MODE == M_LANCZOS_T) {
    // alpha = Re <v, M v>; x = M v - alpha v - beta v_prev with beta = ||x|| of the
    // previous step (0 at the first, where there is no v_prev); v_next = x / ||x||.
    // ||x|| is summed from x itself (a second reduction), not expanded.
    KSum q[1];
    q[0] = KSum{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < E; ++i) q[0].add(TROW(i).x * g[i].x + TROW(i).y * g[i].y);
    float o1[1];
    row_reduce<PL::T, WG, 1>(q, red, tid, o1);
    const float al = o1[0];
    if (a.lz_bprev) {
      const float bp = valid ? gc(a.lz_bprev)[prow * 2 + 1] : 0.f;
#pragma unroll
      for (int i = 0; i < E; ++i) g[i] = g[i] - scl(TROW(i), al) - scl(gload(drow + E0(i)), bp);
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) g[i] = g[i] - scl(TROW(i), al);
    }
    q[0] = KSum{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < E; ++i) q[0].add(norm2(g[i]));
    float o2[1];
    row_reduce<PL::T, WG, 1>(q, red, tid, o2);
    const float nrm = sqrtf(fmaxf(o2[0], 0.f));
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    if (valid) {
#pragma unroll
      for (int i = 0; i < E; ++i) gstore(a.tout + prow * N + E0(i), scl(g[i], inv));
      if (ltid == 0) {
        gw(a.lz_out)[prow * 2 + 0] = al;
        gw(a.lz_out)[prow * 2 + 1] = nrm;
      }
    }
  } else if constexpr (MODE == M_SPEC) {
    // lambda = Re <v, M v> (v has unit norm); x = (M - sigma) v - beta v_prev
    // with sigma = (c + l) lambda / 2, beta = ((c - l) lambda / 2)^2 / 4;
    // v <- x / ||x|| and v_prev <- v / ||x||. v_prev is held as u (din) times
    // the per-row scale s, and the caller swaps the two row buffers every
    // step, so the step writes only x / ||x|| (over u) and the new scale.
    // ||x||^2 expands in sums that come out of the same single reduction as
    // lambda (b = beta s):
    //   |g|^2 + sigma^2 |v|^2 + b^2 |u|^2 - 2 sigma lambda - 2 b Re<u, g> + 2 sigma b Re<u, v>.
    const float sp = valid ? gc(a.vscale)[prow] : 0.f;
    C vp[E];
#pragma unroll
    for (int i = 0; i < E; ++i) vp[i] = gload(drow + E0(i));
    KSum q[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) q[i] = KSum{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < E; ++i) {
      C ti = TROW(i);
      q[0].add(ti.x * g[i].x + ti.y * g[i].y);
      q[1].add(norm2(g[i]));
      q[2].add(vp[i].x * g[i].x + vp[i].y * g[i].y);
      q[3].add(norm2(vp[i]));
      q[4].add(norm2(ti));
      q[5].add(vp[i].x * ti.x + vp[i].y * ti.y);
    }
    float out[6];
    row_reduce<PL::T, WG, 6>(q, red, tid, out);
    const float lam = out[0];
    const float sig = 0.5f * (a.momentum + a.spec_lower) * lam;
    const float rad = 0.5f * (a.momentum - a.spec_lower) * lam;
    const float bs = 0.25f * rad * rad * sp;  // beta s
    const float nn = fmaxf(out[1] + sig * sig * out[4] + bs * bs * out[3] - 2.f * sig * lam - 2.f * bs * out[2] +
                               2.f * sig * bs * out[5],
                           0.f);
    const float inv = (nn > 0.f) ? rsqrtf(nn) : 1.f;
    if (valid) {
#pragma unroll
      for (int i = 0; i < E; ++i)
        gstore(a.tout + prow * N + E0(i), scl(g[i] - scl(TROW(i), sig) - scl(vp[i], bs), inv));
      if (ltid == 0) {
        gw(a.vscale)[prow] = inv;
        if (a.sums) gw(a.sums)[prow * NSUM + 0] = lam;
      }
    }
  } else if constexpr (MODE == M_WAPPLY) {
    KSum q[1];
    q[0] = KSum{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < E; ++i) q[0].add(norm2(g[i]));
    float o1[1];
    row_reduce<PL::T, WG, 1>(q, red, tid, o1);
    if (valid) {
#pragma unroll
      for (int i = 0; i < E; ++i) gstore(a.tout + prow * N + E0(i), g[i]);
      if (ltid == 0) gw(a.sums)[prow * NSUM + 0] = o1[0];
    }
  } else {
    float scale = 1.f;
    if constexpr (MODE == M_ER || MODE == M_BACKPROP || MODE == M_FILT) scale = 1.f / (float)(a.K * N);
    if constexpr (MODE == M_GRAD) scale = -4.f;
    if (valid) {
      if constexpr (MODE == M_ERC) {
#pragma unroll
        for (int i = 0; i < E; ++i) gstore(a.tout + prow * N + E0(i), treg[i]);
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) gstore(a.tout + prow * N + E0(i), scl(g[i], scale));
      }
    }
    if constexpr ((MODE == M_ER || MODE == M_ERC || MODE == M_GRAD || MODE == M_AGRAD) && SUMS) {
      float out[NSUM];
      row_reduce<PL::T, WG, (MODE == M_ER || MODE == M_ERC) ? 2 : 1>(acc, red, tid, out);
      if (valid && ltid == 0 && a.sums) {
        if constexpr (MODE == M_ER || MODE == M_ERC) {
          gw(a.sums)[prow * NSUM + 0] = out[0];
          gw(a.sums)[prow * NSUM + 1] = out[1];
        } else {
          gw(a.sums)[prow * NSUM + 0] = out[0];
        }
      }
    }
  }
}

template <class PL, int MODE, typename IT, bool SUMS = true>
__global__ void __launch_bounds__(Launch<PL>::WG) __attribute__((amdgpu_waves_per_eu(TM_MINW)))
row_kernel(RowArgs a) {
  __shared__ cx<float> lds_all[Launch<PL>::LDS_ELEMS];
  __shared__ float red[Launch<PL>::RED_FLOATS];
  row_body<PL, MODE, IT, SUMS, Launch<PL>::WG>(a, blockIdx.x, lds_all, red);
}

// The same kernel with an explicit workgroup size WGT (WGT / T rows per
// workgroup): the autotuner's wider configurations.
template <class PL, int MODE, typename IT, bool SUMS, int WGT>
__global__ void __launch_bounds__(WGT) __attribute__((amdgpu_waves_per_eu(TM_MINW)))
row_kernel_w(RowArgs a) {
  __shared__ cx<float> lds_all[Launch<PL, WGT>::LDS_ELEMS];
  __shared__ float red[Launch<PL, WGT>::RED_FLOATS];
  row_body<PL, MODE, IT, SUMS, WGT>(a, blockIdx.x, lds_all, red);
}

// ---------------------------------------------------------------- FP64 residual
template <class PL, typename IT>
__global__ void __launch_bounds__(Launch<PL>::WG)
res64_kernel(RowArgs a) {
  using T = double;
  using C = cx<T>;
  constexpr int E = PL::E, N = PL::N, WG = Launch<PL>::WG, RPW = Launch<PL>::RPW;
  extern __shared__ char dyn_lds[];
  C* lds_all = (C*)dyn_lds;
  double* red = (double*)(lds_all + RPW * PL::LDS_ROW);

  const int tid = threadIdx.x;
  const int rloc = tid / PL::T;
  const int ltid = tid % PL::T;
  const int row = blockIdx.x * RPW + rloc;
  const bool valid = row < a.P;
  const size_t prow = valid ? (size_t)row : 0;
  Xbuf<T> xb{lds_all + rloc * PL::LDS_ROW, 0, 0};
  Tw<T> tw{a.tw64 + (PL::N1 - 1), a.tw64 + (PL::N2 - 1)};

  using L0 = Layout0<PL>;
  using LL = LayoutL<PL>;
  int b0[L0::NB];
#pragma unroll
  for (int j = 0; j < L0::NB; ++j) b0[j] = L0::base(ltid, j);
  int kb[LL::NB];
#pragma unroll
  for (int j = 0; j < LL::NB; ++j) kb[j] = LL::kbase(ltid, j);
  C t[E], x[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    cx<float> v = a.tin[prow * N + E0(i)];
    t[i] = C{(double)v.x, (double)v.y};
  }
  double sr = 0.0, si = 0.0;
  for (int m = 0; m < a.K; ++m) {
    const cx<float>* mk = a.masks + (size_t)m * N;
    const size_t mbase = (prow * a.K + m) * (size_t)N;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      cx<float> w = mk[E0(i)];
      x[i] = cmul(t[i], C{(double)w.x, (double)w.y});
    }
    fft_forward<PL, T>(x, xb, ltid, tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      int k = KL(i);
      double iv = (double)load_I<IT>(a.I, mbase + k);
      double r = iv - norm2(x[i]);
      sr += r * r;
      si += iv * iv;
    }
  }
  sr = row_reduce64<PL::T, WG>(sr, red, tid);
  si = row_reduce64<PL::T, WG>(si, red, tid);
  if (valid && ltid == 0) {
    a.sums64[prow * 2 + 0] = sr;
    a.sums64[prow * 2 + 1] = si;
  }
}

#undef E0
#undef KL
#undef TROW
}  // namespace tmk
