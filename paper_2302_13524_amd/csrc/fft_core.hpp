// Row-resident batched 2-D FFT machinery for gfx950.
//
// One row (N = n1*n2 complex values, n1, n2 powers of two) is owned by a
// group of T = N/E threads; each thread holds E values in registers. A
// transform is a sequence of in-place radix passes (Cooley-Tukey, decimation
// in frequency for the forward DFT), each pass transforming one mixed-radix
// digit of one grid axis. Between passes the row goes through LDS once
// (write, barrier, read). The forward DFT leaves the spectrum in
// digit-reversed slots; the adjoint runs the passes in reverse order
// (decimation in time), so it consumes that order and returns natural
// order. Nothing is ever bit-reversed: the pointwise step reads the
// measurement at the digit-reversed frequency of each slot instead.
//
// Pass order: the highest digit of axis 1 (slow axis, stride n2) first,
// then the digits of axis 2 (fast axis), then the remaining axis-1 digits.
// With lanes mapped to consecutive i2 on axis-1 passes, the first pass
// (where the row is loaded from HBM) and the last forward pass (where the
// intensities are read) touch contiguous memory per wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmk {

// ------------------------------------------------------------------ complex
template <typename T>
struct cx {
  T x, y;
};
template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// The sums of two products name the product that is fused: left to the
// compiler, the choice can follow where the code sits (an inlined kernel and
// the same body called out of line rounded differently).
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {fmadd(a.x, b.x, -(a.y * b.y)), fmadd(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {fmadd(a.x, b.x, a.y * b.y), fmadd(a.y, b.x, -(a.x * b.y))};
}
template <typename T>
__device__ __forceinline__ cx<T> scl(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -j (forward) or +j (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cx<T> mulmj(cx<T> a) {
  if constexpr (INV) return {-a.y, a.x};
  else return {a.y, -a.x};
}
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return fmadd(a.x, a.x, a.y * a.y); }

// ------------------------------------------------------- small DFT kernels
// In place, natural order in and out. Forward: V[k] = sum v[h] W^{hk},
// W = exp(-2 pi j / R); INV uses W^{-1}. Unnormalised.
template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = t + b;
  b = t - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> s0 = a0 + a2, d0 = a0 - a2;
  cx<T> s1 = a1 + a3, d1 = mulmj<T, INV>(a1 - a3);
  a0 = s0 + s1;
  a2 = s0 - s1;
  a1 = d0 + d1;
  a3 = d0 - d1;
}

// W_8^k multipliers (k = 1, 2, 3) for the forward (INV=false) direction.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> w8_1(cx<T> a) {
  const T r = T(0.70710678118654752440);
  // forward: (1 - j)/sqrt2 ; inverse: (1 + j)/sqrt2
  if constexpr (INV) return {r * (a.x - a.y), r * (a.x + a.y)};
  else return {r * (a.x + a.y), r * (a.y - a.x)};
}
template <typename T, bool INV>
__device__ __forceinline__ cx<T> w8_3(cx<T> a) {
  const T r = T(0.70710678118654752440);
  // forward: (-1 - j)/sqrt2 ; inverse: (-1 + j)/sqrt2
  if constexpr (INV) return {-r * (a.x + a.y), r * (a.x - a.y)};
  else return {r * (a.y - a.x), -r * (a.x + a.y)};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // DIF 8 = 2 x 4: first radix-2 over the high bit, twiddle W_8^{l k}, then radix-4.
  cx<T> a0 = v[0] + v[4], b0 = v[0] - v[4];
  cx<T> a1 = v[1] + v[5], b1 = v[1] - v[5];
  cx<T> a2 = v[2] + v[6], b2 = v[2] - v[6];
  cx<T> a3 = v[3] + v[7], b3 = v[3] - v[7];
  b1 = w8_1<T, INV>(b1);
  b2 = mulmj<T, INV>(b2);
  b3 = w8_3<T, INV>(b3);
  dft4<T, INV>(a0, a1, a2, a3);  // even outputs: X[2k]
  dft4<T, INV>(b0, b1, b2, b3);  // odd outputs:  X[2k+1]
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

template <typename T, bool INV>
__device__ __forceinline__ cx<T> w16(cx<T> a, int e) {
  // multiply by W_16^e (forward) or W_16^{-e} (inverse), e in 0..9 compile-time
  const T c = T(0.92387953251128675613);   // cos(pi/8)
  const T s = T(0.38268343236508977173);   // sin(pi/8)
  const T r = T(0.70710678118654752440);
  cx<T> w;
  switch (e) {
    case 0: return a;
    case 1: w = {c, -s}; break;
    case 2: w = {r, -r}; break;
    case 3: w = {s, -c}; break;
    case 4: return mulmj<T, INV>(a);
    case 6: w = {-r, -r}; break;
    case 9: w = {-c, s}; break;
    default: w = {T(1), T(0)}; break;
  }
  if constexpr (INV) w.y = -w.y;
  return cmul(a, w);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // DIF 16 = 4 x 4: for each l in [0,4): radix-4 over h (v[4h + l]) -> k1,
  // twiddle W_16^{l k1}, then for each k1 a radix-4 over l -> k2; X[k1 + 4 k2].
  cx<T> u[16];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    cx<T> a0 = v[l], a1 = v[4 + l], a2 = v[8 + l], a3 = v[12 + l];
    dft4<T, INV>(a0, a1, a2, a3);
    u[0 * 4 + l] = a0;
    u[1 * 4 + l] = w16<T, INV>(a1, l);
    u[2 * 4 + l] = w16<T, INV>(a2, 2 * l);
    u[3 * 4 + l] = w16<T, INV>(a3, 3 * l);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> a0 = u[k1 * 4 + 0], a1 = u[k1 * 4 + 1], a2 = u[k1 * 4 + 2], a3 = u[k1 * 4 + 3];
    dft4<T, INV>(a0, a1, a2, a3);
    v[k1 + 0] = a0;
    v[k1 + 4] = a1;
    v[k1 + 8] = a2;
    v[k1 + 12] = a3;
  }
}

template <int R, typename T, bool INV>
__device__ __forceinline__ void dftR(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v[0], v[1]);
  else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 16) dft16<T, INV>(v);
  else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "radix");
}

// ------------------------------------------------------------------ plans
struct PassDesc {
  int axis;  // 1: slow axis (length n1, element stride n2); 2: fast axis
  int lr;    // log2 radix
  int lb;    // log2 block size B (sub-transform length at this pass)
};

struct PlanDesc {
  int np;
  PassDesc p[8];
};

// digits (log2 radices) of a length 2^b axis, most significant first, each
// of at most mb bits (a thread holds a whole radix-2^mb butterfly)
constexpr int ndigits(int b, int mb = 4) { return b == 0 ? 0 : (b + mb - 1) / mb; }
// Split b bits into ndigits(b, mb) digits of 1..mb bits; variant 0 puts the
// larger digits first (most significant), variant 1 the smaller ones.
constexpr int digit_bits(int b, int i, int var = 0, int mb = 4) {
  int n = ndigits(b, mb);
  int base = b / n, extra = b % n;
  int j = var ? (n - 1 - i) : i;
  return base + (j < extra ? 1 : 0);
}

constexpr PlanDesc make_plan(int L1, int L2, int var, int mb = 4) {
  PlanDesc d{};
  d.np = 0;
  int n1d = ndigits(L1, mb), n2d = ndigits(L2, mb);
  int lb1 = L1, lb2 = L2;
  auto push = [&](int axis, int bits) {
    int& lb = (axis == 1) ? lb1 : lb2;
    d.p[d.np].axis = axis;
    d.p[d.np].lr = bits;
    d.p[d.np].lb = lb;
    lb -= bits;
    d.np++;
  };
  int i1 = 0;
  if (n1d >= 2) { push(1, digit_bits(L1, 0, var, mb)); i1 = 1; }
  for (int i = 0; i < n2d; ++i) push(2, digit_bits(L2, i, var, mb));
  for (int i = i1; i < n1d; ++i) push(1, digit_bits(L1, i, var, mb));
  return d;
}

// Values per thread: 16 (LE_ forces another value).
constexpr int default_le(int ln) { return ln >= 4 ? 4 : ln; }

// VAR_ selects the digit order (see digit_bits); the autotuner picks it per grid.
template <int L1_, int L2_, int LE_ = -1, int VAR_ = 0>
struct Plan {
  static constexpr int VAR = VAR_;
  static constexpr int L1 = L1_, L2 = L2_;
  static constexpr int LN = L1 + L2;
  static constexpr int N1 = 1 << L1, N2 = 1 << L2, N = 1 << LN;
  static constexpr int LE = (LE_ >= 0) ? LE_ : default_le(LN);
  static constexpr int MB = LE < 4 ? (LE > 0 ? LE : 1) : 4;  // largest digit, bits
  static constexpr int E = 1 << LE;
  static constexpr int LT = LN - LE;
  static constexpr int T = 1 << LT;  // threads per row
  static constexpr PlanDesc desc = make_plan(L1, L2, VAR_, MB);
  static constexpr int NP = desc.np;
  // LDS: row-major grid with one pad slot after every n2 slots (n2 >= 16)
  static constexpr int PADSH = (L2 >= 4) ? L2 : 30;
  static constexpr int LDS_ROW = N + ((L2 >= 4) ? N1 : 0);
  static __device__ __forceinline__ int lds_addr(int e) { return e + (e >> PADSH); }
};

// Element index of value h of the j-th butterfly a thread executes in pass p.
// ltid: thread index within the row group.
template <class PL, int P>
struct PassGeo {
  static constexpr PassDesc d = PL::desc.p[P];
  static constexpr int LR = d.lr, R = 1 << LR;
  static constexpr int LB = d.lb, B = 1 << LB;
  static constexpr int LS = LB - LR, S = 1 << LS;  // stride between the R values
  static constexpr int NB = PL::E / R;             // butterflies per thread
  static constexpr int AXIS = d.axis;
  static constexpr int LA = (AXIS == 1) ? PL::L1 : PL::L2;  // log2 axis length

  // butterfly coordinates: (l in [0,S), blk in [0, 2^LA / B), other axis coordinate o)
  struct BF {
    int base;  // element index of h = 0
    int l;     // position inside the block (twiddle exponent factor)
  };
  static __device__ __forceinline__ BF coords(int beta) {
    BF r;
    if constexpr (AXIS == 1) {
      // lanes run along i2 (contiguous), then l, then blk
      int i2 = beta & (PL::N2 - 1);
      int rest = beta >> PL::L2;
      int l = rest & (S - 1);
      int blk = rest >> LS;
      r.base = ((blk << LB) + l) * PL::N2 + i2;
      r.l = l;
    } else {
      // lanes run along i1 first (row stride n2 + 1 pad: conflict free), then l, then blk
      int i1 = beta & (PL::N1 - 1);
      int rest = beta >> PL::L1;
      int l = rest & (S - 1);
      int blk = rest >> LS;
      r.base = i1 * PL::N2 + (blk << LB) + l;
      r.l = l;
    }
    return r;
  }
  static constexpr int hstride() { return (AXIS == 1) ? S * PL::N2 : S; }
};

// Twiddle W_B^{l k} = W_LA^{l k 2^(LA-LB)} from an axis table of W_LA^i.
// The tables are read through the constant address space: they are never
// written while a kernel runs, so a wave-uniform index becomes a scalar load
// even where the compiler cannot prove it (after stores, in non-inlined
// functions).
template <class PL, int P, typename T>
__device__ __forceinline__ cx<T> twid(const cx<T>* __restrict__ tw, int l, int k) {
  using G = PassGeo<PL, P>;
  int idx = (l * k) << (G::LA - G::LB);
  const __attribute__((address_space(4))) T* c = (const __attribute__((address_space(4))) T*)tw;
  return cx<T>{c[2 * idx], c[2 * idx + 1]};
}

// Twiddle position l of butterfly j. Lanes of a wave run along the other
// axis first, so when that axis has >= 64 points every lane of a wave has the
// same l: readfirstlane makes that visible to the compiler, which then keeps
// the twiddles in scalar registers (scalar loads from the table).
template <class PL, int P>
__device__ __forceinline__ int pass_l(int ltid, int j) {
  using G = PassGeo<PL, P>;
  int l = G::coords(j * PL::T + ltid).l;
  constexpr bool uniform = (G::AXIS == 1) ? (PL::L2 >= 6) : (PL::L1 >= 6);
  if constexpr (uniform) l = __builtin_amdgcn_readfirstlane(l);
  return l;
}

// Forward pass P on the thread's registers x[E] (values of butterfly j at x[j*R + h]).
template <class PL, int P, typename T>
__device__ __forceinline__ void fwd_pass(cx<T>* x, int ltid, const cx<T>* __restrict__ tw) {
  using G = PassGeo<PL, P>;
#pragma unroll
  for (int j = 0; j < G::NB; ++j) {
    cx<T>* v = x + j * G::R;
    dftR<G::R, T, false>(v);
    if constexpr (G::S > 1) {
      int l = pass_l<PL, P>(ltid, j);
#pragma unroll
      for (int k = 1; k < G::R; ++k) v[k] = cmul(v[k], twid<PL, P, T>(tw, l, k));
    }
  }
}

// Inverse (adjoint) of pass P: conjugate twiddle, then inverse radix DFT.
template <class PL, int P, typename T>
__device__ __forceinline__ void inv_pass(cx<T>* x, int ltid, const cx<T>* __restrict__ tw) {
  using G = PassGeo<PL, P>;
#pragma unroll
  for (int j = 0; j < G::NB; ++j) {
    cx<T>* v = x + j * G::R;
    if constexpr (G::S > 1) {
      int l = pass_l<PL, P>(ltid, j);
#pragma unroll
      for (int k = 1; k < G::R; ++k) v[k] = cmulc(v[k], twid<PL, P, T>(tw, l, k));
    }
    dftR<G::R, T, true>(v);
  }
}

// Base element index (h = 0) of the j-th butterfly a thread executes in pass P;
// value h sits at base + h * hstride().
template <class PL, int P>
__device__ __forceinline__ int bf_base(int ltid, int j) {
  using G = PassGeo<PL, P>;
  return G::coords(j * PL::T + ltid).base;
}

// LDS slot of element base + h * hstride: the padding (one slot per grid row)
// turns the stride into a compile-time constant.
template <class PL, int P>
struct LdsStride {
  using G = PassGeo<PL, P>;
  static constexpr int value = (G::AXIS == 1 && PL::PADSH < 30) ? G::S * (PL::N2 + 1) : G::hstride();
};

// FP32 complex values go to LDS as 8-byte pairs. FP64 complex values go as
// two planes (real parts, then imaginary parts, each LDS_ROW doubles in the
// row's region): every access is then 8 bytes wide with the FP32 addressing,
// which the padding keeps free of bank conflicts (16-byte elements are not).
template <class PL, int P, typename T>
__device__ __forceinline__ void lds_store(cx<T>* lds, const cx<T>* x, int ltid) {
  using G = PassGeo<PL, P>;
#pragma unroll
  for (int j = 0; j < G::NB; ++j) {
    const int a = PL::lds_addr(bf_base<PL, P>(ltid, j));
    if constexpr (sizeof(T) == 8) {
      double* re = (double*)lds + a;
      double* im = re + PL::LDS_ROW;
#pragma unroll
      for (int h = 0; h < G::R; ++h) {
        re[h * LdsStride<PL, P>::value] = x[j * G::R + h].x;
        im[h * LdsStride<PL, P>::value] = x[j * G::R + h].y;
      }
    } else {
      cx<T>* p = lds + a;
#pragma unroll
      for (int h = 0; h < G::R; ++h) p[h * LdsStride<PL, P>::value] = x[j * G::R + h];
    }
  }
}

template <class PL, int P, typename T>
__device__ __forceinline__ void lds_load(const cx<T>* lds, cx<T>* x, int ltid) {
  using G = PassGeo<PL, P>;
#pragma unroll
  for (int j = 0; j < G::NB; ++j) {
    const int a = PL::lds_addr(bf_base<PL, P>(ltid, j));
    if constexpr (sizeof(T) == 8) {
      const double* re = (const double*)lds + a;
      const double* im = re + PL::LDS_ROW;
#pragma unroll
      for (int h = 0; h < G::R; ++h)
        x[j * G::R + h] = cx<T>{re[h * LdsStride<PL, P>::value], im[h * LdsStride<PL, P>::value]};
    } else {
      const cx<T>* p = lds + a;
#pragma unroll
      for (int h = 0; h < G::R; ++h) x[j * G::R + h] = p[h * LdsStride<PL, P>::value];
    }
  }
}

// Natural-order access to the thread's values in the layout of pass 0
// (used for the row t, the masks and the accumulated adjoint).
template <class PL>
struct Layout0 {
  using G = PassGeo<PL, 0>;
  static constexpr int NB = G::NB, R = G::R, HS = G::hstride();
  static __device__ __forceinline__ int base(int ltid, int j) { return bf_base<PL, 0>(ltid, j); }
};

// Spectrum access in the layout of the last forward pass. That pass is the
// lowest digit of its axis (S = 1), so value h of butterfly j holds frequency
// kbase(j) + h * KS (natural raster index k1*n2 + k2).
template <class PL>
struct LayoutL {
  static constexpr int P = PL::NP - 1;
  using G = PassGeo<PL, P>;
  static_assert(G::S == 1, "last pass must be the lowest digit of its axis");
  static constexpr int NB = G::NB, R = G::R;
  static constexpr int KS = (G::AXIS == 1) ? (PL::N1 / G::R) * PL::N2 : PL::N2 / G::R;
  static __device__ __forceinline__ int kbase(int ltid, int j);
};

// A pointer every lane of the wave holds, moved to scalar registers (inside
// non-inlined functions arguments are otherwise taken to differ per lane).
template <typename V>
__device__ __forceinline__ V* wave_uniform(V* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (V*)(((uint64_t)hi << 32) | lo);
}

// Twiddle tables: axis 1 at tw1 (n1 entries W_n1^i), axis 2 at tw2.
template <typename T>
struct Tw {
  const cx<T>* __restrict__ t1;
  const cx<T>* __restrict__ t2;
  __device__ Tw(const cx<T>* a, const cx<T>* b) : t1(wave_uniform(a)), t2(wave_uniform(b)) {}
};

template <class PL, int P, typename T>
__device__ __forceinline__ const cx<T>* tw_of(const Tw<T>& tw) {
  return (PassGeo<PL, P>::AXIS == 1) ? tw.t1 : tw.t2;
}

// LDS exchange buffers of one row. With two buffers (alt != 0) exchange k
// writes buffer k % 2, so one barrier per exchange suffices: every thread's
// reads of exchange k-1 precede its writes of exchange k, and the barrier of
// exchange k orders all of them before the reads of exchange k; the writes of
// exchange k+1 go to the other buffer. With one buffer a second barrier
// protects the reads of the previous exchange.
template <typename T>
struct Xbuf {
  cx<T>* base;
  int alt;     // element offset of the second buffer, 0 if single-buffered
  int parity;  // buffer of the next exchange
  __device__ __forceinline__ cx<T>* next() {
    cx<T>* p = base + (parity ? alt : 0);
    parity ^= (alt != 0);
    return p;
  }
};

template <class PL, int PW, int PR, typename T>
__device__ __forceinline__ void exchange(cx<T>* x, Xbuf<T>& xb, int ltid) {
  cx<T>* lds = xb.next();
  if (xb.alt == 0) __syncthreads();
  lds_store<PL, PW, T>(lds, x, ltid);
  __syncthreads();
  lds_load<PL, PR, T>(lds, x, ltid);
}

// Full forward DFT: x enters in the layout of pass 0 (natural element values),
// leaves in the layout of the last pass holding the digit-reversed spectrum.
template <class PL, int P, typename T>
__device__ __forceinline__ void fwd_from(cx<T>* x, Xbuf<T>& xb, int ltid, const Tw<T>& tw) {
  if constexpr (P < PL::NP) {
    if constexpr (P > 0) exchange<PL, P - 1, P, T>(x, xb, ltid);
    fwd_pass<PL, P, T>(x, ltid, tw_of<PL, P, T>(tw));
    fwd_from<PL, P + 1, T>(x, xb, ltid, tw);
  }
}

// before_last() runs after the last exchange, before the last radix pass
// (loads issued there are in flight during that pass).
struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

template <class PL, int P, typename T, class H>
__device__ __forceinline__ void inv_from(cx<T>* x, Xbuf<T>& xb, int ltid, const Tw<T>& tw, const H& before_last) {
  if constexpr (P >= 0) {
    if constexpr (P < PL::NP - 1) exchange<PL, P + 1, P, T>(x, xb, ltid);
    if constexpr (P == 0) before_last();
    inv_pass<PL, P, T>(x, ltid, tw_of<PL, P, T>(tw));
    inv_from<PL, P - 1, T>(x, xb, ltid, tw, before_last);
  }
}

template <class PL, typename T>
__device__ __forceinline__ void fft_forward(cx<T>* x, Xbuf<T>& xb, int ltid, const Tw<T>& tw) {
  fwd_from<PL, 0, T>(x, xb, ltid, tw);
}
template <class PL, typename T, class H = NoHook>
__device__ __forceinline__ void fft_inverse(cx<T>* x, Xbuf<T>& xb, int ltid, const Tw<T>& tw,
                                            const H& before_last = H{}) {
  inv_from<PL, PL::NP - 1, T>(x, xb, ltid, tw, before_last);
}

// Digit reversal of one axis: slot index s (digits high to low as laid out by
// the DIF passes) -> frequency index k = d_0 + R_0 d_1 + R_0 R_1 d_2 + ...
template <int LA, int VAR, int MB = 4>
__device__ __forceinline__ int digit_rev(int s) {
  constexpr int nd = ndigits(LA, MB);
  int k = 0, shift_out = 0, rem = LA;
#pragma unroll
  for (int i = 0; i < nd; ++i) {
    int b = digit_bits(LA, i, VAR, MB);
    rem -= b;
    int d = (s >> rem) & ((1 << b) - 1);
    k |= d << shift_out;
    shift_out += b;
  }
  return k;
}

// Frequency (natural raster index k1*n2 + k2) held at element slot e after the forward DFT.
template <class PL>
__device__ __forceinline__ int spectrum_index(int e) {
  int s1 = e >> PL::L2, s2 = e & (PL::N2 - 1);
  return (digit_rev<PL::L1, PL::VAR, PL::MB>(s1) << PL::L2) | digit_rev<PL::L2, PL::VAR, PL::MB>(s2);
}

template <class PL>
__device__ __forceinline__ int LayoutL<PL>::kbase(int ltid, int j) {
  return spectrum_index<PL>(bf_base<PL, PL::NP - 1>(ltid, j));
}

}  // namespace tmk
