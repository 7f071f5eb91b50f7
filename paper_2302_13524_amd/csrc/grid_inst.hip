// Instantiates the row kernels for one grid, selected at compile time by
// -DGL1=<log2 n1> -DGL2=<log2 n2>.
#include "row_kernels.hpp"
#include "grids.hpp"

#ifndef GL1
#error "GL1 / GL2 must be defined"
#endif

namespace tmk {

#define TM_CAT2(a, b, c) a##_##b##_##c
#define TM_CAT(a, b, c) TM_CAT2(a, b, c)

// FP64 residual: 8 values per thread (at 128 x 64: 1024 threads, 128 VGPRs, four
// waves per SIMD; 16 values per thread took 248 VGPRs and two waves)
using PLd = Plan<GL1, GL2, (GL1 + GL2 >= 3) ? 3 : GL1 + GL2>;

template <class PLg, typename IT>
static int launch_t(int mode, const RowArgs& a, hipStream_t s) {
  using LC = Launch<PLg>;
  dim3 grid((a.P + LC::RPW - 1) / LC::RPW), block(LC::WG);
  if (a.P <= 0) return 0;
  switch (mode) {
    case M_FWD_FIELD: row_kernel<PLg, M_FWD_FIELD, IT><<<grid, block, 0, s>>>(a); break;
    case M_FWD_INT: row_kernel<PLg, M_FWD_INT, IT><<<grid, block, 0, s>>>(a); break;
    case M_ADJ: row_kernel<PLg, M_ADJ, IT><<<grid, block, 0, s>>>(a); break;
    case M_ER:
      if (a.sums) row_kernel<PLg, M_ER, IT, true><<<grid, block, 0, s>>>(a);
      else row_kernel<PLg, M_ER, IT, false><<<grid, block, 0, s>>>(a);
      break;
    case M_ERC:
      if (a.sums) row_kernel<PLg, M_ERC, IT, true><<<grid, block, 0, s>>>(a);
      else row_kernel<PLg, M_ERC, IT, false><<<grid, block, 0, s>>>(a);
      break;
    case M_GRAD:
      if (a.sums) row_kernel<PLg, M_GRAD, IT, true><<<grid, block, 0, s>>>(a);
      else row_kernel<PLg, M_GRAD, IT, false><<<grid, block, 0, s>>>(a);
      break;
    case M_SPEC: row_kernel<PLg, M_SPEC, IT><<<grid, block, 0, s>>>(a); break;
    case M_LANCZOS: row_kernel<PLg, M_LANCZOS, IT><<<grid, block, 0, s>>>(a); break;
    case M_LANCZOS_T: row_kernel<PLg, M_LANCZOS_T, IT><<<grid, block, 0, s>>>(a); break;
    case M_WAPPLY: row_kernel<PLg, M_WAPPLY, IT><<<grid, block, 0, s>>>(a); break;
    case M_WBACK: row_kernel<PLg, M_WBACK, IT><<<grid, block, 0, s>>>(a); break;
    case M_LS: row_kernel<PLg, M_LS, IT><<<grid, block, 0, s>>>(a); break;
    case M_AGRAD:
      if (a.sums) row_kernel<PLg, M_AGRAD, IT, true><<<grid, block, 0, s>>>(a);
      else row_kernel<PLg, M_AGRAD, IT, false><<<grid, block, 0, s>>>(a);
      break;
    case M_ALS: row_kernel<PLg, M_ALS, IT><<<grid, block, 0, s>>>(a); break;
    case M_FILT: row_kernel<PLg, M_FILT, IT><<<grid, block, 0, s>>>(a); break;
    case M_BACKPROP: row_kernel<PLg, M_BACKPROP, IT><<<grid, block, 0, s>>>(a); break;
    case M_RES64: {
      using LD = Launch<PLd>;
      size_t lds = (size_t)LD::RPW * PLd::LDS_ROW * sizeof(cx<double>) + (LD::WG / 64 + 1) * sizeof(double);
      auto fn = res64_kernel<PLd, IT>;
      hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return (int)e;
      fn<<<dim3((a.P + LD::RPW - 1) / LD::RPW), dim3(LD::WG), lds, s>>>(a);
      break;
    }
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Digit-order variant 1 differs from variant 0 only when an axis splits
// into digits of unequal size.
constexpr bool uneven(int b) { return ndigits(b) >= 2 && b % ndigits(b) != 0; }
constexpr bool kHasVar = uneven(GL1) || uneven(GL2);

int TM_CAT(row_launch, GL1, GL2)(int mode, int ibf16, const RowArgs& a, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  using P0 = Plan<GL1, GL2>;
  return ibf16 ? launch_t<P0, uint16_t>(mode, a, s) : launch_t<P0, float>(mode, a, s);
}

int TM_CAT(row_launchv, GL1, GL2)(int mode, int ibf16, const RowArgs& a, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if constexpr (kHasVar) {
    using P1 = Plan<GL1, GL2, -1, 1>;
    return ibf16 ? launch_t<P1, uint16_t>(mode, a, s) : launch_t<P1, float>(mode, a, s);
  } else {
    using P0 = Plan<GL1, GL2>;
    return ibf16 ? launch_t<P0, uint16_t>(mode, a, s) : launch_t<P0, float>(mode, a, s);
  }
}

// Wider configurations for the autotuner, cfg bits: 1 the digit order
// (variant 1), 2 eight values per thread instead of sixteen, 4 twice the rows
// per workgroup. They apply to the iteration and start kernels the batch also
// runs (error reduction, averaged and cyclic; heavy-ball spectral and Lanczos
// steps) and to the L-BFGS solvers' gradient kernels and the amplitude cost's
// line search (the intensity cost's line search, which holds both transforms
// of a mask at once, spills at eight values per thread and keeps the default
// plan); every other mode runs the default plan of the same digit order.
// Compiled for the grids of the benchmark workloads.
constexpr bool kExt = (GL1 == 5 && GL2 == 5) || (GL1 == 6 && GL2 == 5) || (GL1 == 6 && GL2 == 6) ||
                      (GL1 == 7 && GL2 == 6);

template <int CFG>
struct XCfg {
  static constexpr int LE = (CFG & 2) ? 3 : -1;
  using PX = Plan<GL1, GL2, LE, (CFG & 1) && kHasVar ? 1 : 0>;
  static constexpr int WG0 = Launch<PX>::WG;
  static constexpr int WG = (CFG & 4) ? 2 * WG0 : WG0;
  // twice the rows only up to 512 threads (two waves per SIMD keep a 256-register budget)
  static constexpr bool ok = kExt && (CFG & 6) != 0 && (GL1 + GL2 >= 3) && ((CFG & 4) ? WG <= 512 : WG <= 1024);
};

template <class PX, int WG, typename IT>
static int launch_x(int mode, const RowArgs& a, hipStream_t s) {
  constexpr int RPW = WG / PX::T;
  static_assert(RPW >= 1 && RPW * PX::T == WG, "whole rows per workgroup");
  if (a.P <= 0) return 0;
  dim3 grid((a.P + RPW - 1) / RPW), block(WG);
  switch (mode) {
    case M_LANCZOS: row_kernel_w<PX, M_LANCZOS, IT, true, WG><<<grid, block, 0, s>>>(a); break;
    case M_LANCZOS_T: row_kernel_w<PX, M_LANCZOS_T, IT, true, WG><<<grid, block, 0, s>>>(a); break;
    case M_SPEC: row_kernel_w<PX, M_SPEC, IT, true, WG><<<grid, block, 0, s>>>(a); break;
    case M_ER:
      if (a.sums) row_kernel_w<PX, M_ER, IT, true, WG><<<grid, block, 0, s>>>(a);
      else row_kernel_w<PX, M_ER, IT, false, WG><<<grid, block, 0, s>>>(a);
      break;
    case M_ERC:
      if (a.sums) row_kernel_w<PX, M_ERC, IT, true, WG><<<grid, block, 0, s>>>(a);
      else row_kernel_w<PX, M_ERC, IT, false, WG><<<grid, block, 0, s>>>(a);
      break;
    case M_GRAD:
      if (a.sums) row_kernel_w<PX, M_GRAD, IT, true, WG><<<grid, block, 0, s>>>(a);
      else row_kernel_w<PX, M_GRAD, IT, false, WG><<<grid, block, 0, s>>>(a);
      break;
    case M_AGRAD:
      if (a.sums) row_kernel_w<PX, M_AGRAD, IT, true, WG><<<grid, block, 0, s>>>(a);
      else row_kernel_w<PX, M_AGRAD, IT, false, WG><<<grid, block, 0, s>>>(a);
      break;
    case M_ALS: row_kernel_w<PX, M_ALS, IT, true, WG><<<grid, block, 0, s>>>(a); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

template <int CFG>
static int launch_cfg(int mode, int ibf16, const RowArgs& a, void* stream) {
  using X = XCfg<CFG>;
  if constexpr (!X::ok) {
    return (int)hipErrorInvalidValue;
  } else {
    hipStream_t s = (hipStream_t)stream;
    if (mode == M_LANCZOS || mode == M_ERC || mode == M_ER || mode == M_SPEC || mode == M_GRAD || mode == M_AGRAD ||
        mode == M_ALS)
      return ibf16 ? launch_x<typename X::PX, X::WG, uint16_t>(mode, a, s)
                   : launch_x<typename X::PX, X::WG, float>(mode, a, s);
    if (mode == M_LANCZOS_T && !ibf16) return launch_x<typename X::PX, X::WG, float>(mode, a, s);
    return (CFG & 1) ? TM_CAT(row_launchv, GL1, GL2)(mode, ibf16, a, stream)
                     : TM_CAT(row_launch, GL1, GL2)(mode, ibf16, a, stream);
  }
}

#define TM_CFG_FN(k)                                                                      \
  int TM_CAT(row_launchc##k, GL1, GL2)(int mode, int ibf16, const RowArgs& a, void* s) { \
    return launch_cfg<k>(mode, ibf16, a, s);                                             \
  }
TM_CFG_FN(2)
TM_CFG_FN(3)
TM_CFG_FN(4)
TM_CFG_FN(5)
TM_CFG_FN(6)
TM_CFG_FN(7)

// bit k set: configuration k is compiled for this grid
int TM_CAT(row_cfgmask, GL1, GL2)() {
  return 3 | (XCfg<2>::ok << 2) | (XCfg<3>::ok << 3) | (XCfg<4>::ok << 4) | (XCfg<5>::ok << 5) |
         (XCfg<6>::ok << 6) | (XCfg<7>::ok << 7);
}

// threads per workgroup, rows per workgroup, values per thread of configuration cfg
void TM_CAT(row_cfgshape, GL1, GL2)(int cfg, int* wg, int* rpw, int* ept) {
  *wg = *rpw = *ept = 0;
  auto put = [&](int w, int t, int e) { *wg = w; *rpw = w / t; *ept = e; };
  switch (cfg) {
    case 0: case 1: put(Launch<Plan<GL1, GL2>>::WG, Plan<GL1, GL2>::T, Plan<GL1, GL2>::E); break;
    case 2: if (XCfg<2>::ok) put(XCfg<2>::WG, XCfg<2>::PX::T, XCfg<2>::PX::E); break;
    case 3: if (XCfg<3>::ok) put(XCfg<3>::WG, XCfg<3>::PX::T, XCfg<3>::PX::E); break;
    case 4: if (XCfg<4>::ok) put(XCfg<4>::WG, XCfg<4>::PX::T, XCfg<4>::PX::E); break;
    case 5: if (XCfg<5>::ok) put(XCfg<5>::WG, XCfg<5>::PX::T, XCfg<5>::PX::E); break;
    case 6: if (XCfg<6>::ok) put(XCfg<6>::WG, XCfg<6>::PX::T, XCfg<6>::PX::E); break;
    case 7: if (XCfg<7>::ok) put(XCfg<7>::WG, XCfg<7>::PX::T, XCfg<7>::PX::E); break;
    default: break;
  }
}

void TM_CAT(row_shape, GL1, GL2)(int* wg, int* rpw) {
  *wg = Launch<Plan<GL1, GL2>>::WG;
  *rpw = Launch<Plan<GL1, GL2>>::RPW;
}

}  // namespace tmk
