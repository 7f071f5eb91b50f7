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

using PLd = Plan<GL1, GL2, (GL1 + GL2 >= 4) ? 4 : GL1 + GL2>;  // FP64 residual: 16 values per thread

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

void TM_CAT(row_shape, GL1, GL2)(int* wg, int* rpw) {
  *wg = Launch<Plan<GL1, GL2>>::WG;
  *rpw = Launch<Plan<GL1, GL2>>::RPW;
}

}  // namespace tmk
