// Persistent batched pass over uneven problems. Every work item is one row
// tile of one problem (1 row of 8192 modes, 2 of 4096, 4 of 2048, 8 of
// 1024: tiles of similar FFT work); workgroups stride over the item list, and
// each item runs the same fused row body as the single-problem kernels,
// specialised for its grid and FFT digit order.
#include <hip/hip_runtime.h>

#include "batch.hpp"
#include "row_kernels.hpp"

namespace tmk {

int batch_grid_id(int n1, int n2) {
  if (n1 == 32 && n2 == 32) return 0;
  if (n1 == 64 && n2 == 32) return 1;
  if (n1 == 64 && n2 == 64) return 2;
  if (n1 == 128 && n2 == 64) return 3;
  return -1;
}

int batch_rows_per_item(int g) {
  switch (g) {
    case 0: return Launch<Plan<5, 5>, BATCH_WG>::RPW;
    case 1: return Launch<Plan<6, 5>, BATCH_WG>::RPW;
    case 2: return Launch<Plan<6, 6>, BATCH_WG>::RPW;
    case 3: return Launch<Plan<7, 6>, BATCH_WG>::RPW;
  }
  return 0;
}

namespace {

template <class PL>
constexpr int lds_of() {
  return Launch<PL, BATCH_WG>::LDS_ELEMS;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kLds = cmax(cmax(lds_of<Plan<5, 5>>(), lds_of<Plan<6, 5>>()), cmax(lds_of<Plan<6, 6>>(), lds_of<Plan<7, 6>>()));

// Launch-wide values the item bodies need. They reach the out-of-line bodies as
// scalars: a struct passed to a non-inlined function goes through private
// memory (the row arguments were stored there for every item and read back by
// per-lane loads).
struct ItemLaunch {
  float tau, momentum, lower, er_beta;
  int swap, lz_j, lz_fuse, lz_k;
};

__device__ __forceinline__ float uniform_f(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }

// A table entry at a wave-uniform address, word by word through the constant
// address space (the tables are not written while the kernel runs), so that
// every word is a scalar load.
template <typename S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "whole words");
  typedef const __attribute__((address_space(4))) uint32_t* WordC;
  const WordC src = (WordC)p;
  uint32_t words[sizeof(S) / 4];
#pragma unroll
  for (int k = 0; k < (int)(sizeof(S) / 4); ++k) words[k] = src[k];
  S v;
  __builtin_memcpy(&v, words, sizeof(S));
  return v;
}

// One out-of-line body per specialisation, so that each gets its own register
// allocation instead of the union of all of them. It builds the row arguments
// of item `it` from the problem table (wave-uniform, so scalar loads).
template <class PL, int M, int MODE, typename IT, bool SUMS>
__device__ __attribute__((noinline)) void item_body(const BatchProb* probs, const BatchItem* items, int it,
                                                     const cx<float>* tw32, float tau, float momentum, float lower,
                                                     float er_beta, int swap, int lz_j, int lz_fuse, int lz_k,
                                                     cx<float>* lds, float* red) {
  it = __builtin_amdgcn_readfirstlane(it);
  const ItemLaunch b{uniform_f(tau), uniform_f(momentum), uniform_f(lower), uniform_f(er_beta),
                     __builtin_amdgcn_readfirstlane(swap), __builtin_amdgcn_readfirstlane(lz_j),
                     __builtin_amdgcn_readfirstlane(lz_fuse), __builtin_amdgcn_readfirstlane(lz_k)};
  const BatchItem w = load_uniform(wave_uniform(items) + it);
  const BatchProb pr = load_uniform(wave_uniform(probs) + __builtin_amdgcn_readfirstlane(w.prob));
  RowArgs a;
  a.P = pr.P;
  a.K = pr.K;
  a.masks = pr.masks;
  // spectral steps and ER with momentum read the iterate and the previous
  // one and overwrite the previous one; the two buffers swap roles every step
  const bool mom = MODE == BATCH_ER && b.er_beta != 0.f;
  const bool two = mom || MODE == BATCH_SPEC;
  cx<float>* cur = (two && b.swap) ? pr.vprev : pr.t;
  cx<float>* oth = (two && b.swap) ? pr.t : pr.vprev;
  a.tin = cur;
  a.tout = two ? oth : cur;
  a.din = oth;
  a.vscale = pr.vscale;
  a.I = pr.I;
  a.yin = nullptr;
  a.yout = nullptr;
  a.sums = SUMS ? pr.sums : nullptr;
  a.sums64 = nullptr;
  a.rowmean = pr.rowmean;
  a.tau = b.tau;
  a.momentum = b.momentum;
  a.spec_lower = b.lower;
  a.er_beta = mom ? b.er_beta : 0.f;
  a.lz_bprev = nullptr;
  a.lz_out = nullptr;
  a.lz_sum = nullptr;
  a.lz_mean = nullptr;
  a.lb_sc = nullptr;  // no L-BFGS modes in the batch
  if constexpr (MODE == BATCH_LZ) {
    // step j from V(j) to V(j + 1), V(0) = t, V(i) = lzV + (i - 1) P N; (alpha, beta) into row j of lzH
    const int j = b.lz_j;
    const size_t rs = (size_t)pr.P * pr.N;
    auto V = [&](int i) { return i == 0 ? pr.t : pr.lzV + (size_t)(i - 1) * rs; };
    a.tin = V(j);
    a.din = V(j > 0 ? j - 1 : 0);
    a.tout = V(j + 1);
    a.lz_bprev = j > 0 ? pr.lzH + (size_t)(j - 1) * pr.P * 2 : nullptr;
    a.lz_out = pr.lzH + (size_t)j * pr.P * 2;
    if (j == 0) {  // row sums, means and the unit seed, as the single-problem first step
      a.lz_sum = pr.rowsum;
      a.lz_mean = pr.rowmean;
    }
  }
  a.lz_basis = nullptr;
  a.lz_y = nullptr;
  a.lz_k = 0;
  a.lz_rs = 0;
  if constexpr (MODE == BATCH_ERC) {
    if (b.lz_fuse) {
      a.lz_basis = pr.lzV;
      a.lz_y = pr.lzY;
      a.lz_k = b.lz_k;
      a.lz_rs = (int64_t)pr.P * pr.N;
    }
  }
  a.out_bf16 = 0;
  a.tw32 = wave_uniform(tw32);
  a.tw64 = nullptr;
  row_body<PL, M, IT, SUMS, BATCH_WG, true>(a, w.blk, lds, red);
}

template <int MODE, typename IT, bool SUMS>
__global__ void __launch_bounds__(BATCH_WG) batch_kernel(BatchArgs b) {
  __shared__ cx<float> lds[kLds];
  __shared__ float red[Launch<Plan<7, 6>, BATCH_WG>::RED_FLOATS];
  constexpr int M = (MODE == BATCH_ER) ? M_ER : (MODE == BATCH_ERC) ? M_ERC : (MODE == BATCH_LZ) ? M_LANCZOS : M_SPEC;
  for (int it = blockIdx.x; it < b.n_items; it += gridDim.x) {
    const int code = b.probs[b.items[it].prob].code;
#define TM_ITEM(...)                                                                                      \
  item_body<__VA_ARGS__, M, MODE, IT, SUMS>(b.probs, b.items, it, b.tw32, b.tau, b.momentum, b.lower, b.er_beta, \
                                            b.swap, b.lz_j, b.lz_fuse, b.lz_k, lds, red)
    switch (code) {
      case 0: TM_ITEM(Plan<5, 5, -1, 0>); break;
      case 1: TM_ITEM(Plan<5, 5, -1, 1>); break;
      case 2: TM_ITEM(Plan<6, 5, -1, 0>); break;
      case 3: TM_ITEM(Plan<6, 5, -1, 1>); break;
      case 4:
      case 5: TM_ITEM(Plan<6, 6, -1, 0>); break;
      case 6: TM_ITEM(Plan<7, 6, -1, 0>); break;
      case 7: TM_ITEM(Plan<7, 6, -1, 1>); break;
      default: break;
    }
#undef TM_ITEM
    __syncthreads();  // LDS of this item is free before the next item writes it
  }
}

template <int MODE, typename IT>
int launch_m(int with_sums, const BatchArgs& a, int grid, hipStream_t s) {
  if (with_sums) batch_kernel<MODE, IT, true><<<grid, BATCH_WG, 0, s>>>(a);
  else batch_kernel<MODE, IT, false><<<grid, BATCH_WG, 0, s>>>(a);
  return (int)hipGetLastError();
}

}  // namespace

int batch_launch(int mode, int ibf16, int with_sums, const BatchArgs& a, int grid, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (a.n_items <= 0) return 0;
  if (mode == BATCH_ER) return ibf16 ? launch_m<BATCH_ER, uint16_t>(with_sums, a, grid, s)
                                     : launch_m<BATCH_ER, float>(with_sums, a, grid, s);
  if (mode == BATCH_ERC) return ibf16 ? launch_m<BATCH_ERC, uint16_t>(with_sums, a, grid, s)
                                      : launch_m<BATCH_ERC, float>(with_sums, a, grid, s);
  if (mode == BATCH_LZ) return ibf16 ? launch_m<BATCH_LZ, uint16_t>(0, a, grid, s) : launch_m<BATCH_LZ, float>(0, a, grid, s);
  return ibf16 ? launch_m<BATCH_SPEC, uint16_t>(0, a, grid, s) : launch_m<BATCH_SPEC, float>(0, a, grid, s);
}

}  // namespace tmk
