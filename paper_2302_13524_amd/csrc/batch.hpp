// Uneven multi-TM batches: one persistent launch per iteration covers every
// row of every problem; work items are (problem, row tile).
#pragma once
#include <stdint.h>

#include "fft_core.hpp"

namespace tmk {

constexpr int BATCH_WG = 512;

// Grids the batched kernel is compiled for; code = 2 * grid_id + variant.
// 0: 32 x 32, 1: 64 x 32, 2: 64 x 64, 3: 128 x 64.
int batch_grid_id(int n1, int n2);
// rows per work item (rows of that grid one 512-thread workgroup handles)
int batch_rows_per_item(int grid_id);

struct BatchProb {
  const cx<float>* masks;
  const void* I;
  cx<float>* t;
  cx<float>* vprev;
  float* vscale;        // [P] spectral previous-iterate scale
  float* sums;          // [P][6] or null
  float* rowmean;       // [P] mean of I per row (the first Lanczos step writes it)
  double* rowsum;       // [P] sum of I per row (the same)
  cx<float>* lzV;       // Lanczos basis v_2 .. v_{k+1} [k][P][N] (v_1 is t)
  float* lzH;           // Lanczos (alpha, beta) [k][P][2]
  const double* lzY;    // Ritz coefficients [P][k]
  int K, P, code, N;
};

struct BatchItem {
  int prob, blk;
};

struct BatchArgs {
  const BatchProb* probs;
  const BatchItem* items;
  int n_items;
  int with_sums;         // pass the problems' sums pointers (else null)
  float tau, momentum, lower;
  float er_beta;         // ER Nesterov factor; t and t_prev alternate between t and vprev
  int swap;              // spectral steps, ER with er_beta: the current iterate is in vprev (odd steps)
  int lz_j;              // Lanczos step index (BATCH_LZ)
  int lz_fuse;           // BATCH_ERC: this sweep forms each row's Ritz vector from lz_k basis rows first
  int lz_k;
  const cx<float>* tw32;
};

enum BatchMode { BATCH_ER = 0, BATCH_SPEC = 1, BATCH_ERC = 2, BATCH_LZ = 3 };
// Launch one batched pass (mode BATCH_*) over all items with `grid` workgroups.
int batch_launch(int mode, int ibf16, int with_sums, const BatchArgs& a, int grid, void* stream);

}  // namespace tmk
