// Compiled (log2 n1, log2 n2) grids. Each line instantiates every row
// kernel for one grid in its own object file (grid_inst.hip).
#pragma once
#define TM_GRID_LIST(X) \
  X(0, 4) X(0, 6) X(0, 10) X(2, 2) X(2, 4) X(4, 2) X(3, 3) X(4, 4) X(3, 5) \
  X(5, 5) X(6, 5) X(5, 6) X(6, 6) X(7, 6) X(6, 7) X(7, 5) X(5, 7) X(7, 7)

namespace tmk {
struct RowArgs;
// Launch one row kernel. mode: tmk::Mode; ibf16: intensities are bf16.
// Returns hipSuccess, or hipErrorInvalidValue when (L1, L2) is not compiled.
typedef int (*row_launcher)(int mode, int ibf16, const RowArgs& a, void* stream);
// cfg: launch configuration; 0 and 1 the FFT digit-order variant (0: larger
// digits first, 1: smaller first), bits 2 and 4 (for the Lanczos and cyclic
// ER steps, where compiled) eight values per thread and twice the rows per
// workgroup. nullptr when the grid or the configuration is not compiled.
row_launcher find_row_launcher(int L1, int L2, int cfg = 0);
// bit k set: configuration k is compiled for the grid (0 if the grid is not)
int row_cfg_mask(int L1, int L2);
// workgroup threads, rows per workgroup and values per thread of a configuration (zeros if absent)
void row_cfg_shape(int L1, int L2, int cfg, int* wg, int* rpw, int* ept);
// threads per workgroup and rows per workgroup of a grid
void row_launch_shape(int L1, int L2, int* wg, int* rpw);
}  // namespace tmk
