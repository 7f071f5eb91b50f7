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
// var: FFT digit-order variant (0: larger digits first, 1: smaller first)
row_launcher find_row_launcher(int L1, int L2, int var = 0);
// threads per workgroup and rows per workgroup of a grid
void row_launch_shape(int L1, int L2, int* wg, int* rpw);
}  // namespace tmk
