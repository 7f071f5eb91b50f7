// Table of the per-grid launchers compiled from grid_inst.hip.
#include "grids.hpp"

namespace tmk {

#define TM_DECL(a, b)                                                       \
  int row_launch_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s);  \
  int row_launchv_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  void row_shape_##a##_##b(int* wg, int* rpw);
TM_GRID_LIST(TM_DECL)

row_launcher find_row_launcher(int L1, int L2, int var) {
#define TM_FIND(a, b) \
  if (L1 == a && L2 == b) return var ? &row_launchv_##a##_##b : &row_launch_##a##_##b;
  TM_GRID_LIST(TM_FIND)
  return nullptr;
}

void row_launch_shape(int L1, int L2, int* wg, int* rpw) {
  *wg = 0;
  *rpw = 0;
#define TM_SHAPE(a, b) \
  if (L1 == a && L2 == b) { row_shape_##a##_##b(wg, rpw); return; }
  TM_GRID_LIST(TM_SHAPE)
}

}  // namespace tmk
