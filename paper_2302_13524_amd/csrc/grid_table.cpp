// Table of the per-grid launchers compiled from grid_inst.hip.
#include "grids.hpp"

namespace tmk {

#define TM_DECL(a, b)                                                        \
  int row_launch_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s);   \
  int row_launchv_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s);  \
  int row_launchc2_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_launchc3_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_launchc4_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_launchc5_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_launchc6_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_launchc7_##a##_##b(int mode, int ibf16, const RowArgs& x, void* s); \
  int row_cfgmask_##a##_##b();                                                \
  void row_cfgshape_##a##_##b(int cfg, int* wg, int* rpw, int* ept);          \
  void row_shape_##a##_##b(int* wg, int* rpw);
TM_GRID_LIST(TM_DECL)

row_launcher find_row_launcher(int L1, int L2, int cfg) {
#define TM_FIND(a, b)                                                  \
  if (L1 == a && L2 == b) {                                            \
    if (cfg < 0 || cfg > 7 || !((row_cfgmask_##a##_##b() >> cfg) & 1)) \
      return nullptr;                                                  \
    switch (cfg) {                                                     \
      case 0: return &row_launch_##a##_##b;                            \
      case 1: return &row_launchv_##a##_##b;                           \
      case 2: return &row_launchc2_##a##_##b;                          \
      case 3: return &row_launchc3_##a##_##b;                          \
      case 4: return &row_launchc4_##a##_##b;                          \
      case 5: return &row_launchc5_##a##_##b;                          \
      case 6: return &row_launchc6_##a##_##b;                          \
      default: return &row_launchc7_##a##_##b;                         \
    }                                                                  \
  }
  TM_GRID_LIST(TM_FIND)
  return nullptr;
}

int row_cfg_mask(int L1, int L2) {
#define TM_MASK(a, b) \
  if (L1 == a && L2 == b) return row_cfgmask_##a##_##b();
  TM_GRID_LIST(TM_MASK)
  return 0;
}

void row_cfg_shape(int L1, int L2, int cfg, int* wg, int* rpw, int* ept) {
  *wg = *rpw = *ept = 0;
#define TM_CSHAPE(a, b) \
  if (L1 == a && L2 == b) { row_cfgshape_##a##_##b(cfg, wg, rpw, ept); return; }
  TM_GRID_LIST(TM_CSHAPE)
}

void row_launch_shape(int L1, int L2, int* wg, int* rpw) {
  *wg = 0;
  *rpw = 0;
#define TM_SHAPE(a, b) \
  if (L1 == a && L2 == b) { row_shape_##a##_##b(wg, rpw); return; }
  TM_GRID_LIST(TM_SHAPE)
}

}  // namespace tmk
