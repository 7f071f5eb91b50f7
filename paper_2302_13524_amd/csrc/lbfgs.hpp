// Per-row L-BFGS of Algorithm 1 on the device: direction by the two-loop
// recursion, exact minimiser of the quartic line function, history update.
#pragma once
#include "grids.hpp"

namespace tmk {

struct RowArgs;

// Per row: head, count, alpha, pending, sy[m+1], yy[m+1]. The history is a
// ring of m + 1 slots: up to m accepted pairs and, at slot head, the pending
// pair of the last step, which joins the ring only once s^T y > 0.
constexpr int LB_SLOTS(int m) { return m + 1; }
constexpr int LB_SCALARS(int m) { return 4 + 2 * LB_SLOTS(m); }

struct LbfgsBuffers {
  void* g;    // [P][N] gradient at t
  void* gp;   // [P][N] gradient at the previous t
  void* d;    // [P][N] direction
  void* S;    // [P][m+1][N] steps s_i
  void* Y;    // [P][m+1][N] gradient differences y_i
  void* sc;   // [P][LB_SCALARS(m)] doubles
  float* sums;  // [P][NSUM]
};

// Runs `iters` iterations starting from t (in place), on the intensity cost
// (amplitude = 0) or the amplitude cost (1). Returns a hipError_t.
int run_lbfgs(row_launcher fn, const RowArgs& base, int ibf16, int N, int iters, int m,
              void* t, LbfgsBuffers& b, void* stream, int amplitude);

}  // namespace tmk
