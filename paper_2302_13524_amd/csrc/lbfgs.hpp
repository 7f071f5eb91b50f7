// Per-row L-BFGS of Algorithm 1 on the device: direction by the two-loop
// recursion, exact minimiser of the quartic line function, history update.
#pragma once
#include "grids.hpp"

namespace tmk {

struct RowArgs;

constexpr int LB_SCALARS(int m) { return 4 + 2 * m; }  // head, count, alpha, pending, sy[m], yy[m]

struct LbfgsBuffers {
  void* g;    // [P][N] gradient at t
  void* gp;   // [P][N] gradient at the previous t
  void* d;    // [P][N] direction
  void* S;    // [P][m][N] steps s_i
  void* Y;    // [P][m][N] gradient differences y_i
  void* sc;   // [P][LB_SCALARS(m)] doubles
  float* sums;  // [P][NSUM]
};

// Runs `iters` iterations starting from t (in place), on the intensity cost
// (amplitude = 0) or the amplitude cost (1). Returns a hipError_t.
int run_lbfgs(row_launcher fn, const RowArgs& base, int ibf16, int N, int iters, int m,
              void* t, LbfgsBuffers& b, void* stream, int amplitude);

}  // namespace tmk
