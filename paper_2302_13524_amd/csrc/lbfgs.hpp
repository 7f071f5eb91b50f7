// Per-row L-BFGS of Algorithm 1 on the device: direction by the two-loop
// recursion, exact minimiser of the quartic line function, history update.
#pragma once
#include "grids.hpp"

namespace tmk {

struct RowArgs;

// Per row: head, count, alpha, pending, then S^T Y and Y^T Y over the ring
// slots ([m+1][m+1] each), then the direction's coefficients (1 + 2 (m+1)). The history is a ring of m + 1 slots: up to m
// accepted pairs and, at slot head, the pending pair of the last step, which
// joins the ring only once s^T y > 0.
constexpr int LB_SLOTS(int m) { return m + 1; }
constexpr int LB_SCALARS(int m) { return 4 + 2 * LB_SLOTS(m) * LB_SLOTS(m) + 1 + 2 * LB_SLOTS(m); }
// partial dot products of the direction kernels: doubles per row
constexpr size_t LB_DOTS(int N) { return (size_t)(N > 1024 ? N / 1024 : 1) * (5 + 4 * 16); }

struct LbfgsBuffers {
  void* g;    // [P][N] gradient at t
  void* gp;   // [P][N] gradient at the previous t
  void* d;    // [P][N] direction
  void* S;    // [P][m+1][N] steps s_i
  void* Y;    // [P][m+1][N] gradient differences y_i
  void* sc;   // [P][LB_SCALARS(m)] doubles
  float* sums;  // [P][NSUM]
  void* dots;   // [P][LB_DOTS(N)] doubles
  // optional timing hooks around the direction (mode 20) and step (mode 21) launches
  void* hook_user = nullptr;
  void (*hook_begin)(void* user, int mode, void* stream) = nullptr;
  void (*hook_end)(void* user, int mode, void* stream) = nullptr;
};

// Runs `iters` iterations starting from t (in place), on the intensity cost
// (amplitude = 0) or the amplitude cost (1). Returns a hipError_t.
int run_lbfgs(row_launcher fn, const RowArgs& base, int ibf16, int N, int iters, int m,
              void* t, LbfgsBuffers& b, void* stream, int amplitude);

}  // namespace tmk
