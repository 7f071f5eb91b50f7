// Host-side launchers of the helper kernels (aux_kernels.hip).
#pragma once
#include <stdint.h>

namespace tmk {
int launch_row_isum(const void* I, int bf16, int64_t len, int P, double* rowsum, float* rowmean,
                    void* stream);
int launch_row_rescale(void* t, int N, int P, int mode, const double* rowsum, double denom,
                       void* stream);
int launch_fill_zero(void* p, int64_t bytes, void* stream);
// indices of the rows whose stats record has rho > thr (or rho not finite), in no particular
// order, appended at idx[*count] (count must start at 0)
int launch_flag_rows(const void* stats, int P, double thr, int* idx, int* count, void* stream);
// dst row j <- src row idx[j] (rows of row_bytes, a multiple of 8)
int launch_gather_rows(void* dst, const void* src, const int* idx, int rows, int64_t row_bytes, void* stream);
// for j < rows: row idx[j] of t and its stats record take row j of tf / stf when stf's rho is lower
int launch_select_rows(void* t, const void* tf, void* stats, const void* stf, const int* idx, int rows,
                       int64_t row_bytes, void* stream);
// device-to-device copy by a kernel (graph-capturable); bytes and both
// pointers must be multiples of 8
int launch_copy(void* dst, const void* src, int64_t bytes, void* stream);
// fill n floats with hash-derived values in [lo, hi) (synthetic tuning data)
int launch_fill_hash(float* p, int64_t n, uint32_t seed, float lo, float hi, void* stream);
int launch_finalize(void* stats, int P, const double* sums64, const float* sums, int nsum,
                    int f_idx, int amp_idx, int iters, double rho_flag, void* stream);
// Lanczos start: hist [k][P][2] (alpha_j, beta_{j+1}) -> y [P][k], the unit
// eigenvector of the largest eigenvalue of each row's tridiagonal T (FP64,
// bisection on Sturm counts, then inverse iteration), sign y_0 >= 0.
constexpr int LZ_MAX = 64;
int launch_lz_ritz(const float* hist, int k, int P, double* y, void* stream);
// t[p] <- sum_{j<k} y[p][j] V_j[p] with V_0 = t (in place) and V_j = Vw + (j - 1) P N.
int launch_lz_combine(void* t, const void* Vw, const double* y, int k, int P, int N, void* stream);
// launch_lz_combine followed by launch_row_rescale(mode 1, rowsum, denom)
int launch_lz_combine_scaled(void* t, const void* Vw, const double* y, int k, int P, int N, const double* rowsum,
                             double denom, void* stream);
}  // namespace tmk
