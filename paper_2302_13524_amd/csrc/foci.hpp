// Conjugate-phase foci of retrieved TM rows and their power ratio (Sec. 3).
#pragma once
#include <stdint.h>

namespace tmk {

// u[p][n] = exp(-j arg tm_est[p][n]) (1 where tm_est is 0), [P][N] complex float
int launch_conj_phase(const void* tm_est, void* u, int64_t n, void* stream);
// For every focus p (row p of E [Pf][G] complex, E[p][q] = sum_n u[p][n] tm_true[q][n]):
// peak = brightest pixel (first in raster order on ties), PR = power in the
// (2w+1)^2 grid window around the peak / total power. pix [G] raster indices
// on a g1 x g2 grid.
int launch_foci_pr(const void* E, int Pf, int G, const int32_t* pix, int g1, int g2, int w, float* pr, int32_t* peak,
                   void* stream);

}  // namespace tmk

namespace tmk {
// Dense-probing gradient helpers (the Theta(M N) comparator without FFTs):
// given Y [P][M] = Q t, w[p][i] = -4 conj(Y (I - |Y|^2)) in place and f[p] = sum (I - |Y|^2)^2;
// afterwards grad = conj(H) in place.
int launch_dense_pointwise(void* Y, const float* I, int P, int64_t M, float* f, void* stream);
int launch_conj_inplace(void* x, int64_t n, void* stream);
// C [M][N] = A [M][K] op(B) in complex FP32 on the matrix cores: B is [N][K]
// (trans_b) or [K][N]; conj_c stores conj(C). hipErrorInvalidValue on bad sizes.
int launch_cgemm(int M, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb, int trans_b, void* C,
                 int64_t ldc, int conj_c, void* stream);
}  // namespace tmk

namespace tmk {
// Propagated TM helpers: X [N][G] = columns of tm [P][N] on the grid (pix [P], zero elsewhere);
// H [g1 g2] angular-spectrum kernel; out [G][N] = X^T.
int launch_cols_to_grid(const void* tm, int P, int N, const int32_t* pix, int G, void* X, void* stream);
int launch_make_prop_filter(void* H, int g1, int g2, double lam, double ps, double NA, double z, void* stream);
int launch_fill_c32(void* x, int64_t n, float re, float im, void* stream);
int launch_grid_to_rows(const void* X, int N, int G, void* out, void* stream);
}  // namespace tmk
