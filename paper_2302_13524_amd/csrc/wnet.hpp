// Learned weighting of the spectral start: helper kernels (wnet_kernels.hip).
#pragma once
#include <stdint.h>

namespace tmk {

constexpr int WNET_FEATURES = 64;  // network inputs per table point

// X [nt][64] BF16 features of the table points x_b = b xmax / (nt - 1)
int wnet_features(int nt, float xmax, uint16_t* X, void* stream);
// network outputs O [nt] -> table [nt][2] (T_b, T_{b+1} - T_b)
int wnet_pairs(const float* O, int nt, float* tab, void* stream);
// u = y / ||y|| per row (||y||^2 at sums[p * nsum]); n [P] receives ||y||
int wnet_normalise(const void* y, const float* sums, int nsum, int P, int N, void* u, float* n, void* stream);
// per-row fidelity of u to t, the packed gradient G of minus their mean, and that mean loss [1]
int wnet_loss(const void* u, const void* t, int P, int N, void* G, float* fid, float* loss, void* stream);
// G_y = (G_u - Re(u^H G_u) u) / n
int wnet_normback(const void* Gu, const void* u, const float* n, int P, int N, void* Gy, void* stream);
// dtab [nt] += adjoint of the table lookup applied to gw [P][KN] (intensities I, row means)
int wnet_hist(const float* gw, const void* I, int ibf16, const float* rowmean, int P, int KN, int nt, float xmax,
              float* dtab, void* stream);
// W [P][KN] = T(I / mean_p), the learned weights of every measurement, from the table [nt][2]
int wnet_weights(const void* I, int ibf16, const float* rowmean, int P, int64_t KN, const float* tab, int nt,
                 float xmax, float* W, void* stream);
// warm-start regression of the outputs onto min(x, tau): dO (FP32, BF16) and the mean squared error [1]
int wnet_regress(const float* O, int nt, float xmax, float tau, float* dOf, uint16_t* dOh, float* loss, void* stream);
// dO (FP32, BF16) = dtab
int wnet_dout(const float* dtab, int nt, float* dOf, uint16_t* dOh, void* stream);

}  // namespace tmk
