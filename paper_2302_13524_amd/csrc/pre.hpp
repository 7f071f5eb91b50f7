// Preprocessing of the camera image stack (Sec. 2.2, the paragraph after
// Algorithm 1): half-sampling, fiber mask, per-pixel rows. Device code in
// pre_kernels.hip; host validation in tm_api.hip.
#pragma once
#include <stdint.h>

namespace tmk {

constexpr int PRE_MASK_MAX = 8192;  // half-sampled pixels the one-workgroup mask kernel sorts in LDS

// partial[c][q] = sum over the images of chunk c of stack[i][2y][2x], q = y (W/2) + x (FP64);
// nchunks = pre_energy_chunks(...). u16: 1 for uint16 pixels, 0 for float.
int pre_energy_chunks(const void* stack, int u16, int64_t n_img, int H, int W);
int launch_pre_energy(const void* stack, int u16, int64_t n_img, int H, int W, double* partial, int nchunks,
                      double* energy, void* stream);
// Brightest-first mask reaching frac of the total; pix[0..count) ascending, count into *count_dev.
int launch_pre_mask(const double* energy, int npix, double frac, int32_t* pix, int32_t* count_dev, void* stream);
// out[p][i] = stack[i][2y_p][2x_p] as float (out_bf16 = 0) or bfloat16 bits (1).
int launch_pre_gather(const void* stack, int u16, int64_t n_img, int H, int W, const int32_t* pix, int P, void* out,
                      int out_bf16, void* stream);

}  // namespace tmk
