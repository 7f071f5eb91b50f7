// Learned start network (BF16 MFMA GEMMs, FP32 accumulation and master weights).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace tmk {

enum MlpEpi { MLP_EPI_STORE = 0, MLP_EPI_BIAS = 1, MLP_EPI_BIAS_GELU = 2, MLP_EPI_GELU_BWD = 3 };

struct MlpShape {
  int n_in, hidden, n_out;  // K N, hidden width, 2 N
};

struct MlpParams {
  float* W[3];      // FP32 master weights, W[l] is [fan_in][fan_out] row-major
  uint16_t* Wh[3];  // BF16 copies used by the GEMMs
  float* b[3];      // FP32 biases
};

struct MlpGrads {
  float* dW[3];
  float* db[3];
};

struct MlpAdam {
  float* mW[3];
  float* vW[3];
  float* mb[3];
  float* vb[3];
};

struct MlpWork {
  uint16_t* X;
  float* s;
  float *A1, *A2;
  uint16_t *H1, *H2;
  float* O;
  uint16_t* dOh;
  float* dOf;
  uint16_t *dA2h, *dA1h;
  float *dA2f, *dA1f;
  float* loss;
};

size_t mlp_work_bytes(const MlpShape& sh, int B);
void mlp_work_carve(void* base, const MlpShape& sh, int B, MlpWork* w);
// features, three layers; outputs in w.O (FP32 [B][n_out]) and the row scales w.s
int mlp_forward(const MlpShape& sh, const MlpParams& P, const float* I, int B, int KN, MlpWork& w, void* stream);
// the three layers from features already in w.X (BF16 [B][n_in]); outputs in w.O
int mlp_forward_x(const MlpShape& sh, const MlpParams& P, int B, MlpWork& w, void* stream);
// all parameter gradients from output gradients already in w.dOh / w.dOf (after a forward)
int mlp_backward_dout(const MlpShape& sh, const MlpParams& P, int B, MlpWork& w, MlpGrads& G, void* stream);
// start rows t0 [P][N] complex from w.O and w.s
int mlp_start(const MlpWork& w, int P, int N, void* t0, void* stream);
// loss per row into w.loss and all parameter gradients (after mlp_forward)
int mlp_backward(const MlpShape& sh, const MlpParams& P, const void* t, int B, MlpWork& w, MlpGrads& G,
                 void* stream);
int mlp_adam(const MlpShape& sh, MlpParams& P, const MlpGrads& G, MlpAdam& A, float lr, int step, void* stream);
int mlp_weights_to_bf16(const MlpShape& sh, MlpParams& P, void* stream);
// plain GEMM C = op(A) op(B) (FP32 out), for tests of the MFMA tile
int gemm_bf16(int M, int N, int K, const uint16_t* A, int ta, const uint16_t* B, int tb, float* C, void* stream);

}  // namespace tmk
