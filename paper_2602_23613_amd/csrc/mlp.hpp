// Learned-setup surrogate network: data layout and launchers (see mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace hamg {

constexpr int MLP_IN = 64, MLP_HID = 128, MLP_OUT = 64, MLP_SMAX = 8;
// FP32 master parameters, concatenated row-major: W1 (64x128), b1, W2 (128x128), b2, W3 (128x64), b3
constexpr int64_t MLP_OFF_W1 = 0;
constexpr int64_t MLP_OFF_B1 = MLP_OFF_W1 + (int64_t)MLP_IN * MLP_HID;
constexpr int64_t MLP_OFF_W2 = MLP_OFF_B1 + MLP_HID;
constexpr int64_t MLP_OFF_B2 = MLP_OFF_W2 + (int64_t)MLP_HID * MLP_HID;
constexpr int64_t MLP_OFF_W3 = MLP_OFF_B2 + MLP_HID;
constexpr int64_t MLP_OFF_B3 = MLP_OFF_W3 + (int64_t)MLP_HID * MLP_OUT;
constexpr int64_t MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;

struct MlpDev {
  float* master = nullptr;   // MLP_NPARAM
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t *Wb1 = nullptr, *Wb2 = nullptr, *Wb3 = nullptr;   // BF16 copies of the weights
  const float* b1 = nullptr;
  const float* b2 = nullptr;
  const float* b3 = nullptr;
  int64_t step = 0;
  bool ready = false;
};

// activations of one batch (rows = padded batch size, a multiple of 16)
struct MlpWork {
  int64_t rows = 0;
  float *Z1 = nullptr, *Z2 = nullptr, *dH = nullptr;
  uint16_t *H1 = nullptr, *H2 = nullptr, *dHb = nullptr, *dYb = nullptr;
};

void gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t lda_m, int64_t lda_k,
               const uint16_t* B, int64_t ldb_k, int64_t ldb_n, float* C, int64_t ldc, int accumulate,
               hipStream_t st);
void mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, MlpWork& w, float* Y, hipStream_t st);
void mlp_backward(const MlpDev& m, const uint16_t* X, int64_t n, MlpWork& w, const float* dY,
                  float* grad, hipStream_t st);
void mlp_refresh_bf16(MlpDev& m, hipStream_t st);
void mlp_adam(MlpDev& m, float lr, hipStream_t st);
void mlp_loss(int64_t n, const float* Y, const float* T, const double* Ahat, const int32_t* ahat_idx,
              int64_t nvalid, float* dY, float* row_loss, hipStream_t st);
void mlp_gather(int64_t n, int64_t npad, const int32_t* idx, const uint16_t* X, const float* T,
                uint16_t* Xb, float* Tb, hipStream_t st);
void block_features(int64_t nb, const int64_t* bptr, const int32_t* bdofs, const int64_t* Aptr,
                    const int32_t* Acol, const double* Aval, double eligible_max, uint16_t* X,
                    float* T, double* Ahat, double* dsq, int8_t* eligible, hipStream_t st);
void refine_check(int64_t nb, const int64_t* bptr, const int8_t* eligible, const float* Y,
                  const double* Ahat, int steps, double tol, double* Wout, int8_t* accepted,
                  float* resid, hipStream_t st);

}  // namespace hamg
