// mlp.h -- layout constants and launch wrappers of the surrogate network.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lensed {

constexpr int MLP_IN = 17, MLP_H = 256, MLP_KPAD = 32;
// flat float32 parameters: W1 [256][17], b1, W2 [256][256], b2, W3 [256][256], b3, W4 [1][256], b4
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H * MLP_H;
constexpr int MLP_OFF_W4 = MLP_OFF_B3 + MLP_H;
constexpr int MLP_OFF_B4 = MLP_OFF_W4 + MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B4 + 1;
static_assert(MLP_NPARAM == 136449, "surrogate parameter count");
// bfloat16 weight copies: W1 padded to [256][32], W2, W3, W4
constexpr long MLP_WB_W2 = (long)MLP_H * MLP_KPAD;
constexpr long MLP_WB_W3 = MLP_WB_W2 + (long)MLP_H * MLP_H;
constexpr long MLP_WB_W4 = MLP_WB_W3 + (long)MLP_H * MLP_H;
constexpr long MLP_WB_SIZE = MLP_WB_W4 + MLP_H;

// Device scratch for batches of at most `cap` rows (owned by the context).
struct MlpScratch {
  int cap = 0;
  uint16_t* wb = nullptr;       // [MLP_WB_SIZE]
  uint16_t* X0 = nullptr;       // [cap][32]
  float* Z[3] = {nullptr, nullptr, nullptr};      // [cap][256]
  uint16_t* H[3] = {nullptr, nullptr, nullptr};   // [cap][256]
  float* d = nullptr;           // [cap]
  float* sq = nullptr;          // [cap]
  float* dZ = nullptr;          // [cap][256]
  float* dZ2 = nullptr;
  uint16_t* dZb = nullptr;
  uint16_t* dZb2 = nullptr;
  float* grad = nullptr;        // [MLP_NPARAM] for the fused train step
};

hipError_t mlp_forward(const float* params, const float* norm, const float* x, float* y, int B, const MlpScratch& s,
                       hipStream_t st);
hipError_t mlp_grad(const float* params, const float* norm, const float* x, const float* yt, int B, float* grad,
                    float* loss, const MlpScratch& s, hipStream_t st);
hipError_t mlp_adam(float* params, const float* grad, float* m, float* v, int n, int step, double lr, double beta1,
                    double beta2, double eps, hipStream_t st);

}  // namespace lensed
