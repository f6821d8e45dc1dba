// mlp.h -- launchers of the triage network's kernels (fp32).  Shapes and the
// flat parameter layout are the ones rc.h documents for rc_mlp_*.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rc.h"

namespace rc {

constexpr int MLP_IN = RC_MLP_IN;        // features per instance
constexpr int MLP_H = RC_MLP_HIDDEN;     // width of both hidden layers
constexpr int MLP_PARAMS = RC_MLP_PARAMS;
constexpr float MLP_B1 = 0.9f, MLP_B2 = 0.999f, MLP_EPS = 1e-8f;  // Adam constants

size_t mlp_ws_bytes(uint32_t n);
hipError_t mlp_forward(const float* theta, const float* X, uint32_t n, float* logits, void* ws, hipStream_t st);
// rows (nullable): the minibatch is rows[0..n) of X and y, else rows 0..n-1
hipError_t mlp_grad(const float* theta, const float* X, const float* y, const uint32_t* rows, uint32_t n,
                    float* grad, float* loss, void* ws, hipStream_t st);
hipError_t mlp_train_step(float* theta, float* m, float* v, uint32_t step, const float* X, const float* y,
                          const uint32_t* rows, uint32_t n, float lr, float* loss, void* ws, hipStream_t st);

}  // namespace rc
