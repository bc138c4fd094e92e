// Internal interface of the run-time model (MLP) kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mpg {

constexpr int kMlpHidden = 64;
constexpr int kMlpMaxFeatures = 32;
constexpr int kMlpChunk = 16;   // rows per gradient workgroup

int mlp_num_params(int F);
int mlp_grad_chunks(int rows);
hipError_t launch_mlp_forward(const float* prm, const float* X, int rows, int F, float* out,
                              hipStream_t s);
// partial: mlp_grad_chunks(rows) x (P + 1) floats; grad: P + 1 floats
// (grad[P] = mean squared residual); losses (nullable) gets grad[P] at epoch.
hipError_t launch_mlp_grad(const float* prm, const float* X, const float* t, int rows, int F,
                           float* partial, float* grad, float* losses, int epoch, hipStream_t s);
hipError_t launch_mlp_adam(float* prm, const float* grad, float* m, float* v, int P, float lr,
                           int step, hipStream_t s);

}  // namespace mpg
