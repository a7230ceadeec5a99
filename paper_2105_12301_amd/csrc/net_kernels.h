// Internal interface of the surrogate-network kernels (net.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace edm {

// Flat parameter layout: w1[C][1][KW], b1[C], w2[C][C][KW], b2[C],
// w3[C][C][KW], b3[C], wo[20][C], bo[20].
struct NetParams {
  const float *w1, *b1, *w2, *b2, *w3, *b3, *wo, *bo;
};

constexpr int kNetSlices = 64;  // (series, time) slices of the weight-gradient reduction

int64_t net_param_count(int C);
NetParams net_params(const float *theta, int C);
// Workspace (floats) of one forward/backward pass over B series of length L.
int64_t net_workspace_floats(int C, int64_t B, int64_t L);

hipError_t net_forward(const float *theta, int C, const float *X, int64_t B, int64_t L,
                       int64_t ldx, float *ws, float *logits, hipStream_t st);
// Inference with the C -> C convolutions on BF16 matrix cores (C = 32 or 64);
// uses the first 3 B C L + B C floats of ws plus 2 C C KW BF16 weights.
hipError_t net_forward_bf16(const float *theta, int C, const float *X, int64_t B, int64_t L,
                            int64_t ldx, float *ws, float *logits, hipStream_t st);
hipError_t net_loss_grad(const float *theta, int C, const float *X, const int32_t *labels,
                         int64_t B, int64_t L, int64_t ldx, float *ws, float *loss,
                         float *grad, hipStream_t st);
hipError_t net_adam(float *p, const float *g, float *m, float *v, int64_t n, int step, float lr,
                    float b1, float b2, float eps, hipStream_t st);

}  // namespace edm
