// Device buffers and launchers of the box-predictor MLP (boxnet.hip).
#pragma once

#include <hip/hip_runtime.h>

#define BOXNET_IN 5
#define BOXNET_HIDDEN 64
#define BOXNET_OUT 3
#define BOXNET_PARAMS (64 * 5 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 3 * 64 + 3)

namespace nvp {

struct BoxnetBufs {
    float *params, *grad, *m, *v;  // BOXNET_PARAMS each
    float *norm;                   // input mean[5], std[5]
    float *a0, *h1, *h2, *h3, *y;  // activations, sample-major, max_batch rows
    float *d1, *d2, *d3, *d4;      // deltas
    float *lossb, *loss;           // per-sample loss terms, their sum
};

hipError_t boxnet_forward(const BoxnetBufs &w, int B, const float *x, float *y, hipStream_t s);
// Forward + deltas + weight gradients into grad; loss sum into loss_dev.
hipError_t boxnet_backward(const BoxnetBufs &w, int B, const float *x, const float *t, float tau, float *grad,
                           float *loss_dev, hipStream_t s);
hipError_t boxnet_adam(const BoxnetBufs &w, float lr, float b1, float b2, float eps, int step, hipStream_t s);

}  // namespace nvp
