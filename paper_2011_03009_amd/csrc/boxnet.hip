// Learned truncation-box predictor: a 5-64-64-64-3 tanh MLP in plain FP32
// (no MFMA: the network is tiny and latency-bound).  Kernels for the forward
// pass, the per-sample back-propagated deltas of a pinball (quantile) loss,
// the batch-summed weight gradients (fixed summation order, no atomics, so
// results repeat bitwise) and the Adam update.
//
// Parameter layout (float, row-major W[out][in]):
//   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3]
// Activations and deltas are stored sample-major: a[b][unit].
#include <hip/hip_runtime.h>
#include <math.h>

#include "boxnet.hpp"

namespace nvp {

namespace {

constexpr int I = BOXNET_IN, H = BOXNET_HIDDEN, O = BOXNET_OUT;
constexpr int OW1 = 0, OB1 = OW1 + H * I, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H * H,
              OW4 = OB3 + H, OB4 = OW4 + O * H, NP = OB4 + O;
static_assert(NP == BOXNET_PARAMS, "parameter count");

__device__ __forceinline__ void stage(float *dst, const float *src, int n) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// x: [B][5] raw inputs; writes a0 [B][5] (standardised), h1..h3 [B][64], y [B][3].
__global__ void __launch_bounds__(64) k_fwd(const float *__restrict__ p, const float *__restrict__ norm, int B,
                                            const float *__restrict__ x, float *__restrict__ a0,
                                            float *__restrict__ h1, float *__restrict__ h2, float *__restrict__ h3,
                                            float *__restrict__ y) {
    __shared__ float w[NP];
    stage(w, p, NP);
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float a[I];
#pragma unroll
    for (int j = 0; j < I; ++j) {
        a[j] = (x[b * I + j] - norm[j]) / norm[I + j];
        a0[b * I + j] = a[j];
    }
    float u[H], v[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float s = w[OB1 + i];
#pragma unroll
        for (int j = 0; j < I; ++j) s += w[OW1 + i * I + j] * a[j];
        u[i] = tanhf(s);
    }
#pragma unroll
    for (int i = 0; i < H; ++i) h1[(size_t)b * H + i] = u[i];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float s = w[OB2 + i];
#pragma unroll
        for (int j = 0; j < H; ++j) s += w[OW2 + i * H + j] * u[j];
        v[i] = tanhf(s);
    }
#pragma unroll
    for (int i = 0; i < H; ++i) h2[(size_t)b * H + i] = v[i];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        float s = w[OB3 + i];
#pragma unroll
        for (int j = 0; j < H; ++j) s += w[OW3 + i * H + j] * v[j];
        u[i] = tanhf(s);
    }
#pragma unroll
    for (int i = 0; i < H; ++i) h3[(size_t)b * H + i] = u[i];
#pragma unroll
    for (int k = 0; k < O; ++k) {
        float s = w[OB4 + k];
#pragma unroll
        for (int j = 0; j < H; ++j) s += w[OW4 + k * H + j] * u[j];
        y[b * O + k] = s;
    }
}

// Pinball loss of quantile tau on the mean over B samples and 3 outputs:
// L = (1 / 3B) sum rho(t - y), rho(u) = u (tau - [u < 0]).  Per sample: the loss
// term and the deltas d4 = dL/dy, d3, d2, d1 (through tanh' = 1 - h^2).
__global__ void __launch_bounds__(64) k_delta(const float *__restrict__ p, int B, float tau,
                                              const float *__restrict__ h1, const float *__restrict__ h2,
                                              const float *__restrict__ h3, const float *__restrict__ y,
                                              const float *__restrict__ t, float *__restrict__ d1,
                                              float *__restrict__ d2, float *__restrict__ d3,
                                              float *__restrict__ d4, float *__restrict__ loss) {
    __shared__ float w[NP];
    stage(w, p, NP);
    __syncthreads();
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float sc = 1.0f / (3.0f * (float)B);
    float e[O], l = 0.0f;
#pragma unroll
    for (int k = 0; k < O; ++k) {
        const float u = t[b * O + k] - y[b * O + k];
        l += u * (tau - (u < 0.0f ? 1.0f : 0.0f));
        e[k] = -(tau - (u < 0.0f ? 1.0f : 0.0f)) * sc;
        d4[b * O + k] = e[k];
    }
    loss[b] = l * sc;
    float g3[H], g2[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < O; ++k) s += w[OW4 + k * H + j] * e[k];
        const float h = h3[(size_t)b * H + j];
        g3[j] = s * (1.0f - h * h);
        d3[(size_t)b * H + j] = g3[j];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) s += w[OW3 + i * H + j] * g3[i];
        const float h = h2[(size_t)b * H + j];
        g2[j] = s * (1.0f - h * h);
        d2[(size_t)b * H + j] = g2[j];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < H; ++i) s += w[OW2 + i * H + j] * g2[i];
        const float h = h1[(size_t)b * H + j];
        d1[(size_t)b * H + j] = s * (1.0f - h * h);
    }
}

// One thread per parameter: gradient = sum over b (in order) of delta[b][i] * input[b][j].
__global__ void __launch_bounds__(256) k_wgrad(int B, const float *__restrict__ a0, const float *__restrict__ h1,
                                               const float *__restrict__ h2, const float *__restrict__ h3,
                                               const float *__restrict__ d1, const float *__restrict__ d2,
                                               const float *__restrict__ d3, const float *__restrict__ d4,
                                               float *__restrict__ g) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NP) return;
    const float *dl, *in;
    int nd, ni, i, j;  // delta width, input width, row, column (j < 0: bias)
    if (q < OB1) { dl = d1; nd = H; in = a0; ni = I; i = (q - OW1) / I; j = (q - OW1) % I; }
    else if (q < OW2) { dl = d1; nd = H; in = nullptr; ni = 0; i = q - OB1; j = -1; }
    else if (q < OB2) { dl = d2; nd = H; in = h1; ni = H; i = (q - OW2) / H; j = (q - OW2) % H; }
    else if (q < OW3) { dl = d2; nd = H; in = nullptr; ni = 0; i = q - OB2; j = -1; }
    else if (q < OB3) { dl = d3; nd = H; in = h2; ni = H; i = (q - OW3) / H; j = (q - OW3) % H; }
    else if (q < OW4) { dl = d3; nd = H; in = nullptr; ni = 0; i = q - OB3; j = -1; }
    else if (q < OB4) { dl = d4; nd = O; in = h3; ni = H; i = (q - OW4) / H; j = (q - OW4) % H; }
    else { dl = d4; nd = O; in = nullptr; ni = 0; i = q - OB4; j = -1; }
    float s = 0.0f;
    if (j < 0) {
        for (int b = 0; b < B; ++b) s += dl[(size_t)b * nd + i];
    } else {
        for (int b = 0; b < B; ++b) s += dl[(size_t)b * nd + i] * in[(size_t)b * ni + j];
    }
    g[q] = s;
}

__global__ void __launch_bounds__(256) k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NP) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Sum of the per-sample losses in order (one thread; B is at most a few thousand).
__global__ void k_sum(const float *__restrict__ l, int B, float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int b = 0; b < B; ++b) s += l[b];
        *out = s;
    }
}

}  // namespace

hipError_t boxnet_forward(const BoxnetBufs &w, int B, const float *x, float *y, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd, dim3((B + 63) / 64), dim3(64), 0, s, w.params, w.norm, B, x, w.a0, w.h1, w.h2, w.h3,
                       y);
    return hipGetLastError();
}

hipError_t boxnet_backward(const BoxnetBufs &w, int B, const float *x, const float *t, float tau, float *grad,
                           float *loss_dev, hipStream_t s) {
    hipError_t e = boxnet_forward(w, B, x, w.y, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_delta, dim3((B + 63) / 64), dim3(64), 0, s, w.params, B, tau, w.h1, w.h2, w.h3, w.y, t,
                       w.d1, w.d2, w.d3, w.d4, w.lossb);
    hipLaunchKernelGGL(k_wgrad, dim3((NP + 255) / 256), dim3(256), 0, s, B, w.a0, w.h1, w.h2, w.h3, w.d1, w.d2,
                       w.d3, w.d4, grad);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1), 0, s, w.lossb, B, loss_dev);
    return hipGetLastError();
}

hipError_t boxnet_adam(const BoxnetBufs &w, float lr, float b1, float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, s, w.params, w.grad, w.m, w.v, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace nvp
