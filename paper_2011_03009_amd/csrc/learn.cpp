// C ABI of the truncation-box tools (localisation boxes, truncated focal
// potentials) and of the learned box predictor.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "../../include/nvp.h"
#include "boxnet.hpp"
#include "qbox.hpp"

static_assert(NVP_BOXNET_PARAMS == BOXNET_PARAMS, "parameter count of the header and the kernels");
static_assert(NVP_BOXNET_IN == BOXNET_IN && NVP_BOXNET_OUT == BOXNET_OUT, "network shape");
static_assert(NVP_QBOX_MAX_COUNT == NVP_QBOX_MAX, "box count limit");

namespace nvp {
int ctx_device(const nvp_ctx *c);
void ctx_attach(nvp_ctx *c);  // a network made with the context, until its destroy call
void ctx_detach(nvp_ctx *c);
hipStream_t ctx_stream(const nvp_ctx *c);
nvp_status ctx_fail(nvp_ctx *c, nvp_status s, const char *msg);
nvp_status ctx_hip_fail(nvp_ctx *c, const char *what, hipError_t e);
void ctx_quad_weights(const nvp_ctx *c, double kr, double ki, double h, double *sr, double *si, double *fr,
                      double *fi);
}  // namespace nvp

using nvp::ctx_fail;
using nvp::ctx_hip_fail;

#define LRN_HIP(ctx, call)                                           \
    do {                                                             \
        hipError_t _e = (call);                                      \
        if (_e != hipSuccess) return ctx_hip_fail((ctx), #call, _e); \
    } while (0)

struct nvp_boxnet {
    nvp_ctx *ctx = nullptr;
    int max_batch = 0;
    int step = 0;  // Adam steps taken since the parameters were set
    void *blob = nullptr;
    nvp::BoxnetBufs w{};
};

namespace {

bool dims_ok(const int64_t n[3]) {
    return n && n[0] > 0 && n[1] > 0 && n[2] > 0 && n[0] < (1 << 30) && n[1] < (1 << 30) && n[2] < (1 << 30);
}

// Scratch of the box reductions, allocated per call (the calls are host-side
// steps of a sweep, not the convolution's hot loop).
struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

nvp_status nvp_qbox(nvp_ctx *ctx, const int64_t n[3], const void *f_dev, nvp_prec prec, int count, const double *q0,
                    int64_t *box) {
    if (!ctx) return NVP_E_INVALID;
    if (!dims_ok(n) || !f_dev || !q0 || !box || count < 1 || count > NVP_QBOX_MAX ||
        (prec != NVP_C64 && prec != NVP_C128))
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_qbox: bad argument");
    double frac[NVP_QBOX_MAX];
    for (int i = 0; i < count; ++i) {
        if (!std::isfinite(q0[i]) || q0[i] > 0.0) return ctx_fail(ctx, NVP_E_INVALID, "nvp_qbox: Q0 must be <= 0");
        frac[i] = std::pow(10.0, 2.0 * q0[i]);
    }
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    DevBuf buf;
    const size_t wbytes = 1025 * sizeof(double), fbytes = NVP_QBOX_MAX * sizeof(double);
    LRN_HIP(ctx, hipMalloc(&buf.p, wbytes + fbytes + NVP_QBOX_MAX * 6 * sizeof(int)));
    double *work = static_cast<double *>(buf.p);
    double *frac_dev = reinterpret_cast<double *>(static_cast<char *>(buf.p) + wbytes);
    int *box_dev = reinterpret_cast<int *>(static_cast<char *>(buf.p) + wbytes + fbytes);
    LRN_HIP(ctx, hipMemcpyAsync(frac_dev, frac, count * sizeof(double), hipMemcpyHostToDevice, s));
    LRN_HIP(ctx, nvp::qbox_launch(f_dev, prec == NVP_C128, n, count, frac_dev, work, box_dev, s));
    int hb[NVP_QBOX_MAX * 6];
    LRN_HIP(ctx, hipMemcpyAsync(hb, box_dev, count * 6 * sizeof(int), hipMemcpyDeviceToHost, s));
    LRN_HIP(ctx, hipStreamSynchronize(s));
    for (int i = 0; i < count * 6; ++i) box[i] = hb[i];
    return NVP_OK;
}

nvp_status nvp_box_potential(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev,
                             nvp_prec prec, const int64_t t[3], int count, const int64_t *box, double *out) {
    if (!ctx) return NVP_E_INVALID;
    if (!g || !dims_ok(g->n) || !(g->h > 0) || !std::isfinite(g->h) || !f_dev || !t || !box || !out || count < 1 ||
        count > NVP_QBOX_MAX || (prec != NVP_C64 && prec != NVP_C128) || !std::isfinite(k_re) ||
        !std::isfinite(k_im) || k_im < 0)
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_box_potential: bad argument");
    int ti[3], hb[NVP_QBOX_MAX * 6];
    for (int a = 0; a < 3; ++a) {
        if (t[a] < 0 || t[a] >= g->n[a]) return ctx_fail(ctx, NVP_E_INVALID, "nvp_box_potential: target outside grid");
        ti[a] = (int)t[a];
    }
    for (int q = 0; q < count; ++q)
        for (int a = 0; a < 3; ++a) {
            const int64_t lo = box[q * 6 + a], hi = box[q * 6 + 3 + a];
            if (hi >= lo && (lo < 0 || hi >= g->n[a]))
                return ctx_fail(ctx, NVP_E_INVALID, "nvp_box_potential: box outside the grid");
            // an empty box (hi < lo on some axis) is normalised to an empty index range
            hb[q * 6 + a] = hi >= lo ? (int)lo : 0;
            hb[q * 6 + 3 + a] = hi >= lo ? (int)hi : -1;
        }
    double sr, si, fr, fi;  // self voxel and face-neighbour addition of the context's quadrature rule
    nvp::ctx_quad_weights(ctx, k_re, k_im, g->h, &sr, &si, &fr, &fi);
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    DevBuf buf;
    const size_t wbytes = (size_t)NVP_BOXSUM_BLOCKS * count * sizeof(double2), obytes = count * sizeof(double2);
    LRN_HIP(ctx, hipMalloc(&buf.p, wbytes + obytes + NVP_QBOX_MAX * 6 * sizeof(int)));
    double2 *work = static_cast<double2 *>(buf.p);
    double2 *out_dev = reinterpret_cast<double2 *>(static_cast<char *>(buf.p) + wbytes);
    int *box_dev = reinterpret_cast<int *>(static_cast<char *>(buf.p) + wbytes + obytes);
    LRN_HIP(ctx, hipMemcpyAsync(box_dev, hb, count * 6 * sizeof(int), hipMemcpyHostToDevice, s));
    LRN_HIP(ctx, nvp::boxsum_launch(f_dev, prec == NVP_C128, g->n, ti, g->h, k_re, k_im, sr, si, fr, fi, box_dev,
                                    count, work, out_dev, s));
    LRN_HIP(ctx, hipMemcpyAsync(out, out_dev, obytes, hipMemcpyDeviceToHost, s));
    LRN_HIP(ctx, hipStreamSynchronize(s));
    return NVP_OK;
}

// ---------------------------------------------------------------- box predictor

nvp_status nvp_boxnet_create(nvp_ctx *ctx, int max_batch, nvp_boxnet **out) {
    if (!ctx) return NVP_E_INVALID;
    if (!out || max_batch < 1 || max_batch > NVP_BOXNET_MAX_BATCH)
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_create: bad argument");
    *out = nullptr;
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    const size_t P = BOXNET_PARAMS, B = (size_t)max_batch, H = BOXNET_HIDDEN;
    // params, grad, m, v | norm | a0 | h1 h2 h3 | y | d1 d2 d3 | d4 | lossb | loss
    const size_t nfloat = 4 * P + 2 * BOXNET_IN + B * BOXNET_IN + 3 * B * H + B * BOXNET_OUT + 3 * B * H +
                          B * BOXNET_OUT + B + 1;
    nvp_boxnet *bn = new (std::nothrow) nvp_boxnet;
    if (!bn) return ctx_fail(ctx, NVP_E_NOMEM, "nvp_boxnet_create: allocation");
    hipError_t e = hipMalloc(&bn->blob, nfloat * sizeof(float));
    if (e != hipSuccess) {
        delete bn;
        return ctx_hip_fail(ctx, "nvp_boxnet_create: hipMalloc", e);
    }
    float *f = static_cast<float *>(bn->blob);
    nvp::BoxnetBufs &w = bn->w;
    w.params = f; f += P;
    w.grad = f; f += P;
    w.m = f; f += P;
    w.v = f; f += P;
    w.norm = f; f += 2 * BOXNET_IN;
    w.a0 = f; f += B * BOXNET_IN;
    w.h1 = f; f += B * H;
    w.h2 = f; f += B * H;
    w.h3 = f; f += B * H;
    w.y = f; f += B * BOXNET_OUT;
    w.d1 = f; f += B * H;
    w.d2 = f; f += B * H;
    w.d3 = f; f += B * H;
    w.d4 = f; f += B * BOXNET_OUT;
    w.lossb = f; f += B;
    w.loss = f;
    bn->ctx = ctx;
    bn->max_batch = max_batch;
    hipStream_t s = nvp::ctx_stream(ctx);
    float norm[2 * BOXNET_IN];
    for (int i = 0; i < BOXNET_IN; ++i) {
        norm[i] = 0.0f;
        norm[BOXNET_IN + i] = 1.0f;
    }
    e = hipMemsetAsync(bn->blob, 0, 4 * P * sizeof(float), s);
    if (e == hipSuccess) e = hipMemcpyAsync(w.norm, norm, sizeof(norm), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(bn->blob);
        delete bn;
        return ctx_hip_fail(ctx, "nvp_boxnet_create: initialisation", e);
    }
    nvp::ctx_attach(ctx);
    *out = bn;
    return NVP_OK;
}

nvp_status nvp_boxnet_set_params(nvp_boxnet *bn, const float *params, int64_t n) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (!params || n != BOXNET_PARAMS) return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_set_params: bad argument");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_set_params: non-finite value");
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    LRN_HIP(ctx, hipMemcpyAsync(bn->w.params, params, n * sizeof(float), hipMemcpyHostToDevice, s));
    LRN_HIP(ctx, hipMemsetAsync(bn->w.m, 0, 2 * (size_t)BOXNET_PARAMS * sizeof(float), s));
    LRN_HIP(ctx, hipStreamSynchronize(s));
    bn->step = 0;
    return NVP_OK;
}

nvp_status nvp_boxnet_get_params(nvp_boxnet *bn, float *params, int64_t n) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (!params || n != BOXNET_PARAMS) return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_get_params: bad argument");
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    LRN_HIP(ctx, hipMemcpyAsync(params, bn->w.params, n * sizeof(float), hipMemcpyDeviceToHost, s));
    LRN_HIP(ctx, hipStreamSynchronize(s));
    return NVP_OK;
}

nvp_status nvp_boxnet_set_norm(nvp_boxnet *bn, const float *mean, const float *stdev) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (!mean || !stdev) return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_set_norm: bad argument");
    float norm[2 * BOXNET_IN];
    for (int i = 0; i < BOXNET_IN; ++i) {
        if (!std::isfinite(mean[i]) || !std::isfinite(stdev[i]) || !(stdev[i] > 0.0f))
            return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_set_norm: need finite means and positive deviations");
        norm[i] = mean[i];
        norm[BOXNET_IN + i] = stdev[i];
    }
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    LRN_HIP(ctx, hipMemcpyAsync(bn->w.norm, norm, sizeof(norm), hipMemcpyHostToDevice, s));
    LRN_HIP(ctx, hipStreamSynchronize(s));
    return NVP_OK;
}

nvp_status nvp_boxnet_predict(nvp_boxnet *bn, int batch, const float *x_dev, float *y_dev) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (batch < 1 || batch > bn->max_batch || !x_dev || !y_dev)
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_predict: bad argument");
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    LRN_HIP(ctx, nvp::boxnet_forward(bn->w, batch, x_dev, y_dev, nvp::ctx_stream(ctx)));
    return NVP_OK;
}

nvp_status nvp_boxnet_grads(nvp_boxnet *bn, int batch, const float *x_dev, const float *t_dev, float tau,
                            float *grad_dev, float *loss_host) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (batch < 1 || batch > bn->max_batch || !x_dev || !t_dev || !grad_dev || !(tau > 0.0f && tau < 1.0f))
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_grads: bad argument");
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    LRN_HIP(ctx, nvp::boxnet_backward(bn->w, batch, x_dev, t_dev, tau, grad_dev, bn->w.loss, s));
    if (loss_host) {
        LRN_HIP(ctx, hipMemcpyAsync(loss_host, bn->w.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        LRN_HIP(ctx, hipStreamSynchronize(s));
    }
    return NVP_OK;
}

nvp_status nvp_boxnet_train_step(nvp_boxnet *bn, int batch, const float *x_dev, const float *t_dev, float tau,
                                 float lr, float *loss_host) {
    if (!bn) return NVP_E_INVALID;
    nvp_ctx *ctx = bn->ctx;
    if (batch < 1 || batch > bn->max_batch || !x_dev || !t_dev || !(tau > 0.0f && tau < 1.0f) ||
        !std::isfinite(lr) || lr < 0.0f)
        return ctx_fail(ctx, NVP_E_INVALID, "nvp_boxnet_train_step: bad argument");
    LRN_HIP(ctx, hipSetDevice(nvp::ctx_device(ctx)));
    hipStream_t s = nvp::ctx_stream(ctx);
    LRN_HIP(ctx, nvp::boxnet_backward(bn->w, batch, x_dev, t_dev, tau, bn->w.grad, bn->w.loss, s));
    LRN_HIP(ctx, nvp::boxnet_adam(bn->w, lr, NVP_BOXNET_BETA1, NVP_BOXNET_BETA2, NVP_BOXNET_EPS, bn->step + 1, s));
    bn->step += 1;
    if (loss_host) {
        LRN_HIP(ctx, hipMemcpyAsync(loss_host, bn->w.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        LRN_HIP(ctx, hipStreamSynchronize(s));
    }
    return NVP_OK;
}

nvp_status nvp_boxnet_destroy(nvp_boxnet *bn) {
    if (!bn) return NVP_E_INVALID;
    (void)hipSetDevice(nvp::ctx_device(bn->ctx));
    (void)hipStreamSynchronize(nvp::ctx_stream(bn->ctx));
    if (bn->blob) (void)hipFree(bn->blob);
    nvp::ctx_detach(bn->ctx);
    delete bn;
    return NVP_OK;
}

}  // extern "C"
