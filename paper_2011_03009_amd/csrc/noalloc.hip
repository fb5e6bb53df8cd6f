// The volume potential for callers that cannot allocate device memory: its
// work buffers (the kernel-spectrum octant and the two pass buffers of the
// circulant convolution) live in one fixed device array, `scratch`, instead
// of memory the library allocates.
//
// The array's name in host code is only a host-side stand-in for the device
// symbol; its device address is looked up once per device, at context
// creation with that device current (noalloc_setup), and only that address
// is handed to kernels.  Every call on a device uses that device's one copy
// of the array, so calls that overlap on one GPU race; calls enqueued on one
// stream run one after another.  Each call writes every scratch byte it later
// reads (the spectrum pass writes the whole octant it multiplies by, the
// passes write every row the next pass reads), so nothing needs clearing and
// the contents a previous call left are never used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/nvp.h"

namespace nvp {
int ctx_device(const nvp_ctx *c);
nvp_status ctx_fail(nvp_ctx *c, nvp_status s, const char *msg);
nvp_status ctx_hip_fail(nvp_ctx *c, const char *what, hipError_t e);
nvp_status vp_buffers(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev, void *u_dev,
                      nvp_prec prec, size_t bytes[3], void *khat, void *A, void *B);
}  // namespace nvp

namespace {

static __device__ __align__(256) unsigned char scratch[NVP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once set up

size_t round256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

namespace nvp {

// Called by nvp_ctx_create with the context's device current.
nvp_status noalloc_setup(nvp_ctx *ctx) {
    const int d = ctx_device(ctx);
    if (d < 0 || d >= kMaxDevices) return ctx_fail(ctx, NVP_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[d]) return NVP_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return ctx_hip_fail(ctx, "hipGetSymbolAddress(scratch)", e);
    if (!p) return ctx_fail(ctx, NVP_E_HIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch[d] = p;
    return NVP_OK;
}

}  // namespace nvp

extern "C" nvp_status nvp_volume_potential_noalloc(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g,
                                                   const void *f_dev, void *u_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    size_t b[3];
    nvp_status st = nvp::vp_buffers(ctx, k_re, k_im, g, f_dev, u_dev, prec, b, nullptr, nullptr, nullptr);
    if (st) return st;
    const size_t o1 = round256(b[0]), o2 = o1 + round256(b[1]), need = o2 + round256(b[2]);
    if (need > (size_t)NVP_NOALLOC_SCRATCH_BYTES) {
        const std::string msg = "nvp_volume_potential_noalloc: this grid needs " + std::to_string(need) +
                                " bytes of scratch; the fixed scratch holds " +
                                std::to_string((size_t)NVP_NOALLOC_SCRATCH_BYTES);
        return nvp::ctx_fail(ctx, NVP_E_UNSUPPORTED, msg.c_str());
    }
    const int d = nvp::ctx_device(ctx);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (d >= 0 && d < kMaxDevices) base = g_scratch[d];
    }
    if (!base) return nvp::ctx_fail(ctx, NVP_E_STATE, "nvp_volume_potential_noalloc: scratch not set up");
    unsigned char *p = static_cast<unsigned char *>(base);
    return nvp::vp_buffers(ctx, k_re, k_im, g, f_dev, u_dev, prec, b, p, p + o1, p + o2);
}
