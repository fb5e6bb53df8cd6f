// The incident (first-harmonic) field of a transducer modelled as equal-weight
// point sources on its surface (Section 3.2, the incident-field equation:
// a weighted sum of free-space Green's functions exp(i k r) / (4 pi r) over
// the surface points), evaluated at the voxel centres of a grid.  This is the
// input p_1 of the harmonic cascade and, on the paper's CPU, the most
// expensive step of the method (Section 6, timing discussion).
//
// One voxel per thread; every thread walks the same points in the same order,
// so their coordinates come through the scalar cache and the loop carries no
// divergence.  complex64 output: distances, phases and the reduction of the
// phase to half a turn in FP64 (the phase k r reaches ~10^3 rad, which FP32
// cannot resolve to 1e-7); the sine and cosine of the reduced phase from the
// transcendental unit (its sin/cos instructions take turns), the decay and
// 1/r in FP32; the sums in FP64.  complex128 output: FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/nvp.h"

namespace nvp {
int ctx_device(const nvp_ctx *c);
hipStream_t ctx_stream(const nvp_ctx *c);
nvp_status ctx_fail(nvp_ctx *c, nvp_status s, const char *msg);
nvp_status ctx_hip_fail(nvp_ctx *c, const char *what, hipError_t e);
}  // namespace nvp

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kBlock = 256;

template <bool DBL>
__global__ void __launch_bounds__(kBlock)
k_incident(const double *__restrict__ pts, int n_p, double ox, double oy, double oz, double h, int Ny, int Nz,
           int64_t N, double kr, double ki, double sr, double si, void *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    const int64_t t = v / Nz;
    const int iz = (int)(v - t * Nz), iy = (int)(t % Ny), ix = (int)(t / Ny);
    const double x = ox + ix * h, y = oy + iy * h, z = oz + iz * h;
    const double krt = kr * (1.0 / kTwoPi);  // Re k in turns per unit length
    double ar = 0.0, ai = 0.0;
#pragma unroll 4
    for (int j = 0; j < n_p; ++j) {
        const double dx = x - pts[3 * j], dy = y - pts[3 * j + 1], dz = z - pts[3 * j + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        double r;
        float rinv = 0.0f;
        if constexpr (DBL) {
            r = sqrt(r2);
        } else {
            // FP32 square root (relative error e ~ 2^-23) and one Newton step in
            // FP64, r = r0 + (r2 - r0^2) / (2 r0): error ~ e^2 r, below 1e-13 r
            const float r0f = __builtin_amdgcn_sqrtf((float)r2);
            rinv = __builtin_amdgcn_rcpf(r0f);
            const double r0 = r0f;
            r = fma(fma(-r0, r0, r2), 0.5 * (double)rinv, r0);
        }
        if constexpr (DBL) {
            double s, c;
            sincos(kr * r, &s, &c);
            const double a = exp(-ki * r) / r;
            ar = fma(a, c, ar);
            ai = fma(a, s, ai);
        } else {
            const double turns = krt * r;
            const float tf = (float)(turns - rint(turns));  // k_re r in turns, reduced to [-1/2, 1/2]
            const float s = __builtin_amdgcn_sinf(tf), c = __builtin_amdgcn_cosf(tf);
            const float a = __expf((float)(-ki * r)) * rinv;
            ar = fma((double)a, (double)c, ar);
            ai = fma((double)a, (double)s, ai);
        }
    }
    constexpr double inv4pi = 1.0 / (2.0 * kTwoPi);
    const double re = (sr * ar - si * ai) * inv4pi, im = (sr * ai + si * ar) * inv4pi;
    if constexpr (DBL)
        static_cast<double2 *>(out)[v] = make_double2(re, im);
    else
        static_cast<float2 *>(out)[v] = make_float2((float)re, (float)im);
}

}  // namespace

extern "C" nvp_status nvp_incident_field(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                                         const double *points_dev, int64_t n_points, const nvp_grid *g,
                                         void *out_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    if (!points_dev || !g || !out_dev || n_points < 1 || n_points > INT32_MAX ||
        (prec != NVP_C64 && prec != NVP_C128))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_field: bad argument");
    if (!std::isfinite(k_re) || !std::isfinite(k_im) || k_im < 0.0 || !std::isfinite(s_re) || !std::isfinite(s_im))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_field: k must be finite with Im k >= 0, scale finite");
    if (!(g->h > 0.0) || !std::isfinite(g->h) || g->n[0] < 1 || g->n[1] < 1 || g->n[2] < 1 ||
        g->n[0] >= (1 << 30) || g->n[1] >= (1 << 30) || g->n[2] >= (1 << 30) || !std::isfinite(g->origin[0]) ||
        !std::isfinite(g->origin[1]) || !std::isfinite(g->origin[2]))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_field: bad grid");
    const int64_t N = g->n[0] * g->n[1] * g->n[2];
    const int64_t blocks = (N + kBlock - 1) / kBlock;
    if (blocks > INT32_MAX) return nvp::ctx_fail(ctx, NVP_E_UNSUPPORTED, "nvp_incident_field: grid too large");
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    const hipStream_t s = nvp::ctx_stream(ctx);
    auto kern = prec == NVP_C128 ? k_incident<true> : k_incident<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), 0, s, points_dev, (int)n_points, g->origin[0],
                       g->origin[1], g->origin[2], g->h, (int)g->n[1], (int)g->n[2], N, k_re, k_im, s_re, s_im,
                       out_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "k_incident launch", e);
    return NVP_OK;
}
