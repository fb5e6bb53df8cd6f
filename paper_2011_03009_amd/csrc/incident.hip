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
#include <string>
#include <vector>

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

// sum_j exp(i k r_j) / r_j at (x, y, z) (without the 1 / (4 pi)).
template <bool DBL>
__device__ __forceinline__ double2 monopole_sum(const double *__restrict__ pts, int n_p, double x, double y, double z,
                                                double kr, double ki) {
    const double krt = kr * (1.0 / kTwoPi);  // Re k in turns per unit length
    double ar = 0.0, ai = 0.0;
#pragma unroll 4
    for (int j = 0; j < n_p; ++j) {
        const double dx = x - pts[3 * j], dy = y - pts[3 * j + 1], dz = z - pts[3 * j + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        if constexpr (DBL) {
            const double r = sqrt(r2);
            double s, c;
            sincos(kr * r, &s, &c);
            const double a = exp(-ki * r) / r;
            ar = fma(a, c, ar);
            ai = fma(a, s, ai);
        } else {
            // FP32 square root (relative error e ~ 2^-23) and one Newton step in
            // FP64, r = r0 + (r2 - r0^2) / (2 r0): error ~ e^2 r, below 1e-13 r
            const float r0f = __builtin_amdgcn_sqrtf((float)r2);
            const float rinv = __builtin_amdgcn_rcpf(r0f);
            const double r0 = r0f;
            const double r = fma(fma(-r0, r0, r2), 0.5 * (double)rinv, r0);
            const double turns = krt * r;
            const float tf = (float)(turns - rint(turns));  // k_re r in turns, reduced to [-1/2, 1/2]
            const float s = __builtin_amdgcn_sinf(tf), c = __builtin_amdgcn_cosf(tf);
            const float a = __expf((float)(-ki * r)) * rinv;
            ar = fma((double)a, (double)c, ar);
            ai = fma((double)a, (double)s, ai);
        }
    }
    return make_double2(ar, ai);
}

template <bool DBL> __device__ __forceinline__ void put(void *out, int64_t v, double2 a, double sr, double si) {
    constexpr double inv4pi = 1.0 / (2.0 * kTwoPi);
    const double re = (sr * a.x - si * a.y) * inv4pi, im = (sr * a.y + si * a.x) * inv4pi;
    if constexpr (DBL)
        static_cast<double2 *>(out)[v] = make_double2(re, im);
    else
        static_cast<float2 *>(out)[v] = make_float2((float)re, (float)im);
}

// At the voxel centres of a grid: voxel v = (ix * Ny + iy) * Nz + iz.
template <bool DBL>
__global__ void __launch_bounds__(kBlock)
k_incident(const double *__restrict__ pts, int n_p, double ox, double oy, double oz, double h, int Ny, int Nz,
           int64_t N, double kr, double ki, double sr, double si, void *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    const int64_t t = v / Nz;
    const int iz = (int)(v - t * Nz), iy = (int)(t % Ny), ix = (int)(t / Ny);
    put<DBL>(out, v, monopole_sum<DBL>(pts, n_p, ox + ix * h, oy + iy * h, oz + iz * h, kr, ki), sr, si);
}

// At a list of targets (n x 3 doubles).
template <bool DBL>
__global__ void __launch_bounds__(kBlock)
k_incident_at(const double *__restrict__ pts, int n_p, const double *__restrict__ tg, int64_t N, double kr,
              double ki, double sr, double si, void *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (v >= N) return;
    put<DBL>(out, v, monopole_sum<DBL>(pts, n_p, tg[3 * v], tg[3 * v + 1], tg[3 * v + 2], kr, ki), sr, si);
}

}  // namespace

namespace {

bool points_ok(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im, const double *points_dev,
               int64_t n_points, const char *who, nvp_status *st) {
    if (!points_dev || n_points < 1 || n_points > INT32_MAX) {
        *st = nvp::ctx_fail(ctx, NVP_E_INVALID, (std::string(who) + ": bad points").c_str());
        return false;
    }
    if (!std::isfinite(k_re) || !std::isfinite(k_im) || k_im < 0.0 || !std::isfinite(s_re) || !std::isfinite(s_im)) {
        *st = nvp::ctx_fail(ctx, NVP_E_INVALID,
                            (std::string(who) + ": k must be finite with Im k >= 0, scale finite").c_str());
        return false;
    }
    return true;
}

hipError_t launch_at(const double *pts, int n_p, const double *tg, int64_t N, double kr, double ki, double sr,
                     double si, void *out, bool dbl, hipStream_t s) {
    const int64_t blocks = (N + kBlock - 1) / kBlock;
    auto kern = dbl ? k_incident_at<true> : k_incident_at<false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kBlock), 0, s, pts, n_p, tg, N, kr, ki, sr, si, out);
    return hipGetLastError();
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" nvp_status nvp_incident_field(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                                         const double *points_dev, int64_t n_points, const nvp_grid *g,
                                         void *out_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    nvp_status st = NVP_OK;
    if (!points_ok(ctx, k_re, k_im, s_re, s_im, points_dev, n_points, "nvp_incident_field", &st)) return st;
    if (!g || !out_dev || (prec != NVP_C64 && prec != NVP_C128))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_field: bad argument");
    if (!(g->h > 0.0) || !std::isfinite(g->h) || g->n[0] < 1 || g->n[1] < 1 || g->n[2] < 1 ||
        g->n[0] >= (1 << 30) || g->n[1] >= (1 << 30) || g->n[2] >= (1 << 30) || !std::isfinite(g->origin[0]) ||
        !std::isfinite(g->origin[1]) || !std::isfinite(g->origin[2]))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_field: bad grid");
    // one thread per voxel: at most 2^31 - 1 workgroups of kBlock threads
    if ((double)g->n[0] * (double)g->n[1] * (double)g->n[2] > (double)INT32_MAX * kBlock)
        return nvp::ctx_fail(ctx, NVP_E_UNSUPPORTED, "nvp_incident_field: grid too large");
    const int64_t N = g->n[0] * g->n[1] * g->n[2];
    const int64_t blocks = (N + kBlock - 1) / kBlock;
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


extern "C" nvp_status nvp_incident_at(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                                      const double *points_dev, int64_t n_points, const double *targets_dev,
                                      int64_t n_targets, void *out_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    nvp_status st = NVP_OK;
    if (!points_ok(ctx, k_re, k_im, s_re, s_im, points_dev, n_points, "nvp_incident_at", &st)) return st;
    if (!targets_dev || !out_dev || n_targets < 1 || (prec != NVP_C64 && prec != NVP_C128))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_incident_at: bad argument");
    if ((n_targets + kBlock - 1) / kBlock > INT32_MAX)
        return nvp::ctx_fail(ctx, NVP_E_UNSUPPORTED, "nvp_incident_at: too many targets");
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    e = launch_at(points_dev, (int)n_points, targets_dev, n_targets, k_re, k_im, s_re, s_im, out_dev,
                  prec == NVP_C128, nvp::ctx_stream(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "k_incident_at launch", e);
    return NVP_OK;
}

extern "C" nvp_status nvp_radiated_power(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                                         const double *points_dev, int64_t n_points, const double centre[3],
                                         double radius, double rho0, double c0, int n_r, int n_theta,
                                         double *power) {
    if (!ctx) return NVP_E_INVALID;
    nvp_status st = NVP_OK;
    if (!points_ok(ctx, k_re, k_im, s_re, s_im, points_dev, n_points, "nvp_radiated_power", &st)) return st;
    if (!centre || !power || !(radius > 0.0) || !std::isfinite(radius) || !(rho0 > 0.0) || !(c0 > 0.0) ||
        !std::isfinite(rho0) || !std::isfinite(c0) || n_r < 1 || n_r > 4096 || n_theta < 1 || n_theta > 4096 ||
        !std::isfinite(centre[0]) || !std::isfinite(centre[1]) || !std::isfinite(centre[2]))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_radiated_power: bad argument");
    // midpoint nodes in r and theta on the disc x = centre[0] around the x axis
    const int64_t N = (int64_t)n_r * n_theta;
    std::vector<double> tg(3 * N), wr(n_r);
    const double dr = radius / n_r, dth = kTwoPi / n_theta;
    for (int a = 0; a < n_r; ++a) {
        const double r = (a + 0.5) * dr;
        wr[a] = r * dr * dth;
        for (int b = 0; b < n_theta; ++b) {
            const double th = (b + 0.5) * dth;
            double *q = &tg[3 * ((int64_t)a * n_theta + b)];
            q[0] = centre[0];
            q[1] = centre[1] + r * std::cos(th);
            q[2] = centre[2] + r * std::sin(th);
        }
    }
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    const hipStream_t s = nvp::ctx_stream(ctx);
    DevMem buf;
    e = hipMalloc(&buf.p, N * (3 * sizeof(double) + 2 * sizeof(double)));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_radiated_power: scratch", e);
    double *tg_dev = static_cast<double *>(buf.p), *p_dev = tg_dev + 3 * N;
    std::vector<double> p(2 * N);
    e = hipMemcpyAsync(tg_dev, tg.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_at(points_dev, (int)n_points, tg_dev, N, k_re, k_im, s_re, s_im, p_dev, true, s);
    if (e == hipSuccess) e = hipMemcpyAsync(p.data(), p_dev, 2 * N * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_radiated_power", e);
    double sum = 0.0;
    for (int a = 0; a < n_r; ++a) {
        double ring = 0.0;
        for (int b = 0; b < n_theta; ++b) {
            const double *q = &p[2 * ((int64_t)a * n_theta + b)];
            ring += q[0] * q[0] + q[1] * q[1];
        }
        sum += wr[a] * ring;
    }
    *power = sum / (2.0 * rho0 * c0);
    return NVP_OK;
}
