// Volume integral equations of an inhomogeneous medium (Section 7, the
// equations for the harmonics in an inhomogeneous domain): with the
// background wavenumber kb and the contrast q(y) = k(y)^2 - kb^2,
//     p(x) - int G_kb(x, y) q(y) p(y) dy = rhs(x),
// discretised with the same midpoint-rule kernel as the volume potential:
//     p_i - sum_j K_kb(x_i - x_j) q_j p_j = rhs_i.
// Solved by BiCGStab (van der Vorst's stabilised bi-conjugate gradients) with
// the library's FFT volume potential as the operator.  The vector updates,
// the inner products (accumulated in FP64) and the scalar recurrence are the
// kernels below; an iteration waits once, for the residual norm.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "../../include/nvp.h"

namespace nvp {
int ctx_device(const nvp_ctx *c);
hipStream_t ctx_stream(const nvp_ctx *c);
nvp_status ctx_fail(nvp_ctx *c, nvp_status s, const char *msg);
nvp_status ctx_hip_fail(nvp_ctx *c, const char *what, hipError_t e);
}  // namespace nvp

namespace {

constexpr int kBlock = 256;
constexpr int kDotBlocks = 1024;

template <typename V> struct Real;
template <> struct Real<float2> { using type = float; };
template <> struct Real<double2> { using type = double; };

template <typename V> __device__ __forceinline__ V mk(double x, double y) {
    using R = typename Real<V>::type;
    return V{(R)x, (R)y};
}

// out = q * x
template <typename V>
__global__ void __launch_bounds__(kBlock) k_mul(V *__restrict__ out, const V *__restrict__ q, const V *__restrict__ x,
                                                int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V a = q[i], b = x[i];
    out[i] = V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// out = a + al * b + be * c; a null operand counts as zero.  out may be any
// of the operands (each element is read before it is written).
template <typename V>
__global__ void __launch_bounds__(kBlock) k_lin3(V *out, const V *a, const V *b, const V *c, double2 al, double2 be,
                                                 int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const V A = a ? a[i] : mk<V>(0.0, 0.0), B = b ? b[i] : mk<V>(0.0, 0.0), C = c ? c[i] : mk<V>(0.0, 0.0);
    const V p = mk<V>(al.x, al.y), r = mk<V>(be.x, be.y);
    out[i] = V{A.x + p.x * B.x - p.y * B.y + r.x * C.x - r.y * C.y, A.y + p.x * B.y + p.y * B.x + r.x * C.y + r.y * C.x};
}

// Partial sums of conj(a_i) b_i in FP64, one per workgroup (grid-stride).
template <typename V>
__global__ void __launch_bounds__(kBlock) k_dot(const V *__restrict__ a, const V *__restrict__ b, int64_t n,
                                                double2 *__restrict__ part) {
    __shared__ double sr[kBlock], si[kBlock];
    double re = 0.0, im = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double ax = a[i].x, ay = a[i].y, bx = b[i].x, by = b[i].y;
        re += ax * bx + ay * by;
        im += ax * by - ay * bx;
    }
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sr[0], si[0]);
}

// out = f inside the voxel box [lo, hi] (inclusive, per axis), 0 outside;
// grid (ceil(Nz / kBlock), Ny, Nx).
template <typename V>
__global__ void __launch_bounds__(kBlock) k_box_mask(const V *__restrict__ f, V *__restrict__ out, int64_t Ny,
                                                     int64_t Nz, int64_t lx, int64_t ly, int64_t lz, int64_t hx,
                                                     int64_t hy, int64_t hz) {
    const int64_t iz = (int64_t)blockIdx.x * kBlock + threadIdx.x, iy = blockIdx.y, ix = blockIdx.z;
    if (iz >= Nz) return;
    const int64_t i = (ix * Ny + iy) * Nz + iz;
    const bool in = ix >= lx && ix <= hx && iy >= ly && iy <= hy && iz >= lz && iz <= hz;
    out[i] = in ? f[i] : mk<V>(0.0, 0.0);
}

// Partial sums of |a - b|^2 and |a|^2 in FP64, one pair per workgroup.
template <typename V>
__global__ void __launch_bounds__(kBlock) k_diff_norms(const V *__restrict__ a, const V *__restrict__ b, int64_t n,
                                                       double2 *__restrict__ part) {
    __shared__ double sd[kBlock], sa[kBlock];
    double d = 0.0, q = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double ax = a[i].x, ay = a[i].y, dx = ax - (double)b[i].x, dy = ay - (double)b[i].y;
        d += dx * dx + dy * dy;
        q += ax * ax + ay * ay;
    }
    sd[threadIdx.x] = d;
    sa[threadIdx.x] = q;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sd[threadIdx.x] += sd[threadIdx.x + w];
            sa[threadIdx.x] += sa[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sd[0], sa[0]);
}

using cd = std::complex<double>;

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

// out = a + al[0] b + be[0] c with the coefficients read from device memory
// (the recurrence's scalars never leave the device); as k_lin3 otherwise.
// Nothing is written once the recurrence has flagged a breakdown, so that the
// iterate stays the last good one.
template <typename V>
__global__ void __launch_bounds__(kBlock) k_lin3d(V *out, const V *a, const V *b, const V *c,
                                                  const double2 *__restrict__ al, const double2 *__restrict__ be,
                                                  const double2 *__restrict__ flag, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n || flag->x != 0.0) return;
    const double2 A2 = al ? *al : make_double2(0.0, 0.0), B2 = be ? *be : make_double2(0.0, 0.0);
    const V A = a ? a[i] : mk<V>(0.0, 0.0), B = b ? b[i] : mk<V>(0.0, 0.0), C = c ? c[i] : mk<V>(0.0, 0.0);
    const V p = mk<V>(A2.x, A2.y), r = mk<V>(B2.x, B2.y);
    out[i] = V{A.x + p.x * B.x - p.y * B.y + r.x * C.x - r.y * C.y, A.y + p.x * B.y + p.y * B.x + r.x * C.y + r.y * C.x};
}

// The scalar state of BiCGStab on the device, one double2 (complex) each.
enum Sc { RHO, ALPHA, OMEGA, RHO1, RV, TS, TT, RN2, RNI, BETA, NBO, NAL, NOM, FLAG, NSC };

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Sums the kDotBlocks-or-fewer partial dot products into sc[slot] (one
// workgroup, fixed order), then takes the step of the recurrence that this
// dot product completes:
//   RHO1: beta = (rho1 / rho) (alpha / omega), coefficients beta and -beta omega
//         for p = r + beta (p - omega v); flags a breakdown (rho1 or omega zero);
//   RV:   alpha = rho1 / rv (flag rv zero), coefficient -alpha for s = r - alpha v;
//   TT:   omega = ts / tt (0 when tt is 0), coefficient -omega for r = s - omega t;
//   RNI:  the iteration's residual norm squared, kept in RN2, and rho = rho1 for
//         the next iteration (RN2 alone: a norm with no step of the recurrence).
__global__ void __launch_bounds__(kBlock) k_dot_finish(const double2 *__restrict__ part, int nb, double2 *sc,
                                                       int slot) {
    __shared__ double sr[kBlock], si[kBlock];
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nb; i += kBlock) re += part[i].x, im += part[i].y;
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            sr[threadIdx.x] += sr[threadIdx.x + w];
            si[threadIdx.x] += si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x) return;
    const double2 v = make_double2(sr[0], si[0]);
    sc[slot] = v;
    if (slot == RHO1) {
        const double2 rho = sc[RHO], al = sc[ALPHA], om = sc[OMEGA];
        if ((v.x == 0.0 && v.y == 0.0) || (om.x == 0.0 && om.y == 0.0)) {
            sc[FLAG].x = 1.0;
            return;
        }
        const double2 beta = cmuld(cdiv(v, rho), cdiv(al, om));
        sc[BETA] = beta;
        const double2 bo = cmuld(beta, om);
        sc[NBO] = make_double2(-bo.x, -bo.y);
    } else if (slot == RV) {
        if (v.x == 0.0 && v.y == 0.0) {
            sc[FLAG].x = 1.0;
            return;
        }
        const double2 al = cdiv(sc[RHO1], v);
        sc[ALPHA] = al;
        sc[NAL] = make_double2(-al.x, -al.y);
    } else if (slot == TT) {
        const double2 om = v.x > 0.0 ? cdiv(sc[TS], v) : make_double2(0.0, 0.0);
        sc[OMEGA] = om;
        sc[NOM] = make_double2(-om.x, -om.y);
    } else if (slot == RNI) {
        sc[RN2] = v;
        sc[RHO] = sc[RHO1];
    }
}

// The solver's state for one call: vectors of n complex values of type V.
template <typename V> struct Solver {
    nvp_ctx *ctx;
    hipStream_t s;
    int64_t n;
    double kr, ki;
    const nvp_grid *g;
    nvp_prec prec;
    const V *q;
    double2 *part;  // kDotBlocks partial sums
    double2 *sc;    // NSC scalars
    V *tmp, *u;     // operator scratch
    nvp_status st = NVP_OK;

    unsigned blocks() const { return (unsigned)((n + kBlock - 1) / kBlock); }
    bool ok(hipError_t e, const char *what) {
        if (e != hipSuccess && st == NVP_OK) st = nvp::ctx_hip_fail(ctx, what, e);
        return st == NVP_OK;
    }
    bool lin3(V *out, const V *a, const V *b, const V *c, cd al, cd be) {
        hipLaunchKernelGGL(k_lin3<V>, dim3(blocks()), dim3(kBlock), 0, s, out, a, b, c,
                           make_double2(al.real(), al.imag()), make_double2(be.real(), be.imag()), n);
        return ok(hipGetLastError(), "k_lin3");
    }
    bool lin3d(V *out, const V *a, const V *b, const V *c, int al, int be) {
        hipLaunchKernelGGL(k_lin3d<V>, dim3(blocks()), dim3(kBlock), 0, s, out, a, b, c, al < 0 ? nullptr : sc + al,
                           be < 0 ? nullptr : sc + be, sc + FLAG, n);
        return ok(hipGetLastError(), "k_lin3d");
    }
    // y = A x = x - V[q x] = x + u, with u = -V[q x] the raw operator's output
    bool apply(V *y, const V *x) {
        hipLaunchKernelGGL(k_mul<V>, dim3(blocks()), dim3(kBlock), 0, s, tmp, q, x, n);
        if (!ok(hipGetLastError(), "k_mul")) return false;
        const nvp_status e = nvp_volume_potential(ctx, kr, ki, g, tmp, u, prec);
        if (e != NVP_OK) {
            st = e;
            return false;
        }
        return lin3(y, x, u, nullptr, 1.0, 0.0);
    }
    // sc[slot] = sum conj(a) b, and the recurrence step it completes (device only)
    bool dot(const V *a, const V *b, int slot) {
        const unsigned nb = (unsigned)std::min<int64_t>(kDotBlocks, blocks());
        hipLaunchKernelGGL(k_dot<V>, dim3(nb), dim3(kBlock), 0, s, a, b, n, part);
        if (!ok(hipGetLastError(), "k_dot")) return false;
        hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(kBlock), 0, s, part, (int)nb, sc, slot);
        return ok(hipGetLastError(), "k_dot_finish");
    }
    // reads sc[RN2] and the breakdown flag: the one wait of an iteration
    bool read(double *rn2, bool *broke) {
        double2 h[2];
        if (!ok(hipMemcpyAsync(&h[0], sc + RN2, sizeof(double2), hipMemcpyDeviceToHost, s), "residual copy") ||
            !ok(hipMemcpyAsync(&h[1], sc + FLAG, sizeof(double2), hipMemcpyDeviceToHost, s), "flag copy") ||
            !ok(hipStreamSynchronize(s), "residual sync"))
            return false;
        *rn2 = std::max(0.0, h[0].x);
        *broke = h[1].x != 0.0;
        return true;
    }
};

__global__ void k_scalars_init(double2 *sc) {
    const int i = threadIdx.x;
    if (i < NSC) sc[i] = (i == RHO || i == ALPHA || i == OMEGA) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
}

// BiCGStab (van der Vorst) with the recurrence's scalars kept on the device:
// each iteration enqueues its two operator applications, five dot products
// with their scalar steps and the vector updates, and waits once, to read the
// residual norm and the breakdown flag.
template <typename V>
nvp_status bicgstab(nvp_ctx *ctx, double kr, double ki, const nvp_grid *g, nvp_prec prec, const void *q_dev,
                    const void *rhs_dev, void *p_dev, double tol, int max_iter, int *iters, double *relres) {
    const int64_t n = g->n[0] * g->n[1] * g->n[2];
    DevMem mem;
    hipError_t e = hipMalloc(&mem.p, 8 * n * sizeof(V) + (kDotBlocks + NSC) * sizeof(double2));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_vie_solve: work vectors", e);
    V *w = static_cast<V *>(mem.p);
    V *r = w, *rh = w + n, *pv = w + 2 * n, *v = w + 3 * n, *sv = w + 4 * n, *t = w + 5 * n;
    double2 *part = reinterpret_cast<double2 *>(w + 8 * n);
    Solver<V> S{ctx, nvp::ctx_stream(ctx), n, kr, ki, g, prec, static_cast<const V *>(q_dev), part,
                part + kDotBlocks, w + 6 * n, w + 7 * n};
    const V *b = static_cast<const V *>(rhs_dev);
    V *x = static_cast<V *>(p_dev);
    *iters = 0;
    hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(64), 0, S.s, S.sc);
    if (!S.ok(hipGetLastError(), "k_scalars_init")) return S.st;
    double bn2 = 0.0, rn2 = 0.0;
    bool broke = false;
    if (!S.dot(b, b, RN2) || !S.read(&bn2, &broke)) return S.st;
    const double bn = std::sqrt(bn2);
    if (bn == 0.0) {  // the solution is zero
        S.lin3(x, nullptr, nullptr, nullptr, 0.0, 0.0);
        *relres = 0.0;
        return S.st;
    }
    // r = b - A x, rh = r, p = v = 0
    if (!S.apply(t, x) || !S.lin3(r, b, t, nullptr, -1.0, 0.0) || !S.lin3(rh, r, nullptr, nullptr, 0.0, 0.0) ||
        !S.lin3(pv, nullptr, nullptr, nullptr, 0.0, 0.0) || !S.lin3(v, nullptr, nullptr, nullptr, 0.0, 0.0) ||
        !S.dot(r, r, RN2) || !S.read(&rn2, &broke))
        return S.st;
    int it = 0;
    while (std::sqrt(rn2) / bn > tol && it < max_iter) {
        ++it;
        if (!S.dot(rh, r, RHO1) || !S.lin3d(pv, r, pv, v, BETA, NBO) || !S.apply(v, pv) || !S.dot(rh, v, RV) ||
            !S.lin3d(sv, r, v, nullptr, NAL, -1) || !S.apply(t, sv) || !S.dot(t, sv, TS) || !S.dot(t, t, TT) ||
            !S.lin3d(x, x, pv, sv, ALPHA, OMEGA) || !S.lin3d(r, sv, t, nullptr, NOM, -1) || !S.dot(r, r, RNI) ||
            !S.read(&rn2, &broke))
            return S.st;
        if (broke) return nvp::ctx_fail(ctx, NVP_E_STATE, "nvp_vie_solve: BiCGStab breakdown");
    }
    *iters = it;
    // the true residual of the returned solution
    if (!S.apply(t, x) || !S.lin3(r, b, t, nullptr, -1.0, 0.0) || !S.dot(r, r, RN2) || !S.read(&rn2, &broke))
        return S.st;
    *relres = std::sqrt(rn2) / bn;
    return NVP_OK;
}

}  // namespace

extern "C" nvp_status nvp_vie_solve(nvp_ctx *ctx, double kb_re, double kb_im, const nvp_grid *g, const void *q_dev,
                                    const void *rhs_dev, void *p_dev, nvp_prec prec, double tol, int max_iter,
                                    int *iters, double *relres) {
    if (!ctx) return NVP_E_INVALID;
    if (!g || !q_dev || !rhs_dev || !p_dev || !iters || !relres || p_dev == q_dev || p_dev == rhs_dev ||
        !(tol > 0.0) || !std::isfinite(tol) || max_iter < 1 || (prec != NVP_C64 && prec != NVP_C128) ||
        g->n[0] < 1 || g->n[1] < 1 || g->n[2] < 1)
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_vie_solve: bad argument");
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    return prec == NVP_C128
               ? bicgstab<double2>(ctx, kb_re, kb_im, g, prec, q_dev, rhs_dev, p_dev, tol, max_iter, iters, relres)
               : bicgstab<float2>(ctx, kb_re, kb_im, g, prec, q_dev, rhs_dev, p_dev, tol, max_iter, iters, relres);
}

namespace nvp {

// Copies f ([Nx][Ny][Nz]) to out with every voxel outside the inclusive box
// lo..hi set to zero (the volume potential of a source restricted to a box).
hipError_t launch_box_mask(const void *f, void *out, bool dbl, const int64_t n[3], const int64_t box[6],
                           hipStream_t s) {
    const dim3 grid((unsigned)((n[2] + kBlock - 1) / kBlock), (unsigned)n[1], (unsigned)n[0]);
    if (dbl)
        hipLaunchKernelGGL(k_box_mask<double2>, grid, dim3(kBlock), 0, s, static_cast<const double2 *>(f),
                           static_cast<double2 *>(out), n[1], n[2], box[0], box[1], box[2], box[3], box[4], box[5]);
    else
        hipLaunchKernelGGL(k_box_mask<float2>, grid, dim3(kBlock), 0, s, static_cast<const float2 *>(f),
                           static_cast<float2 *>(out), n[1], n[2], box[0], box[1], box[2], box[3], box[4], box[5]);
    return hipGetLastError();
}

}  // namespace nvp

extern "C" nvp_status nvp_field_lin3(nvp_ctx *ctx, int64_t n, void *out_dev, const void *a_dev, const void *b_dev,
                                     const void *c_dev, const double al[2], const double be[2], nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    if (n < 0 || !out_dev || !al || !be || (prec != NVP_C64 && prec != NVP_C128) || !std::isfinite(al[0]) ||
        !std::isfinite(al[1]) || !std::isfinite(be[0]) || !std::isfinite(be[1]))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_field_lin3: bad argument");
    if (n == 0) return NVP_OK;
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    const double2 A = make_double2(al[0], al[1]), B = make_double2(be[0], be[1]);
    hipStream_t s = nvp::ctx_stream(ctx);
    if (prec == NVP_C128)
        hipLaunchKernelGGL(k_lin3<double2>, grid, dim3(kBlock), 0, s, static_cast<double2 *>(out_dev),
                           static_cast<const double2 *>(a_dev), static_cast<const double2 *>(b_dev),
                           static_cast<const double2 *>(c_dev), A, B, n);
    else
        hipLaunchKernelGGL(k_lin3<float2>, grid, dim3(kBlock), 0, s, static_cast<float2 *>(out_dev),
                           static_cast<const float2 *>(a_dev), static_cast<const float2 *>(b_dev),
                           static_cast<const float2 *>(c_dev), A, B, n);
    e = hipGetLastError();
    return e == hipSuccess ? NVP_OK : nvp::ctx_hip_fail(ctx, "k_lin3", e);
}

extern "C" nvp_status nvp_field_diff_norms(nvp_ctx *ctx, int64_t n, const void *a_dev, const void *b_dev,
                                           nvp_prec prec, double out[2]) {
    if (!ctx) return NVP_E_INVALID;
    if (n < 0 || !a_dev || !b_dev || !out || (prec != NVP_C64 && prec != NVP_C128))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_field_diff_norms: bad argument");
    out[0] = out[1] = 0.0;
    if (n == 0) return NVP_OK;
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    hipStream_t s = nvp::ctx_stream(ctx);
    const unsigned nb = (unsigned)std::min<int64_t>(kDotBlocks, (n + kBlock - 1) / kBlock);
    DevMem part;
    e = hipMalloc(&part.p, nb * sizeof(double2));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_field_diff_norms: partial sums", e);
    if (prec == NVP_C128)
        hipLaunchKernelGGL(k_diff_norms<double2>, dim3(nb), dim3(kBlock), 0, s, static_cast<const double2 *>(a_dev),
                           static_cast<const double2 *>(b_dev), n, static_cast<double2 *>(part.p));
    else
        hipLaunchKernelGGL(k_diff_norms<float2>, dim3(nb), dim3(kBlock), 0, s, static_cast<const float2 *>(a_dev),
                           static_cast<const float2 *>(b_dev), n, static_cast<double2 *>(part.p));
    e = hipGetLastError();
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "k_diff_norms", e);
    std::vector<double2> h(nb);
    e = hipMemcpyAsync(h.data(), part.p, nb * sizeof(double2), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_field_diff_norms: result", e);
    for (const double2 &v : h) out[0] += v.x, out[1] += v.y;
    return NVP_OK;
}
