// Difference-frequency products of the harmonic cascade (Section 2: equation
// "cascade_1" before the truncation to "cascade_2").  Matching the
// coefficients of e^{-i n w t} in the Westervelt equation gives, besides the
// sum-frequency products p_m p_{n-m} that the paper keeps, the products
// 2 p_m conj(p_{m-n}) for m > n.  This kernel accumulates one such product on a
// harmonic's grid from two fields on grids of their own: the tensor-product
// transfer of each field (order 1 or 3, the cascade's transfer), optionally
// zero at targets outside the hull of the source's voxel centres (a higher
// harmonic vanishes outside its own box), then out += scale a conj(b), all in
// FP64 arithmetic.
#include <hip/hip_runtime.h>

#include <cmath>
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
constexpr double kHullEps = 1e-9;  // in source voxels: a target this close to the hull is inside

// One field's stencil tables on the target grid: per axis the first source
// index and K weights per target index (all zero where the target is outside
// a zero-outside field's hull).  identity: the field is on the target grid.
struct Stencil {
    const void *p;
    int64_t s0, s1;
    const int *b[3];
    const double *w[3];
    int identity;
};

template <typename V> struct Real;
template <> struct Real<float2> { using type = float; };
template <> struct Real<double2> { using type = double; };

template <typename V, int K>
__device__ __forceinline__ double2 sample(const Stencil &f, int ix, int iy, int iz, int Ny, int Nz) {
    const V *p = static_cast<const V *>(f.p);
    if (f.identity) {
        const V v = p[((int64_t)ix * Ny + iy) * Nz + iz];
        return make_double2((double)v.x, (double)v.y);
    }
    const int bx = f.b[0][ix], by = f.b[1][iy], bz = f.b[2][iz];
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        const double wa = f.w[0][ix * K + a];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const double wac = wa * f.w[1][iy * K + c];
            const V *row = p + (int64_t)(bx + a) * f.s0 + (int64_t)(by + c) * f.s1 + bz;
#pragma unroll
            for (int d = 0; d < K; ++d) {
                const double w = wac * f.w[2][iz * K + d];
                re += w * (double)row[d].x;
                im += w * (double)row[d].y;
            }
        }
    }
    return make_double2(re, im);
}

template <typename V, int K>
__global__ void __launch_bounds__(kBlock) k_difference(V *__restrict__ out, Stencil a, Stencil b, int Nx, int Ny,
                                                       int Nz, double scale) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (int64_t)Nx * Ny * Nz) return;
    const int iz = (int)(i % Nz), iy = (int)((i / Nz) % Ny), ix = (int)(i / ((int64_t)Ny * Nz));
    const double2 u = sample<V, K>(a, ix, iy, iz, Ny, Nz), v = sample<V, K>(b, ix, iy, iz, Ny, Nz);
    // scale * u * conj(v)
    const double re = scale * (u.x * v.x + u.y * v.y), im = scale * (u.y * v.x - u.x * v.y);
    V o = out[i];
    using R = typename Real<V>::type;
    o.x = (R)((double)o.x + re);
    o.y = (R)((double)o.y + im);
    out[i] = o;
}

bool grid_valid(const nvp_grid *g) {
    return g && std::isfinite(g->h) && g->h > 0 && g->n[0] >= 1 && g->n[1] >= 1 && g->n[2] >= 1 &&
           std::isfinite(g->origin[0]) && std::isfinite(g->origin[1]) && std::isfinite(g->origin[2]);
}

bool same(const nvp_grid *a, const nvp_grid *b) {
    return a->h == b->h && a->origin[0] == b->origin[0] && a->origin[1] == b->origin[1] &&
           a->origin[2] == b->origin[2] && a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->n[2] == b->n[2];
}

// Host tables of one field on grid gt, appended to `ints` and `dbls`; offsets
// into them per axis in ob / ow.  Returns false if an axis is too short.
bool tables(const nvp_grid *gt, const nvp_grid *gs, int zero_outside, int order, std::vector<int> &ints,
            std::vector<double> &dbls, size_t ob[3], size_t ow[3]) {
    const int K = order + 1;
    for (int ax = 0; ax < 3; ++ax) {
        const int64_t n = gt->n[ax];
        std::vector<int32_t> base((size_t)n);
        std::vector<double> w((size_t)n * K);
        if (nvp_transfer_axis(gt->origin[ax], gt->h, n, gs->origin[ax], gs->h, gs->n[ax], order, base.data(),
                              w.data()) != NVP_OK)
            return false;
        if (zero_outside)
            for (int64_t i = 0; i < n; ++i) {
                const double x = gt->origin[ax] + (double)i * gt->h;
                const double s = (x - gs->origin[ax]) / gs->h;
                if (s < -kHullEps || s > (double)(gs->n[ax] - 1) + kHullEps)
                    for (int j = 0; j < K; ++j) w[(size_t)i * K + j] = 0.0;
            }
        ob[ax] = ints.size();
        ow[ax] = dbls.size();
        ints.insert(ints.end(), base.begin(), base.end());
        dbls.insert(dbls.end(), w.begin(), w.end());
    }
    return true;
}

struct DevMem {
    void *p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" nvp_status nvp_difference_term(nvp_ctx *ctx, const nvp_grid *gt, void *out_dev, const nvp_grid *ga,
                                          const void *a_dev, int zero_a, const nvp_grid *gb, const void *b_dev,
                                          int zero_b, int order, double scale, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    if (!grid_valid(gt) || !grid_valid(ga) || !grid_valid(gb) || !out_dev || !a_dev || !b_dev || out_dev == a_dev ||
        out_dev == b_dev || (order != 1 && order != 3) || !std::isfinite(scale) ||
        (prec != NVP_C64 && prec != NVP_C128))
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_difference_term: bad argument");
    const int64_t nt = gt->n[0] * gt->n[1] * gt->n[2];
    if (gt->n[0] > INT32_MAX || gt->n[1] > INT32_MAX || gt->n[2] > INT32_MAX)
        return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_difference_term: grid too large");
    std::vector<int> ints;
    std::vector<double> dbls;
    size_t ob[2][3] = {}, ow[2][3] = {};
    const nvp_grid *gs[2] = {ga, gb};
    const int zo[2] = {zero_a, zero_b};
    bool ident[2];
    for (int f = 0; f < 2; ++f) {
        ident[f] = same(gt, gs[f]);
        if (!ident[f] && !tables(gt, gs[f], zo[f], order, ints, dbls, ob[f], ow[f]))
            return nvp::ctx_fail(ctx, NVP_E_INVALID, "nvp_difference_term: a source axis is shorter than order + 1");
    }
    hipError_t e = hipSetDevice(nvp::ctx_device(ctx));
    if (e != hipSuccess) return nvp::ctx_hip_fail(ctx, "hipSetDevice", e);
    hipStream_t s = nvp::ctx_stream(ctx);
    const size_t ib = ints.size() * sizeof(int), db = dbls.size() * sizeof(double);
    const size_t ib_al = (ib + 255) / 256 * 256;
    DevMem mem;
    if (ib + db > 0) {
        e = hipMalloc(&mem.p, ib_al + db);
        if (e != hipSuccess) return nvp::ctx_fail(ctx, NVP_E_NOMEM, "nvp_difference_term: stencil tables");
        if ((e = hipMemcpyAsync(mem.p, ints.data(), ib, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(static_cast<char *>(mem.p) + ib_al, dbls.data(), db, hipMemcpyHostToDevice, s)) !=
                hipSuccess)
            return nvp::ctx_hip_fail(ctx, "nvp_difference_term: table upload", e);
    }
    const int *ibase = static_cast<const int *>(mem.p);
    const double *dbase = reinterpret_cast<const double *>(static_cast<const char *>(mem.p) + ib_al);
    Stencil st[2];
    const void *src[2] = {a_dev, b_dev};
    for (int f = 0; f < 2; ++f) {
        st[f].p = src[f];
        st[f].s0 = gs[f]->n[1] * gs[f]->n[2];
        st[f].s1 = gs[f]->n[2];
        st[f].identity = ident[f];
        for (int ax = 0; ax < 3; ++ax) {
            st[f].b[ax] = ident[f] ? nullptr : ibase + ob[f][ax];
            st[f].w[ax] = ident[f] ? nullptr : dbase + ow[f][ax];
        }
    }
    const unsigned blocks = (unsigned)((nt + kBlock - 1) / kBlock);
    const int Nx = (int)gt->n[0], Ny = (int)gt->n[1], Nz = (int)gt->n[2];
    if (prec == NVP_C128) {
        if (order == 1)
            hipLaunchKernelGGL((k_difference<double2, 2>), dim3(blocks), dim3(kBlock), 0, s,
                               static_cast<double2 *>(out_dev), st[0], st[1], Nx, Ny, Nz, scale);
        else
            hipLaunchKernelGGL((k_difference<double2, 4>), dim3(blocks), dim3(kBlock), 0, s,
                               static_cast<double2 *>(out_dev), st[0], st[1], Nx, Ny, Nz, scale);
    } else {
        if (order == 1)
            hipLaunchKernelGGL((k_difference<float2, 2>), dim3(blocks), dim3(kBlock), 0, s,
                               static_cast<float2 *>(out_dev), st[0], st[1], Nx, Ny, Nz, scale);
        else
            hipLaunchKernelGGL((k_difference<float2, 4>), dim3(blocks), dim3(kBlock), 0, s,
                               static_cast<float2 *>(out_dev), st[0], st[1], Nx, Ny, Nz, scale);
    }
    if ((e = hipGetLastError()) != hipSuccess) return nvp::ctx_hip_fail(ctx, "k_difference", e);
    // the tables are freed when this call returns: wait for the kernel
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return nvp::ctx_hip_fail(ctx, "nvp_difference_term", e);
    return NVP_OK;
}
