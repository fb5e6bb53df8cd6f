// The lower harmonics as the source build sees them: a field on its own grid
// with per-axis interpolation tables onto the target grid.  Device structs
// shared by the fused x pass and the separate source kernel.
#pragma once

#include "fft_core.hpp"
#include "common.hpp"

namespace nvp {

// Source term of harmonic n fused into the forward x pass:
//   f_n(x) = sum_{m=1}^{n-1} T_m[p_m](x) T_{n-m}[p_{n-m}](x),
// where T_m interpolates p_m from its own grid with separable K-point weights
// (K = 2 linear, K = 4 cubic Lagrange) from per-axis tables, or reads it
// directly when p_m lives on the target grid.
template <typename R> struct FieldDev {
    const cx<R> *__restrict__ p;
    int64_t s0, s1;                      // strides of the field's own grid
    const int *__restrict__ b[3];        // base source index per target index, per axis
    const R *__restrict__ w[3];          // K weights per target index, per axis
    int identity;
};

template <typename R, int K> struct LdSource {
    FieldDev<R> f[NVP_MAX_FIELDS];
    int nf;      // n - 1 fields
    int Nx, Nz;  // target grid (Ny implied by the column count)

    __device__ __forceinline__ cx<R> interp(const FieldDev<R> &g, int ix, int iy, int iz) const {
        if (g.identity) return g.p[ix * g.s0 + (int64_t)iy * g.s1 + iz];
        const int bx = g.b[0][ix], by = g.b[1][iy], bz = g.b[2][iz];
        R wx[K], wy[K], wz[K];
#pragma unroll
        for (int a = 0; a < K; ++a) {
            wx[a] = g.w[0][ix * K + a];
            wy[a] = g.w[1][iy * K + a];
            wz[a] = g.w[2][iz * K + a];
        }
        const cx<R> *base = g.p + (int64_t)bx * g.s0 + (int64_t)by * g.s1 + bz;
        cx<R> acc = czero<R>();
#pragma unroll
        for (int a = 0; a < K; ++a) {
            cx<R> ay = czero<R>();
#pragma unroll
            for (int c = 0; c < K; ++c) {
                const cx<R> *row = base + a * g.s0 + c * g.s1;
                cx<R> az = czero<R>();
#pragma unroll
                for (int d = 0; d < K; ++d) az = cadd<R>(az, cscale<R>(row[d], wz[d]));
                ay = cadd<R>(ay, cscale<R>(az, wy[c]));
            }
            acc = cadd<R>(acc, cscale<R>(ay, wx[a]));
        }
        return acc;
    }

    // sum_{a+b = nf-1} v_a v_b over the transferred fields
    __device__ __forceinline__ cx<R> products(const cx<R> *v) const {
        cx<R> s = czero<R>();
#pragma unroll
        for (int a = 0; a < NVP_MAX_FIELDS; ++a)
#pragma unroll
            for (int b = 0; b < NVP_MAX_FIELDS; ++b)
                if (a + b == nf - 1) s = cadd<R>(s, cmul<R>(v[a], v[b]));
        return s;
    }

    // f_n at target voxel (ix, iy, iz)
    __device__ __forceinline__ cx<R> value(int ix, int iy, int iz) const {
        cx<R> v[NVP_MAX_FIELDS];
#pragma unroll
        for (int i = 0; i < NVP_MAX_FIELDS; ++i) v[i] = i < nf ? interp(f[i], ix, iy, iz) : czero<R>();
        return products(v);
    }
};

}  // namespace nvp
