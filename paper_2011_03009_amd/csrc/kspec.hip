// Launchers of the transfer + source kernel and small run-time queries of the compiled plans.
#include <math.h>
#include <stdlib.h>

#include "passes_impl.hpp"
#include "source.hpp"
#include "source_wf.hpp"

namespace nvp {

// The kernel of equation "quad" depends on a voxel offset d only through the
// integer |d|^2: ktab[q] = h^3 G_k(sqrt(q) h) for q >= 1, and the self value
// for q = 0, in FP64.  The octant rows below read it, so each distinct
// distance is evaluated once instead of once per offset.  `face` is added at
// q = 1, the six face neighbours (the corrected quadrature's face weight).
__global__ void __launch_bounds__(256) k_kradial(double2 *__restrict__ ktab, int64_t n, double h, double kr, double ki,
                                                 double2 self, double2 face) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    if (q == 0) {
        ktab[0] = self;
        return;
    }
    const double d = h * sqrt((double)q);
    const double mag = h * h * h * exp(-ki * d) / (4.0 * M_PI * d);
    double sn, cs;
    sincos(kr * d, &sn, &cs);
    ktab[q] = q == 1 ? make_double2(mag * cs + face.x, mag * sn + face.y) : make_double2(mag * cs, mag * sn);
}

hipError_t launch_kradial(double2 *ktab, int64_t n, double h, double kr, double ki, double self_re, double self_im,
                          double face_re, double face_im, hipStream_t s) {
    hipLaunchKernelGGL(k_kradial, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ktab, n, h, kr, ki,
                       make_double2(self_re, self_im), make_double2(face_re, face_im));
    return hipGetLastError();
}

template <typename R, int K, int NF>
static hipError_t source_nf(const LdSource<R, K> &ld, const SourceArgs &a, void *out, int Ny, int cxl, hipStream_t s) {
    if constexpr (source_wf(sizeof(R))) {
        auto kern = k_source_wf<R, K, NF, NVP_SRC_PREW, NVP_SRC_CXM>;
        constexpr size_t lds = SrcWfLds<R, K, NF, NVP_SRC_PREW, NVP_SRC_CXM>::BYTES;
        static_assert(lds == source_lds_bytes(NF, K, sizeof(R)), "the host sizes this kernel's LDS layout");
        if (cxl < 1 || cxl > NVP_SRC_CXM) return hipErrorInvalidValue;
        if (lds > 98304) return hipErrorInvalidValue;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        dim3 grid((unsigned)((a.Nz + 31) / 32), (unsigned)((Ny + 7) / 8), (unsigned)((a.Nx + cxl - 1) / cxl));
        hipLaunchKernelGGL(kern, grid, dim3(NF * 64), lds, s, ld, static_cast<cx<R> *>(out), Ny, cxl);
        return hipGetLastError();
    } else {
        constexpr int RY = source_rows(sizeof(R)), PRE = source_pre(sizeof(R));
        auto kern = k_source<R, K, NF, NVP_SRC_TY, NVP_SRC_TZ, RY, PRE, NVP_SRC_CXM>;
        constexpr size_t lds = SrcLds<R, K, NF, NVP_SRC_TY, NVP_SRC_TZ, RY, PRE, NVP_SRC_CXM>::BYTES;
        static_assert(lds == source_lds_bytes(NF, K, sizeof(R)), "the host sizes this kernel's LDS layout");
        if (cxl < 1 || cxl > NVP_SRC_CXM) return hipErrorInvalidValue;
        if (lds > 98304) return hipErrorInvalidValue;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        dim3 grid((unsigned)((a.Nz + NVP_SRC_TZ - 1) / NVP_SRC_TZ),
                  (unsigned)((Ny + RY * NVP_SRC_TY - 1) / (RY * NVP_SRC_TY)), (unsigned)((a.Nx + cxl - 1) / cxl));
        hipLaunchKernelGGL(kern, grid, dim3(NVP_SRC_TY * NVP_SRC_TZ), lds, s, ld, static_cast<cx<R> *>(out), Ny,
                           cxl);
        return hipGetLastError();
    }
}

template <typename R, int K>
static hipError_t source_k(const SourceArgs &a, void *out, int Ny, int cxl, hipStream_t s) {
    LdSource<R, K> ld;
    for (int i = 0; i < NVP_MAX_FIELDS; ++i) {
        const FieldArgs &f = a.f[i < a.nf ? i : 0];
        ld.f[i].p = static_cast<const cx<R> *>(f.p);
        ld.f[i].s0 = f.s0;
        ld.f[i].s1 = f.s1;
        for (int ax = 0; ax < 3; ++ax) {
            ld.f[i].b[ax] = f.b[ax];
            ld.f[i].w[ax] = static_cast<const R *>(f.w[ax]);
        }
        ld.f[i].identity = f.identity;
    }
    ld.nf = a.nf;
    ld.Nx = a.Nx;
    ld.Nz = a.Nz;
    switch (a.nf) {
    case 1: return source_nf<R, K, 1>(ld, a, out, Ny, cxl, s);
    case 2: return source_nf<R, K, 2>(ld, a, out, Ny, cxl, s);
    case 3: return source_nf<R, K, 3>(ld, a, out, Ny, cxl, s);
    case 4: return source_nf<R, K, 4>(ld, a, out, Ny, cxl, s);
    case 5: return source_nf<R, K, 5>(ld, a, out, Ny, cxl, s);
    case 6: return source_nf<R, K, 6>(ld, a, out, Ny, cxl, s);
    case 7: return source_nf<R, K, 7>(ld, a, out, Ny, cxl, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_source_c64(const SourceArgs &a, void *out, int Ny, int cxl, hipStream_t s) {
    if (a.order == 1) return source_k<float, 2>(a, out, Ny, cxl, s);
    if (a.order == 3) return source_k<float, 4>(a, out, Ny, cxl, s);
    return hipErrorInvalidValue;
}

hipError_t launch_source_c128(const SourceArgs &a, void *out, int Ny, int cxl, hipStream_t s) {
    if (a.order == 1) return source_k<double, 2>(a, out, Ny, cxl, s);
    if (a.order == 3) return source_k<double, 4>(a, out, Ny, cxl, s);
    return hipErrorInvalidValue;
}

bool length_supported(int L) { return plan_for(L).S > 0; }

int zconv_quads_override() {
    static const int v = [] {
        const char *e = getenv("NVP_ZCONV_QUADS");
        return e ? atoi(e) : 0;
    }();
    return v;
}

int strided_tile_cols(int L, int dbl) { return dbl ? strided_cols<double>(L) : strided_cols<float>(L); }

int zconv_slots_per_block(int L, int dbl) { return zconv_slots_for(L, dbl ? sizeof(double2) : sizeof(float2)); }

}  // namespace nvp
