// FP64 kernel tabulation and the FP64 passes of the kernel spectrum.
#include <math.h>
#include <stdlib.h>

#include "passes_impl.hpp"

namespace nvp {

__global__ void k_ktab(double2 *__restrict__ out, int64_t Hx, int64_t Hy, int64_t Hz, int64_t Nx, int64_t Ny,
                       int64_t Nz, double h, double kr, double ki, double2 self) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Hx * Hy * Hz) return;
    const int64_t i = idx / (Hy * Hz), rem = idx % (Hy * Hz), j = rem / Hz, k = rem % Hz;
    double2 v = make_double2(0.0, 0.0);
    if (i < Nx && j < Ny && k < Nz) {
        if (i == 0 && j == 0 && k == 0) {
            v = self;
        } else {
            const double d = h * sqrt((double)(i * i + j * j + k * k));
            const double mag = h * h * h * exp(-ki * d) / (4.0 * M_PI * d);
            double sn, cs;
            sincos(kr * d, &sn, &cs);
            v = make_double2(mag * cs, mag * sn);
        }
    }
    out[idx] = v;
}

hipError_t launch_ktab(double2 *out, const int64_t H[3], const int64_t N[3], double h, double kr, double ki,
                       double self_re, double self_im, hipStream_t s) {
    const int64_t tot = H[0] * H[1] * H[2];
    const int bs = 256;
    hipLaunchKernelGGL(k_ktab, dim3((unsigned)((tot + bs - 1) / bs)), dim3(bs), 0, s, out, H[0], H[1], H[2], N[0],
                       N[1], N[2], h, kr, ki, make_double2(self_re, self_im));
    return hipGetLastError();
}

template <typename R, int K>
static hipError_t source_k(const SourceArgs &a, void *out, int Ny, int64_t lds_elems, hipStream_t s) {
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
    auto kern = k_source<R, K, NVP_SRC_TX, NVP_SRC_TY, NVP_SRC_TZ>;
    const size_t lds = (size_t)lds_elems * sizeof(cx<R>);
    hipError_t e = allow_lds(kern, lds > 65536 ? 163840 : lds);
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((a.Nz + NVP_SRC_TZ - 1) / NVP_SRC_TZ), (unsigned)((Ny + NVP_SRC_TY - 1) / NVP_SRC_TY),
              (unsigned)((a.Nx + NVP_SRC_TX - 1) / NVP_SRC_TX));
    hipLaunchKernelGGL(kern, grid, dim3(NVP_SRC_TY * NVP_SRC_TZ), lds, s, ld, static_cast<cx<R> *>(out), Ny,
                       lds_elems);
    return hipGetLastError();
}

hipError_t launch_source_c64(const SourceArgs &a, void *out, int Ny, int64_t lds_elems, hipStream_t s) {
    if (a.order == 1) return source_k<float, 2>(a, out, Ny, lds_elems, s);
    if (a.order == 3) return source_k<float, 4>(a, out, Ny, lds_elems, s);
    return hipErrorInvalidValue;
}

hipError_t launch_source_c128(const SourceArgs &a, void *out, int Ny, int64_t lds_elems, hipStream_t s) {
    if (a.order == 1) return source_k<double, 2>(a, out, Ny, lds_elems, s);
    if (a.order == 3) return source_k<double, 4>(a, out, Ny, lds_elems, s);
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
int threads_per_column(int L) { return plan_threads(L); }

}  // namespace nvp
