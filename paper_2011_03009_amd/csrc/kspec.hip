// FP64 kernel tabulation and the FP64 passes of the kernel spectrum.
#include <math.h>
#include <stdlib.h>

#include "kernels.hpp"

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
