// Truncation boxes of a source term (Section 5).  (1) The localisation
// measure Q(x) = log10(|f(x)| / max |f|): for each threshold Q0 the smallest
// voxel box outside which Q < Q0, i.e. the bounding box of the voxels with
// |f|^2 >= 10^(2 Q0) max |f|^2.  Squared magnitudes are formed in FP64 without
// contraction (exact for complex64 inputs), so the integer box is reproducible.
// (2) The midpoint-rule potential at one voxel centre with the source
// restricted to each of a list of boxes (the truncation-convergence sweep).
#include <stdint.h>

#include "qbox.hpp"

namespace nvp {

namespace {

template <typename T> __device__ __forceinline__ double mag2(T v) {
    const double x = (double)v.x, y = (double)v.y;
    return __dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y));
}

// Block maxima of |f|^2 (grid-stride), one value per block.
template <typename T>
__global__ void __launch_bounds__(256) k_max(const T *__restrict__ f, int64_t n, double *__restrict__ part) {
    __shared__ double s[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, mag2(f[i]));
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_max_final(const double *__restrict__ part, int n, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m = fmax(m, part[i]);
        *out = m;
    }
}

__global__ void k_box_init(int *__restrict__ box, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count * 6) box[i] = (i % 6) < 3 ? 0x7fffffff : -1;  // lo = +inf, hi = -1
}

// box[q] = {lo_x, lo_y, lo_z, hi_x, hi_y, hi_z} over voxels with |f|^2 >= frac[q] * max.
template <typename T>
__global__ void __launch_bounds__(256) k_box(const T *__restrict__ f, int n0, int n1, int n2,
                                             const double *__restrict__ maxv, const double *__restrict__ frac,
                                             int count, int *__restrict__ box) {
    const int64_t n = (int64_t)n0 * n1 * n2;
    const double mx = *maxv;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double m = mag2(f[i]);
        const int x = (int)(i / ((int64_t)n1 * n2)), y = (int)((i / n2) % n1), z = (int)(i % n2);
        for (int q = 0; q < count; ++q) {
            if (m >= __dmul_rn(frac[q], mx)) {
                int *b = box + q * 6;
                atomicMin(b + 0, x);
                atomicMin(b + 1, y);
                atomicMin(b + 2, z);
                atomicMax(b + 3, x);
                atomicMax(b + 4, y);
                atomicMax(b + 5, z);
            }
        }
    }
}

}  // namespace

hipError_t qbox_launch(const void *f, bool dbl, const int64_t n[3], int count, const double *frac_dev,
                       double *work, int *box_dev, hipStream_t s) {
    const int64_t tot = n[0] * n[1] * n[2];
    const int blocks = 1024;
    double *part = work, *mx = work + blocks;
    if (dbl) hipLaunchKernelGGL(k_max<double2>, dim3(blocks), dim3(256), 0, s, (const double2 *)f, tot, part);
    else hipLaunchKernelGGL(k_max<float2>, dim3(blocks), dim3(256), 0, s, (const float2 *)f, tot, part);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(1), 0, s, part, blocks, mx);
    hipLaunchKernelGGL(k_box_init, dim3(1), dim3(256), 0, s, box_dev, count);
    if (dbl)
        hipLaunchKernelGGL(k_box<double2>, dim3(blocks), dim3(256), 0, s, (const double2 *)f, (int)n[0], (int)n[1],
                           (int)n[2], mx, frac_dev, count, box_dev);
    else
        hipLaunchKernelGGL(k_box<float2>, dim3(blocks), dim3(256), 0, s, (const float2 *)f, (int)n[0], (int)n[1],
                           (int)n[2], mx, frac_dev, count, box_dev);
    return hipGetLastError();
}

namespace {

// Midpoint-rule potential at one voxel centre t restricted to boxes:
// part[q][blk] = -sum over this block's share of the voxels j of box q
// (blockIdx.y) of K(x_t - x_j) f_j, K from the quadrature of Section 3.1 (self
// voxel: the ball integral, others: h^3 e^{ik|d|h} / (4 pi |d| h)), in FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_boxsum(const T *__restrict__ f, int n1, int n2, int t0, int t1, int t2,
                                                double h, double kr, double ki, double s_re, double s_im,
                                                double f_re, double f_im, const int *__restrict__ box,
                                                double2 *__restrict__ part) {
    __shared__ double2 red[256];
    const int q = blockIdx.y;
    const int lx = box[q * 6 + 0], ly = box[q * 6 + 1], lz = box[q * 6 + 2];
    const int ex = box[q * 6 + 3] - lx + 1, ey = box[q * 6 + 4] - ly + 1, ez = box[q * 6 + 5] - lz + 1;
    const int64_t nb = (ex > 0 && ey > 0 && ez > 0) ? (int64_t)ex * ey * ez : 0;
    const double c = h * h * h / (4.0 * 3.14159265358979323846);
    double ar = 0.0, ai = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = lx + (int)(i / ((int64_t)ey * ez)), y = ly + (int)((i / ez) % ey), z = lz + (int)(i % ez);
        double kre, kim;
        if (x == t0 && y == t1 && z == t2) {
            kre = s_re;
            kim = s_im;
        } else {
            const double dx = (double)(x - t0), dy = (double)(y - t1), dz = (double)(z - t2);
            const double rh = sqrt(dx * dx + dy * dy + dz * dz);
            const double r = h * rh;
            const double mag = c * exp(-ki * r) / r;
            double sn, cs;
            sincos(kr * r, &sn, &cs);
            kre = mag * cs;
            kim = mag * sn;
            if (abs(x - t0) + abs(y - t1) + abs(z - t2) == 1) {
                kre += f_re;
                kim += f_im;
            }
        }
        const T v = f[((int64_t)x * n1 + y) * n2 + z];
        const double vr = (double)v.x, vi = (double)v.y;
        ar -= kre * vr - kim * vi;
        ai -= kre * vi + kim * vr;
    }
    red[threadIdx.x] = make_double2(ar, ai);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[threadIdx.x].x += red[threadIdx.x + w].x;
            red[threadIdx.x].y += red[threadIdx.x + w].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)q * gridDim.x + blockIdx.x] = red[0];
}

// out[q] = sum over blocks, in block order.
__global__ void k_boxsum_final(const double2 *__restrict__ part, int blocks, int count, double2 *__restrict__ out) {
    const int q = threadIdx.x;
    if (blockIdx.x != 0 || q >= count) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < blocks; ++b) {
        sr += part[(size_t)q * blocks + b].x;
        si += part[(size_t)q * blocks + b].y;
    }
    out[q] = make_double2(sr, si);
}

}  // namespace

hipError_t boxsum_launch(const void *f, bool dbl, const int64_t n[3], const int t[3], double h, double kr, double ki,
                         double s_re, double s_im, double f_re, double f_im, const int *box_dev, int count,
                         double2 *work, double2 *out_dev, hipStream_t s) {
    const int blocks = NVP_BOXSUM_BLOCKS;
    if (dbl)
        hipLaunchKernelGGL(k_boxsum<double2>, dim3(blocks, count), dim3(256), 0, s, (const double2 *)f, (int)n[1],
                           (int)n[2], t[0], t[1], t[2], h, kr, ki, s_re, s_im, f_re, f_im, box_dev, work);
    else
        hipLaunchKernelGGL(k_boxsum<float2>, dim3(blocks, count), dim3(256), 0, s, (const float2 *)f, (int)n[1],
                           (int)n[2], t[0], t[1], t[2], h, kr, ki, s_re, s_im, f_re, f_im, box_dev, work);
    hipLaunchKernelGGL(k_boxsum_final, dim3(1), dim3(64), 0, s, work, blocks, count, out_dev);
    return hipGetLastError();
}

}  // namespace nvp
