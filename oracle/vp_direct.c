/*
 * ORACLE — test infrastructure only.  Plain FP64 direct evaluation of the
 * discrete volume potential; shares no code with the HIP library.
 *
 * For a uniform voxel grid of n[0] x n[1] x n[2] cubes of side h (C order,
 * z fastest, complex values interleaved re/im) and a source f, it computes
 *
 *     out_i = sum_j K(x_i - x_j) f_j
 *
 * with the quadrature of the paper's Section 3.1 (equation "quad"):
 *   off-diagonal voxels: midpoint rule, K(r) = h^3 exp(i k |r|) / (4 pi |r|)
 *     (the Green's function of equation "green" times the voxel volume);
 *   the self voxel: the exact integral of the Green's function over the
 *     sphere of equal volume, radius a = (3 / (4 pi))^(1/3) h,
 *     K(0) = (exp(i k a) (1 - i k a) - 1) / k^2.
 * The volume potential of equation "vol_pot_approx" is u = -out.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* K at integer voxel offset (dx, dy, dz), written out with real arithmetic. */
static void kernel_at(int64_t dx, int64_t dy, int64_t dz, double h, double kr, double ki,
                      double *re, double *im)
{
    if (dx == 0 && dy == 0 && dz == 0) {
        /* (e^{ika}(1 - ika) - 1) / k^2 */
        double a = cbrt(3.0 / (4.0 * M_PI)) * h;
        double ar = kr * a, ai = ki * a;            /* k a */
        double mag = exp(-ai);                      /* e^{i k a} = e^{-Im(ka)} (cos + i sin) Re(ka) */
        double er = mag * cos(ar), ei = mag * sin(ar);
        double br = 1.0 + ai, bi = -ar;             /* 1 - i k a */
        double nr = er * br - ei * bi - 1.0;
        double ni = er * bi + ei * br;
        double k2r = kr * kr - ki * ki, k2i = 2.0 * kr * ki;
        double den = k2r * k2r + k2i * k2i;
        *re = (nr * k2r + ni * k2i) / den;
        *im = (ni * k2r - nr * k2i) / den;
        return;
    }
    double dist = h * sqrt((double)(dx * dx + dy * dy + dz * dz));
    double mag = h * h * h * exp(-ki * dist) / (4.0 * M_PI * dist);
    *re = mag * cos(kr * dist);
    *im = mag * sin(kr * dist);
}

/* Tabulate K for offsets [0,n0) x [0,n1) x [0,n2) (C order, interleaved). */
int oracle_kernel_table(const int64_t n[3], double h, double kr, double ki, double *tab)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n[0]; ++a)
        for (int64_t b = 0; b < n[1]; ++b)
            for (int64_t c = 0; c < n[2]; ++c) {
                int64_t o = ((a * n[1] + b) * n[2] + c) * 2;
                kernel_at(a, b, c, h, kr, ki, &tab[o], &tab[o + 1]);
            }
    return 0;
}

static int64_t iabs64(int64_t v) { return v < 0 ? -v : v; }

/*
 * out[t] = sum_j K(x_{i_t} - x_j) f_j for targets i_t (flat C-order indices);
 * targets == NULL means every voxel, in order.  Returns 0, or 2 if the kernel
 * table cannot be allocated.
 */
int oracle_conv_direct(const int64_t n[3], double h, double kr, double ki, const double *f,
                       int64_t n_targets, const int64_t *targets, double *out)
{
    const int64_t N = n[0] * n[1] * n[2];
    double *tab = (double *)malloc((size_t)N * 2 * sizeof(double));
    if (!tab) return 2;
    oracle_kernel_table(n, h, kr, ki, tab);
    if (!targets) n_targets = N;

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < n_targets; ++t) {
        int64_t i = targets ? targets[t] : t;
        int64_t ix = i / (n[1] * n[2]), iy = (i / n[2]) % n[1], iz = i % n[2];
        double sr = 0.0, si = 0.0;
        for (int64_t jx = 0; jx < n[0]; ++jx) {
            int64_t ax = iabs64(ix - jx);
            for (int64_t jy = 0; jy < n[1]; ++jy) {
                int64_t ay = iabs64(iy - jy);
                const double *krow = tab + (ax * n[1] + ay) * n[2] * 2;
                const double *frow = f + (jx * n[1] + jy) * n[2] * 2;
                for (int64_t jz = 0; jz < n[2]; ++jz) {
                    int64_t az = iabs64(iz - jz);
                    double kre = krow[2 * az], kim = krow[2 * az + 1];
                    double fre = frow[2 * jz], fim = frow[2 * jz + 1];
                    sr += kre * fre - kim * fim;
                    si += kre * fim + kim * fre;
                }
            }
        }
        out[2 * t] = sr;
        out[2 * t + 1] = si;
    }
    free(tab);
    return 0;
}
