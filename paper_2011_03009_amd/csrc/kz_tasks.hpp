// Tasks of the kernel-tabulation pass (k_kz): which octant rows a task fills.
//
// Octant row (i, j), 0 <= i < Hx, 0 <= j < Hy, holds the z transform of the
// kernel at the offsets (i, j, k); the kernel depends on the offset only
// through i^2 + j^2 + k^2 and vanishes for i >= Nx or j >= Ny.  Rows (i, j)
// and (j, i) of the square S x S, S = min(Nx, Ny), are therefore equal, and
// one task computes both.  Task q < S (S + 1) / 2 is the pair (i, j), i <= j,
// of the upper triangle; the remaining tasks are the rows outside the square,
// one each: first i >= S (all j), then i < S, j >= S.
#pragma once

#include <math.h>
#include <stdint.h>

#include "fft_core.hpp"

namespace nvp {

struct KzTask {
    int64_t r0, r1;  // rows r0 = i Hy + j and r1 = j Hy + i (r1 = r0 on the diagonal and outside the square)
    int i, j;
};

__host__ __device__ constexpr int64_t kz_task_count(int64_t Hx, int64_t Hy, int64_t S) {
    return S * (S + 1) / 2 + Hx * Hy - S * S;
}

// Task q in [0, kz_task_count); S <= min(Hx, Hy) and S < 2^26.
__host__ __device__ inline KzTask kz_task(int64_t q, int64_t Hx, int64_t Hy, int64_t S) {
    KzTask t;
    const int64_t T1 = S * (S + 1) / 2;
    if (q < T1) {
        // j (j + 1) / 2 <= q < (j + 1) (j + 2) / 2
        int64_t j = (int64_t)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
        while (j * (j + 1) / 2 > q) --j;
        while ((j + 1) * (j + 2) / 2 <= q) ++j;
        const int64_t i = q - j * (j + 1) / 2;
        t.i = (int)i;
        t.j = (int)j;
        t.r0 = i * Hy + j;
        t.r1 = j * Hy + i;
        return t;
    }
    int64_t r = q - T1;
    const int64_t below = (Hx - S) * Hy;  // rows i >= S
    if (r < below) {
        t.i = (int)(S + r / Hy);
        t.j = (int)(r % Hy);
    } else {
        r -= below;
        t.i = (int)(r / (Hy - S));
        t.j = (int)(S + r % (Hy - S));
    }
    t.r0 = t.r1 = (int64_t)t.i * Hy + t.j;
    return t;
}

}  // namespace nvp
