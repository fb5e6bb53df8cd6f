// Exhaustive check of the kernel-tabulation tasks (paper_2011_03009_amd/csrc/kz_tasks.hpp):
// for each octant shape, every row is written by exactly one task (twice-written
// rows are the mirror pairs of one task), every index lies in the octant, a
// pair's rows are (i, j) and (j, i) inside the square of nonzero rows, and each
// task's (i, j) names its first row.  Prints "OK <shapes>" or a diagnostic.
#define NVP_HOST_EMULATION 1
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hip/hip_runtime.h"
void __syncthreads() {}
namespace nvp {
inline void wave_sync() {}
}  // namespace nvp

#include "kz_tasks.hpp"

using namespace nvp;

#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");        \
            std::exit(1);                      \
        }                                      \
    } while (0)

int main() {
    // (Hx, Hy, Nx, Ny): octant rows M/2 + 1 >= N, nonzero rows below N
    const int64_t shapes[][4] = {{257, 257, 256, 256}, {321, 257, 320, 256}, {385, 257, 384, 256},
                                 {449, 257, 448, 256}, {257, 449, 256, 448}, {1, 1, 1, 1},
                                 {2, 3, 1, 2},         {9, 5, 8, 3},         {5, 9, 5, 9},
                                 {577, 577, 568, 568}, {721, 577, 716, 568}, {2049, 33, 2000, 17}};
    int n = 0;
    for (const auto &sh : shapes) {
        const int64_t Hx = sh[0], Hy = sh[1], Nx = sh[2], Ny = sh[3];
        const int64_t S = Nx < Ny ? Nx : Ny;
        const int64_t T = kz_task_count(Hx, Hy, S);
        std::vector<int> hits((size_t)(Hx * Hy), 0);
        for (int64_t q = 0; q < T; ++q) {
            const KzTask t = kz_task(q, Hx, Hy, S);
            CHECK(t.i >= 0 && t.i < Hx && t.j >= 0 && t.j < Hy, "task %lld of %lldx%lld: (%d, %d) outside",
                  (long long)q, (long long)Hx, (long long)Hy, t.i, t.j);
            CHECK(t.r0 == (int64_t)t.i * Hy + t.j, "task %lld: first row %lld is not (%d, %d)", (long long)q,
                  (long long)t.r0, t.i, t.j);
            if (t.r1 != t.r0) {
                CHECK(t.i < t.j && t.j < S && t.r1 == (int64_t)t.j * Hy + t.i, "task %lld: bad pair", (long long)q);
                ++hits[(size_t)t.r1];
            }
            ++hits[(size_t)t.r0];
        }
        for (int64_t r = 0; r < Hx * Hy; ++r)
            CHECK(hits[(size_t)r] == 1, "%lldx%lld (N %lldx%lld): row %lld written %d times", (long long)Hx,
                  (long long)Hy, (long long)Nx, (long long)Ny, (long long)r, hits[(size_t)r]);
        CHECK(T == S * (S + 1) / 2 + Hx * Hy - S * S, "task count");
        ++n;
    }
    std::printf("OK %d\n", n);
    return 0;
}
