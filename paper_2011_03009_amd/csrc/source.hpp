// The transfer + source-build kernel (k_source), specialised on the number
// of transferred fields; launched from kspec.hip only.
#pragma once

#include "kernels.hpp"

namespace nvp {

// Transfer + source build as a kernel of its own (writes f_n, read by a plain
// forward x pass afterwards), compiled for each field count NF = n - 1.  One workgroup per target tile of TX x TY x TZ
// voxels (z fastest); for every field that needs interpolating it loads the
// source block the tile's stencils touch into LDS once (coalesced along z),
// interpolates along z inside LDS, then along y and x in registers (a thread
// owns one (y, z) column of the tile); fields on the target grid are read
// directly.  Two workgroup barriers per field.  Each thread keeps its voxels'
// interpolated values in registers and finally writes sum_m v_m v_{n-m}.  The
// host checks that the source blocks of every tile fit the LDS budget given
// at launch and that their x spans fit the registers.
// floor(a / b) for 0 <= a < 2^22 and b >= 1, given inv_b = 1/b in float:
// (a + 1/2) / b lies at least 1/(2b) from an integer, far more than the
// rounding of the float product.
__device__ __forceinline__ int div_small(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

template <typename R, int K, int NF, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TY *TZ)
k_source(LdSource<R, K> src, cx<R> *__restrict__ out, int Ny, int64_t lds_elems) {
    cx<R> *lds = reinterpret_cast<cx<R> *>(nvp_smem);
    const int Nx = src.Nx, Nz = src.Nz;
    const int tz = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    const int ix0 = blockIdx.z * TX, iy0 = blockIdx.y * TY, iz0 = blockIdx.x * TZ;
    const int ix1 = min(ix0 + TX, Nx), iy1 = min(iy0 + TY, Ny), iz1 = min(iz0 + TZ, Nz);
    const int iy = iy0 + ty, iz = iz0 + tz;
    const bool inyz = iy < Ny && iz < Nz;
    // element offsets in 32 bits: the host checks that every grid involved
    // has fewer than 2^32 elements
    auto at = [](const FieldDev<R> &g, int x, int y, int z) {
        return g.p + ((uint32_t)x * (uint32_t)g.s0 + (uint32_t)y * (uint32_t)g.s1 + (uint32_t)z);
    };
    cx<R> v[NF][TX];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int a = 0; a < TX; ++a) v[i][a] = czero<R>();
    // A field's source block [sx0, sx0+SX) x [sy0, sy0+SY) x [sz0, sz0+SZ).
    struct Block {
        int sx0, sy0, sz0, SX, SY, SZ;
    };
    auto block_of = [&](const FieldDev<R> &g) {
        Block b;
        b.sx0 = g.b[0][ix0];
        b.sy0 = g.b[1][iy0];
        b.sz0 = g.b[2][iz0];
        b.SX = g.b[0][ix1 - 1] + K - b.sx0;
        b.SY = g.b[1][iy1 - 1] + K - b.sy0;
        b.SZ = g.b[2][iz1 - 1] + K - b.sz0;
        return b;
    };
    // The next field's block is loaded into registers (up to PR rows of PZ
    // z-values per thread) while this one is interpolated, so that its load
    // latency overlaps the work; a larger block is loaded when it is reached.
    // (complex64 only: complex128 values would spill registers)
    constexpr bool PIPE = sizeof(R) == 4;
    constexpr int PR = PIPE ? 10 : 1, PZ = 1;
    cx<R> pre[PR][PZ];
    int pre_field = -1;
    auto fits = [&](const Block &b) { return PIPE && b.SX * b.SY <= PR * TY && b.SZ <= PZ * TZ; };
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const FieldDev<R> &g = src.f[i];
        if (g.identity) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
                if (inyz && ix0 + a < Nx) v[i][a] = *at(g, ix0 + a, iy, iz);
            continue;
        }
        const Block bk = block_of(g);
        const int sx0 = bk.sx0, sy0 = bk.sy0, sz0 = bk.sz0, SX = bk.SX, SY = bk.SY, SZ = bk.SZ;
        const int rows = SX * SY;
        const float inv_sy = 1.0f / (float)SY;
        cx<R> *S = lds;                         // [SX][SY][SZ]
        cx<R> *T1 = lds + (lds_elems - (int64_t)rows * TZ);  // [SX][SY][TZ]
        // the tile's z and y stencils: one per thread (z = tz, y = ty), loaded
        // before the block so that their latency overlaps its loads
        const int zz = iz0 + tz, yy = iy0 + ty;
        const bool okz = zz < Nz, oky = yy < Ny;
        const int oz = okz ? g.b[2][zz] - sz0 : 0, oy = oky ? g.b[1][yy] - sy0 : 0;
        // a voxel's K weights are contiguous and aligned to their size (the
        // host aligns each table to 256 bytes): one vector load each
        struct alignas(sizeof(R) * K) Wk {
            R v[K];
        };
        R wx[TX][K];
        int ox[TX];
        const Wk wzv = okz ? *reinterpret_cast<const Wk *>(g.w[2] + zz * K) : Wk{};
        const Wk wyv = oky ? *reinterpret_cast<const Wk *>(g.w[1] + yy * K) : Wk{};
        const R *wz = wzv.v, *wy = wyv.v;
#pragma unroll
        for (int a = 0; a < TX; ++a) {
            const bool okx = ix0 + a < Nx;
            ox[a] = okx ? g.b[0][ix0 + a] - sx0 : 0;
#pragma unroll
            for (int b = 0; b < K; ++b) wx[a][b] = okx ? g.w[0][(ix0 + a) * K + b] : R(0);
        }
        // rows of SZ contiguous source values, TZ lanes per row
        if (pre_field == i) {
#pragma unroll
            for (int r = 0; r < PR; ++r) {
                const int row = ty + r * TY;
#pragma unroll
                for (int z = 0; z < PZ; ++z) {
                    const int sz = tz + z * TZ;
                    if (row < rows && sz < SZ) S[row * SZ + sz] = pre[r][z];
                }
            }
        } else {
            for (int row = ty; row < rows; row += TY) {
                const int sx = div_small(row, inv_sy), sy = row - sx * SY;
                const cx<R> *sp = at(g, sx0 + sx, sy0 + sy, sz0);
                for (int sz = tz; sz < SZ; sz += TZ) S[row * SZ + sz] = sp[sz];
            }
        }
        __syncthreads();
        if (i + 1 < NF && !src.f[i + 1 < NF ? i + 1 : i].identity) {
            const FieldDev<R> &gn = src.f[i + 1 < NF ? i + 1 : i];
            const Block nb = block_of(gn);
            if (fits(nb)) {
#pragma unroll
                for (int r = 0; r < PR; ++r) {
                    const int row = ty + r * TY;
                    const int sx = div_small(row, 1.0f / (float)nb.SY), sy = row - sx * nb.SY;
                    const cx<R> *sp = at(gn, nb.sx0 + sx, nb.sy0 + sy, nb.sz0);
#pragma unroll
                    for (int z = 0; z < PZ; ++z) {
                        const int sz = tz + z * TZ;
                        if (row < nb.SX * nb.SY && sz < nb.SZ) pre[r][z] = sp[sz];
                    }
                }
                pre_field = i + 1;
            }
        }
        // z interpolation: T1[row][z] for this thread's z
        for (int row = ty; row < rows; row += TY) {
            cx<R> acc = czero<R>();
#pragma unroll
            for (int d = 0; d < K; ++d) acc = cadd<R>(acc, cscale<R>(S[row * SZ + oz + d], wz[d]));
            T1[row * TZ + tz] = acc;
        }
        __syncthreads();
        // y interpolation of this thread's (y, z) for every source x-row of
        // the block, kept in registers: the x stencils of a tile span at most
        // TX - 1 + K rows (the host checks it)
        constexpr int SXM = TX - 1 + K;
        cx<R> t2[SXM];
#pragma unroll
        for (int sx = 0; sx < SXM; ++sx) {
            cx<R> acc = czero<R>();
            if (sx < SX) {
#pragma unroll
                for (int c = 0; c < K; ++c)
                    acc = cadd<R>(acc, cscale<R>(T1[((sx * SY) + oy + c) * TZ + tz], wy[c]));
            }
            t2[sx] = acc;
        }
        // x interpolation: the stencil offset of target row a is the same for
        // the whole workgroup, so the branch on it is uniform
#pragma unroll
        for (int a = 0; a < TX; ++a) {
            if (ix0 + a < Nx) {
                const int o = __builtin_amdgcn_readfirstlane(ox[a]);
                cx<R> acc = czero<R>();
#pragma unroll
                for (int q = 0; q < TX; ++q)
                    if (o == q) {
#pragma unroll
                        for (int b = 0; b < K; ++b) acc = cadd<R>(acc, cscale<R>(t2[q + b], wx[a][b]));
                    }
                v[i][a] = acc;
            }
        }
    }
    if (!inyz) return;
#pragma unroll
    for (int a = 0; a < TX; ++a) {
        const int ix = ix0 + a;
        if (ix >= Nx) break;
        // sum_{b + c = NF - 1} v_b v_c, the source term of harmonic NF + 1
        cx<R> f = czero<R>();
#pragma unroll
        for (int b = 0; b < NF; ++b) f = cadd<R>(f, cmul<R>(v[b][a], v[NF - 1 - b][a]));
        out[((uint32_t)ix * (uint32_t)Ny + (uint32_t)iy) * (uint32_t)Nz + (uint32_t)iz] = f;
    }
}

}  // namespace nvp
