// The transfer + source-build kernel (k_source), specialised on the number of
// transferred fields; launched from kspec.hip only.  The body is a plain
// function of its thread and workgroup indices so that it also runs on host
// threads (tests/fft_host/source_harness.cpp).
#pragma once

#include "field_dev.hpp"

namespace nvp {

// floor(a / b) for 0 <= a < 2^22 and b >= 1, given inv_b = 1/b in float:
// (a + 1/2) / b lies at least 1/(2b) from an integer, far more than the
// rounding of the float product.
__device__ __forceinline__ int div_small(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// f_n = sum_{m=1}^{n-1} T_m[p_m] T_{n-m}[p_{n-m}] on the target grid (the
// source of equation "cascade_2", Section 2), with T_m the separable K-point
// transfer of Section 6 from p_m's own grid.  NF = n - 1 fields.
//
// A workgroup owns a TY x TZ tile of target (y, z) columns and walks cx
// target x planes.  Because an axis table's base index never decreases along
// the axis, the source x planes a field needs arrive in order: each one is
// loaded once per workgroup (its SY x SZ block for the tile, coalesced along
// z, through LDS), interpolated along z and then y, and kept in a circular
// ring of the field's last K planes that every thread holds in registers for
// its own (y, z).  A target plane's x interpolation then reads only the
// ring.  A field's next plane is loaded into registers as soon as the
// current one is in LDS, so its latency overlaps the interpolation work in
// between; the tile's y and z weights and the chunk's x tables sit in LDS,
// so the only loads the loop waits for are the planes it consumes.  (Those
// loads are issued without branches, from addresses clamped into the block,
// and the ring is written and read at a workgroup-uniform position through
// uniform branches, so that the compiler never copies a register a load is
// still writing and never shifts the ring.)  All fields that advance at a
// target plane share two workgroup barriers.  Fields already on the target
// grid are read directly, each plane's value loaded before the plane's
// interpolation work and used after it.
//
// LDS (SrcLds, fixed offsets): per field a source-plane region of PRE TY TZ
// entries and a z-row region of 2 RY TY TZ entries, then per field the z and
// y weights ((TZ + RY TY) K reals), the x weights (CXM K reals) and the x
// stencils' ends (CXM ints).  Each thread owns RY target rows of the tile
// (ty, ty + TY, ...), which spreads the per-plane control and synchronisation
// over RY voxels.  Limits the host checks: SY <= 2 RY TY, SY * SZ <= PRE TY TZ,
// cx <= CXM and every grid below 2^32 elements (32-bit offsets).
template <typename R, int K, int NF, int TY, int TZ, int RY, int PRE, int CXM> struct SrcLds {
    static constexpr int NT = TY * TZ, TYT = RY * TY, ZR = 2 * RY, SREG = PRE * NT, TREG = ZR * NT;
    static constexpr size_t WOFF = (size_t)NF * (SREG + TREG) * sizeof(cx<R>);  // bytes
    static constexpr size_t WPER = (size_t)((TZ + TYT) * K + CXM * K) * sizeof(R);
    static constexpr size_t XOFF = WOFF + NF * WPER;
    static constexpr size_t BYTES = XOFF + (size_t)NF * CXM * sizeof(int);
    unsigned char *base;
    __device__ __forceinline__ cx<R> *plane(int i) const { return reinterpret_cast<cx<R> *>(base) + i * SREG; }
    __device__ __forceinline__ cx<R> *zrows(int i) const {
        return reinterpret_cast<cx<R> *>(base) + NF * SREG + i * TREG;
    }
    __device__ __forceinline__ R *wz(int i) const { return reinterpret_cast<R *>(base + WOFF + i * WPER); }
    __device__ __forceinline__ R *wy(int i) const { return wz(i) + TZ * K; }
    __device__ __forceinline__ R *wx(int i) const { return wz(i) + (TZ + TYT) * K; }
    __device__ __forceinline__ int *xend(int i) const { return reinterpret_cast<int *>(base + XOFF) + i * CXM; }
};

template <typename R, int K, int NF, int TY, int TZ, int RY, int PRE, int CXM>
__device__ __forceinline__ void source_tile(const LdSource<R, K> &src, cx<R> *__restrict__ out, int Ny, int cxl,
                                            unsigned char *lds, int tid, int bz, int by, int bx) {
    using L = SrcLds<R, K, NF, TY, TZ, RY, PRE, CXM>;
    constexpr int NT = L::NT, TYT = L::TYT, ZR = L::ZR;
    static_assert(NT >= TYT * K && NT >= TZ * K, "one weight per thread at set-up");
    static_assert(K == 2 || K == 4, "ring positions are taken modulo K with a mask");
    const L lay{lds};
    const int Nx = src.Nx, Nz = src.Nz;
    const int tz = tid % TZ, ty = tid / TZ;
    const int iz0 = bz * TZ, iy0 = by * TYT, ix0 = bx * cxl;
    const int iz1 = min(iz0 + TZ, Nz), iy1 = min(iy0 + TYT, Ny), ix1 = min(ix0 + cxl, Nx);
    const int iz = iz0 + tz;
    const bool okz = iz < Nz;
    int iy[RY];
    bool oky[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        iy[r] = iy0 + ty + r * TY;
        oky[r] = iy[r] < Ny;
    }
    auto plane = [](const FieldDev<R> &g, int x) { return g.p + (uint32_t)x * (uint32_t)g.s0; };

    int nxt[NF], endx[NF], blk[NF], szs[NF], sys[NF];  // workgroup-uniform
    int oz[NF], oy[NF][RY];
    uint32_t goff[NF][PRE];  // this thread's share of a plane's block, relative to the plane
    cx<R> pre[NF][PRE];      // the field's next plane, in flight
    cx<R> ring[NF][RY][K];   // source plane p, interpolated at (iy[r], iz), at ring[i][r][p % K]
    // a field on the target grid is read at (ix, iyc, izc), in bounds for every thread
    uint32_t idoff[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) idoff[r] = (uint32_t)min(iy[r], Ny - 1) * (uint32_t)Nz + (uint32_t)min(iz, Nz - 1);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const FieldDev<R> &g = src.f[i];
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int k = 0; k < K; ++k) ring[i][r][k] = czero<R>();
#pragma unroll
        for (int j = 0; j < PRE; ++j) pre[i][j] = czero<R>();
        if (g.identity) {
            nxt[i] = endx[i] = blk[i] = szs[i] = sys[i] = oz[i] = 0;
#pragma unroll
            for (int r = 0; r < RY; ++r) oy[i][r] = 0;
#pragma unroll
            for (int j = 0; j < PRE; ++j) goff[i][j] = 0;
            continue;
        }
        const int sy0 = g.b[1][iy0], sz0 = g.b[2][iz0];
        sys[i] = g.b[1][iy1 - 1] + K - sy0;
        szs[i] = g.b[2][iz1 - 1] + K - sz0;
        blk[i] = sys[i] * szs[i];
        nxt[i] = g.b[0][ix0];
        endx[i] = g.b[0][ix1 - 1] + K;
        const float inv = 1.0f / (float)szs[i];
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
            const int e = tid + j * NT;
            const int r = div_small(e, inv), c = e - r * szs[i];
            // beyond the block: the block's first entry (loaded, never stored)
            goff[i][j] = e < blk[i] ? (uint32_t)(sy0 + r) * (uint32_t)g.s1 + (uint32_t)(sz0 + c)
                                    : (uint32_t)sy0 * (uint32_t)g.s1 + (uint32_t)sz0;
            pre[i][j] = plane(g, nxt[i])[goff[i][j]];
        }
        oz[i] = okz ? g.b[2][iz] - sz0 : 0;
#pragma unroll
        for (int r = 0; r < RY; ++r) oy[i][r] = oky[r] ? g.b[1][iy[r]] - sy0 : 0;
        // the tile's z and y weights (zero beyond the grid) and the chunk's x tables
        R *wz = lay.wz(i), *wy = lay.wy(i), *wx = lay.wx(i);
        int *xe = lay.xend(i);
        if (tid < TZ * K) wz[tid] = iz0 + tid / K < Nz ? g.w[2][iz0 * K + tid] : R(0);
        if (tid < TYT * K) wy[tid] = iy0 + tid / K < Ny ? g.w[1][iy0 * K + tid] : R(0);
        for (int e = tid; e < (ix1 - ix0) * K; e += NT) wx[e] = g.w[0][ix0 * K + e];
        for (int e = tid; e < ix1 - ix0; e += NT) xe[e] = g.b[0][ix0 + e] + K;
    }
    __syncthreads();

    for (int ix = ix0; ix < ix1; ++ix) {
        cx<R> idv[NF][RY];
#pragma unroll
        for (int i = 0; i < NF; ++i)
            if (src.f[i].identity) {
#pragma unroll
                for (int r = 0; r < RY; ++r) idv[i][r] = plane(src.f[i], ix)[idoff[r]];
            }
        int need[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i)
            need[i] = src.f[i].identity ? 0 : __builtin_amdgcn_readfirstlane(lay.xend(i)[ix - ix0]);
        // advance every field whose ring does not yet end at its stencil's last plane
        for (;;) {
            unsigned act = 0;  // bit i: field i advances
#pragma unroll
            for (int i = 0; i < NF; ++i) act |= nxt[i] < need[i] ? 1u << i : 0u;
            if (!act) break;
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                if (!(act >> i & 1)) continue;
                cx<R> *S = lay.plane(i);
#pragma unroll
                for (int j = 0; j < PRE; ++j)
                    if (tid + j * NT < blk[i]) S[tid + j * NT] = pre[i][j];
                // the next plane (the last one again at the chunk's end)
                const cx<R> *P = plane(src.f[i], min(nxt[i] + 1, endx[i] - 1));
#pragma unroll
                for (int j = 0; j < PRE; ++j) pre[i][j] = P[goff[i][j]];
            }
            __syncthreads();
            // z: rows ty, ty + TY, ... of the block, at this thread's z stencil
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                if (!(act >> i & 1)) continue;
                const cx<R> *S = lay.plane(i);
                cx<R> *T = lay.zrows(i);
                const R *wz = lay.wz(i) + tz * K;
                R w[K];
#pragma unroll
                for (int d = 0; d < K; ++d) w[d] = wz[d];
#pragma unroll
                for (int h = 0; h < ZR; ++h) {
                    const int row = ty + h * TY;
                    if (row < sys[i]) {
                        cx<R> acc = czero<R>();
#pragma unroll
                        for (int d = 0; d < K; ++d) acc = cadd<R>(acc, cscale<R>(S[row * szs[i] + oz[i] + d], w[d]));
                        T[row * TZ + tz] = acc;
                    }
                }
            }
            __syncthreads();
            // y: this thread's (iy[r], iz), into the ring at the plane's position
#pragma unroll
            for (int i = 0; i < NF; ++i) {
                if (!(act >> i & 1)) continue;
                const cx<R> *T = lay.zrows(i);
                const int pos = nxt[i] & (K - 1);
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const R *wy = lay.wy(i) + (ty + r * TY) * K;
                    cx<R> acc = czero<R>();
#pragma unroll
                    for (int c = 0; c < K; ++c) acc = cadd<R>(acc, cscale<R>(T[(oy[i][r] + c) * TZ + tz], wy[c]));
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (pos == k) ring[i][r][k] = acc;
                }
                ++nxt[i];
            }
        }
        // x: the ring holds planes need - K .. need - 1, the stencil of ix;
        // plane need - K + b sits at (need + b) % K
        cx<R> v[NF][RY];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const FieldDev<R> &g = src.f[i];
            if (g.identity) {
#pragma unroll
                for (int r = 0; r < RY; ++r) v[i][r] = idv[i][r];
                continue;
            }
            const R *wx = lay.wx(i) + (ix - ix0) * K;
            R w[K];
#pragma unroll
            for (int b = 0; b < K; ++b) w[b] = wx[b];
            const int pos = need[i] & (K - 1);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                cx<R> acc = czero<R>();
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (pos == k) {
#pragma unroll
                        for (int b = 0; b < K; ++b) acc = cadd<R>(acc, cscale<R>(ring[i][r][(k + b) & (K - 1)], w[b]));
                    }
                v[i][r] = acc;
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (oky[r] && okz) {
                // sum_{b + c = NF - 1} v_b v_c, the source term of harmonic NF + 1
                cx<R> f = czero<R>();
#pragma unroll
                for (int b = 0; b < NF; ++b) f = cadd<R>(f, cmul<R>(v[b][r], v[NF - 1 - b][r]));
                out[((uint32_t)ix * (uint32_t)Ny + (uint32_t)iy[r]) * (uint32_t)Nz + (uint32_t)iz] = f;
            }
    }
}

#ifndef NVP_HOST_EMULATION
extern __shared__ __align__(16) unsigned char nvp_smem[];

template <typename R, int K, int NF, int TY, int TZ, int RY, int PRE, int CXM>
__global__ void __launch_bounds__(TY *TZ)
k_source(LdSource<R, K> src, cx<R> *__restrict__ out, int Ny, int cxl) {
    source_tile<R, K, NF, TY, TZ, RY, PRE, CXM>(src, out, Ny, cxl, nvp_smem, (int)threadIdx.x, (int)blockIdx.x,
                                                (int)blockIdx.y, (int)blockIdx.z);
}
#endif

}  // namespace nvp
