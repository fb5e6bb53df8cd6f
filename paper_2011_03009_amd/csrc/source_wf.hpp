// The transfer + source-build kernel with one wavefront per transferred field
// (k_source_wf); launched from kspec.hip only.  The body is a plain function
// of its thread and workgroup indices so that it also runs on host threads
// (tests/fft_host/source_harness.cpp).
#pragma once

#include "field_dev.hpp"

namespace nvp {

// f_n = sum_{m=1}^{n-1} T_m[p_m] T_{n-m}[p_{n-m}] on the target grid (the
// source of equation "cascade_2", Section 2), with T_m the separable K-point
// transfer of Section 6 from p_m's own grid.  NF = n - 1 fields.
//
// A workgroup of NF wavefronts owns a tile of 8 x 32 target (y, z) columns
// and walks cx target x planes; wavefront w transfers field w for the whole
// tile, each lane for the four voxels (ty0 + 2h, tz), h < 4.  Because an axis
// table's base index never decreases along the axis, the source x planes a
// field needs arrive in order: the wavefront loads each one once (its SY x SZ
// block for the tile, coalesced along z, into its own LDS region),
// interpolates it along z and then y, and keeps it in a circular ring of the
// last K planes in registers; a target plane's x interpolation reads only the
// ring.  Every step of a field's plane pipeline stays inside its wavefront,
// so it synchronises with wave_sync only, and the next plane is loaded into
// registers as soon as the current one is in LDS.  Per target plane the
// wavefronts exchange their interpolated values through LDS (two buffers, by
// the plane's parity) with one workgroup barrier, then each forms the source
// product for its share of the tile's voxels.  A field already on the target
// grid is read directly.
//
// LDS (SrcWfLds, fixed offsets): per field a source-plane region of PREW 64
// entries and a z-row region of 16 x 32 entries; two exchange buffers of NF x
// 256 entries; then per field the x weights (CXM K reals) and the x stencils'
// ends (CXM ints).  Limits the host checks: SY <= 16, SY * SZ <= 64 PREW,
// cx <= CXM and every grid below 2^32 elements (32-bit offsets).
template <typename R, int K, int NF, int PREW, int CXM> struct SrcWfLds {
    static constexpr int TZ = 32, TYT = 8, NV = TYT * TZ, ZRM = 16;
    static constexpr int SREG = PREW * 64, TREG = ZRM * TZ;
    static constexpr size_t VOFF = (size_t)NF * (SREG + TREG) * sizeof(cx<R>);
    static constexpr size_t WOFF = VOFF + (size_t)2 * NF * NV * sizeof(cx<R>);
    static constexpr size_t XOFF = WOFF + (size_t)NF * CXM * K * sizeof(R);
    static constexpr size_t BYTES = XOFF + (size_t)NF * CXM * sizeof(int);
    unsigned char *base;
    __device__ __forceinline__ cx<R> *plane(int i) const { return reinterpret_cast<cx<R> *>(base) + i * SREG; }
    __device__ __forceinline__ cx<R> *zrows(int i) const {
        return reinterpret_cast<cx<R> *>(base) + NF * SREG + i * TREG;
    }
    __device__ __forceinline__ cx<R> *vals(int par, int i) const {
        return reinterpret_cast<cx<R> *>(base + VOFF) + (par * NF + i) * NV;
    }
    __device__ __forceinline__ R *wx(int i) const { return reinterpret_cast<R *>(base + WOFF) + i * CXM * K; }
    __device__ __forceinline__ int *xend(int i) const { return reinterpret_cast<int *>(base + XOFF) + i * CXM; }
};

template <typename R, int K, int NF, int PREW, int CXM>
__device__ __forceinline__ void source_tile_wf(const LdSource<R, K> &src, cx<R> *__restrict__ out, int Ny, int cxl,
                                               unsigned char *lds, int tid, int bz, int by, int bx) {
    using L = SrcWfLds<R, K, NF, PREW, CXM>;
    constexpr int TZ = L::TZ, TYT = L::TYT, NV = L::NV, VL = NV / 64;
    static_assert(K == 2 || K == 4, "ring positions are taken modulo K with a mask");
    static_assert(VL == 4 && TZ == 32, "a lane owns the voxels (ty0 + 2h, tz) of the tile");
    const L lay{lds};
    const int Nx = src.Nx, Nz = src.Nz;
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tz = lane & (TZ - 1), ty0 = lane >> 5;
    const int iz0 = bz * TZ, iy0 = by * TYT, ix0 = bx * cxl;
    const int iz1 = min(iz0 + TZ, Nz), iy1 = min(iy0 + TYT, Ny), ix1 = min(ix0 + cxl, Nx);
    const int iz = iz0 + tz;
    const bool okz = iz < Nz;
    const FieldDev<R> &g = src.f[w];
    const bool ident = g.identity != 0;
    auto plane = [&](int x) { return g.p + (uint32_t)x * (uint32_t)g.s0; };

    int nxt = 0, endx = 0, blk = 0, szs = 0, sys = 0, oz = 0;  // wavefront-uniform but oz
    int oy[VL];
    uint32_t goff[PREW], idoff[VL];
    cx<R> pre[PREW];
    cx<R> ring[VL][K];  // source plane p, interpolated at this lane's voxel h, at ring[h][p % K]
    R wz[K], wy[VL][K];
#pragma unroll
    for (int h = 0; h < VL; ++h) {
        const int iy = iy0 + ty0 + 2 * h;
        idoff[h] = (uint32_t)min(iy, Ny - 1) * (uint32_t)Nz + (uint32_t)min(iz, Nz - 1);
        oy[h] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            ring[h][k] = czero<R>();
            wy[h][k] = R(0);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) wz[k] = R(0);
#pragma unroll
    for (int j = 0; j < PREW; ++j) {
        goff[j] = 0;
        pre[j] = czero<R>();
    }
    if (!ident) {
        const int sy0 = g.b[1][iy0], sz0 = g.b[2][iz0];
        sys = g.b[1][iy1 - 1] + K - sy0;
        szs = g.b[2][iz1 - 1] + K - sz0;
        blk = sys * szs;
        nxt = g.b[0][ix0];
        endx = g.b[0][ix1 - 1] + K;
        const float inv = 1.0f / (float)szs;
#pragma unroll
        for (int j = 0; j < PREW; ++j) {
            const int e = lane + j * 64;
            const int r = div_small(e, inv), c = e - r * szs;
            // beyond the block: the block's first entry (loaded, never stored)
            goff[j] = e < blk ? (uint32_t)(sy0 + r) * (uint32_t)g.s1 + (uint32_t)(sz0 + c)
                              : (uint32_t)sy0 * (uint32_t)g.s1 + (uint32_t)sz0;
            pre[j] = plane(nxt)[goff[j]];
        }
        if (okz) {
            oz = g.b[2][iz] - sz0;
#pragma unroll
            for (int k = 0; k < K; ++k) wz[k] = g.w[2][iz * K + k];
        }
#pragma unroll
        for (int h = 0; h < VL; ++h) {
            const int iy = iy0 + ty0 + 2 * h;
            if (iy < Ny) {
                oy[h] = g.b[1][iy] - sy0;
#pragma unroll
                for (int k = 0; k < K; ++k) wy[h][k] = g.w[1][iy * K + k];
            }
        }
        // the chunk's x tables, read by this wavefront only
        R *wx = lay.wx(w);
        int *xe = lay.xend(w);
        for (int e = lane; e < (ix1 - ix0) * K; e += 64) wx[e] = g.w[0][ix0 * K + e];
        for (int e = lane; e < ix1 - ix0; e += 64) xe[e] = g.b[0][ix0 + e] + K;
        wave_sync();
    }

    int par = 0;
    for (int ix = ix0; ix < ix1; ++ix, par ^= 1) {
        cx<R> v[VL];
        if (ident) {
#pragma unroll
            for (int h = 0; h < VL; ++h) v[h] = plane(ix)[idoff[h]];
        } else {
            const int need = __builtin_amdgcn_readfirstlane(lay.xend(w)[ix - ix0]);
            cx<R> *S = lay.plane(w);
            cx<R> *T = lay.zrows(w);
            // advance the ring until it ends at the stencil's last plane
            while (nxt < need) {
#pragma unroll
                for (int j = 0; j < PREW; ++j)
                    if (lane + j * 64 < blk) S[lane + j * 64] = pre[j];
                // the next plane (the last one again at the chunk's end)
                const cx<R> *P = plane(min(nxt + 1, endx - 1));
#pragma unroll
                for (int j = 0; j < PREW; ++j) pre[j] = P[goff[j]];
                wave_sync();
                // z: rows ty0, ty0 + 2, ... of the block, at this lane's z stencil
#pragma unroll
                for (int q = 0; q < L::ZRM / 2; ++q) {
                    const int row = ty0 + 2 * q;
                    if (row < sys) {
                        cx<R> acc = czero<R>();
#pragma unroll
                        for (int d = 0; d < K; ++d) acc = cadd<R>(acc, cscale<R>(S[row * szs + oz + d], wz[d]));
                        T[row * TZ + tz] = acc;
                    }
                }
                wave_sync();
                // y: this lane's voxels, into the ring at the plane's position
                const int pos = nxt & (K - 1);
#pragma unroll
                for (int h = 0; h < VL; ++h) {
                    cx<R> acc = czero<R>();
#pragma unroll
                    for (int c = 0; c < K; ++c) acc = cadd<R>(acc, cscale<R>(T[(oy[h] + c) * TZ + tz], wy[h][c]));
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        if (pos == k) ring[h][k] = acc;
                }
                ++nxt;
            }
            // x: the ring holds planes need - K .. need - 1, the stencil of ix;
            // plane need - K + b sits at (need + b) % K
            const R *wxp = lay.wx(w) + (ix - ix0) * K;
            R wxv[K];
#pragma unroll
            for (int b = 0; b < K; ++b) wxv[b] = wxp[b];
            const int pos = need & (K - 1);
#pragma unroll
            for (int h = 0; h < VL; ++h) {
                cx<R> acc = czero<R>();
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (pos == k) {
#pragma unroll
                        for (int b = 0; b < K; ++b) acc = cadd<R>(acc, cscale<R>(ring[h][(k + b) & (K - 1)], wxv[b]));
                    }
                v[h] = acc;
            }
        }
        // the tile's values of every field, then the source product
        cx<R> *V = lay.vals(par, w);
#pragma unroll
        for (int h = 0; h < VL; ++h) V[lane + 64 * h] = v[h];
        __syncthreads();
        for (int u = lane + 64 * w; u < NV; u += 64 * NF) {
            const int iy = iy0 + (u >> 5), izu = iz0 + (u & (TZ - 1));
            if (iy < Ny && izu < Nz) {
                // sum_{b + c = NF - 1} v_b v_c, the source term of harmonic NF + 1
                cx<R> f = czero<R>();
#pragma unroll
                for (int b = 0; b < NF; ++b) f = cadd<R>(f, cmul<R>(lay.vals(par, b)[u], lay.vals(par, NF - 1 - b)[u]));
                out[((uint32_t)ix * (uint32_t)Ny + (uint32_t)iy) * (uint32_t)Nz + (uint32_t)izu] = f;
            }
        }
    }
}

#ifndef NVP_HOST_EMULATION
extern __shared__ __align__(16) unsigned char nvp_smem[];

template <typename R, int K, int NF, int PREW, int CXM>
__global__ void __launch_bounds__(NF * 64)
k_source_wf(LdSource<R, K> src, cx<R> *__restrict__ out, int Ny, int cxl) {
    source_tile_wf<R, K, NF, PREW, CXM>(src, out, Ny, cxl, nvp_smem, (int)threadIdx.x, (int)blockIdx.x,
                                        (int)blockIdx.y, (int)blockIdx.z);
}
#endif

}  // namespace nvp
