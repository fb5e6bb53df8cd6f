// Pass kernels of the pruned 3-D circulant convolution.
//
// Array layout: C order [x][y][z], z fastest.  For harmonic grid N = (Nx, Ny, Nz)
// and circulant M = (Mx, My, Mz) the five passes are
//   x fwd : source [Nx][Ny][Nz] (built on the fly)     -> A [Mx][Ny][Nz]
//   y fwd : A                                           -> B [Mx][My][Nz]
//   z     : B, per (kx, ky) pencil: FFT_z, times K^, IFFT_z, in place
//   y inv : B                                           -> A [Mx][Ny][Nz]
//   x inv : A, times C_n / (Mx My Mz)                    -> p_n [Nx][Ny][Nz]
// Only the first N inputs of a forward transform are nonzero and only the
// first N outputs of an inverse transform are kept, so neither the zero half
// of the padded source nor the discarded half of the result touches memory.
#pragma once

#include "fft_core.hpp"
#include "field_dev.hpp"
#include "kz_tasks.hpp"
#include "launch.hpp"

namespace nvp {

// ---------------------------------------------------------------- loaders and storers

// Element m of column (o, col) at p[o*os + m*ms + col].  Pruned: zero for
// m >= n.  Mirrored: the column holds entries 0..L/2 of an even sequence of
// length L, and entry m > L/2 equals entry L - m.
template <typename R, int L> struct LdPlain {
    const cx<R> *p;  // may alias the output: in-place passes
    int64_t os, ms;
    int n;
    int mirror;
    __device__ __forceinline__ cx<R> operator()(int64_t o, int64_t col, int m) const {
        if (mirror) {
            const int mm = m <= L / 2 ? m : L - m;
            return p[o * os + (int64_t)mm * ms + col];
        }
        return m < n ? p[o * os + (int64_t)m * ms + col] : czero<R>();
    }
};

template <typename R, typename Rout> __device__ __forceinline__ cx<Rout> cvt(cx<R> v);
template <> __device__ __forceinline__ float2 cvt<float, float>(float2 v) { return v; }
template <> __device__ __forceinline__ double2 cvt<double, double>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 cvt<double, float>(double2 v) {
    return make_float2((float)v.x, (float)v.y);
}

// Stores element m < n of column (o, col), times a real scale when SC.
template <typename R, typename Rout, bool SC> struct StPlain {
    cx<Rout> *p;
    int64_t os, ms;
    int n;
    R scale;
    __device__ __forceinline__ void operator()(int64_t o, int64_t col, int m, cx<R> v) const {
        if (m < n) p[o * os + (int64_t)m * ms + col] = cvt<R, Rout>(SC ? cscale<R>(v, scale) : v);
    }
};

// ---------------------------------------------------------------- LDS helpers

extern __shared__ __align__(16) unsigned char nvp_smem[];

// LDS slot of a contiguous pencil (see PencilSlot).
template <typename R> __host__ __device__ constexpr int padded(int m) { return pencil_pad<R>(m); }
template <typename R> __host__ __device__ constexpr int slot_len(int L) { return padded<R>(L) + 1; }

// Copies n entries of a twiddle table into LDS (all threads of the workgroup).
template <typename R> __device__ __forceinline__ void stage_table(cx<R> *dst, const cx<R> *src, int n) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
}

// A twiddle table is staged in LDS behind the workgroup's data only when it
// costs no occupancy: as many workgroups fit per CU (160 KiB) with it as without.
template <typename R> constexpr bool tw_fits(size_t data_elems, size_t tw_elems) {
    const size_t d = data_elems * sizeof(cx<R>), w = (data_elems + tw_elems) * sizeof(cx<R>);
    return w <= 163840 && 163840 / w == 163840 / d;
}

// ---------------------------------------------------------------- kernels

// Columns strided by `ms` with T consecutive columns (contiguous in memory)
// per workgroup: lanes run over columns first, so every row access of a wave
// reads T * sizeof(complex) contiguous bytes.  grid = (ceil(inner / T), outer).
// SG: -1 forward, +1 inverse.  MIRROR: the columns hold entries 0..L/2 of even
// sequences; they are read once into LDS and the transform takes its first
// stage from there.
// LDS bytes of a k_strided workgroup's columns: L complex values per column,
// except in the mirror passes (the FP64 kernel spectrum), which stage their
// L/2+1 input entries as complex values and then exchange through one real
// plane (real parts, then imaginary parts), so that a column needs about L
// reals.  (The same split measured slower for the complex64 passes.)
template <typename R, int L, int T, bool MIRROR> constexpr size_t strided_data_bytes() {
    if constexpr (MIRROR) {
        const size_t a = (size_t)T * L * sizeof(R), b = (size_t)T * (L / 2 + 1) * sizeof(cx<R>);
        return a > b ? a : b;
    } else {
        return (size_t)T * L * sizeof(cx<R>);
    }
}

// One workgroup's tile: columns bx T .. bx T + T-1 of outer index o.
template <typename R, int L, int T, int SG, bool MIRROR, class Ld, class St>
__device__ __forceinline__ void strided_tile(Ld ld, St st, const cx<R> *__restrict__ tw, int64_t inner, int64_t bx,
                                             int64_t o) {
    using F = Fft<R, L>;
    constexpr int NT = plan_tw_len(L, false);
    constexpr size_t DATA = strided_data_bytes<R, L, T, MIRROR>();
    constexpr bool TWL = tw_fits<R>(DATA / sizeof(cx<R>), NT);
    cx<R> *lds = reinterpret_cast<cx<R> *>(nvp_smem);
    cx<R> *twl = reinterpret_cast<cx<R> *>(nvp_smem + DATA);
    auto twf = [&](int e) { return TWL ? twl[e] : tw[e]; };
    const int tid = threadIdx.x, c = tid % T, t = tid / T;
    const int64_t col = bx * T + c;
    const bool act = col < inner;
    auto store = [&](int m, cx<R> v) {
        if (act) st(o, col, m, v);
    };
    if constexpr (MIRROR) {
        constexpr int NH = (L / 2 + F::P) / F::P;  // entries 0..L/2 per thread, all loads issued first
        cx<R> h[NH];
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int m = t + i * F::P;
            h[i] = (act && m <= L / 2) ? ld(o, col, m) : czero<R>();
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int m = t + i * F::P;
            if (m <= L / 2) lds[m * T + c] = h[i];
        }
        if constexpr (TWL) stage_table<R>(twl, tw, NT);
        __syncthreads();
        F::template run<SG, true>(t, twf, [&](int m) { return lds[(m <= L / 2 ? m : L - m) * T + c]; }, store,
                                  SplitCols<R, T>{reinterpret_cast<R *>(nvp_smem), c});
    } else {
        // forward passes read columns whose upper half is zero (M >= 2N - 1);
        // inverse passes keep at most the lower half
        constexpr bool ZH = SG < 0, OH = SG > 0;
        cx<R> v[F::E];
        F::template load0<ZH>(v, t, [&](int m) { return act ? ld(o, col, m) : czero<R>(); });
        if constexpr (TWL) {
            stage_table<R>(twl, tw, NT);
            __syncthreads();  // the engine reads a stage's twiddles before its LDS exchange
        }
        F::template compute<SG, ZH, OH>(v, t, twf, store, [&](int m) -> cx<R> & { return lds[m * T + c]; });
    }
}

// Waves per SIMD the FP64 mirror passes are compiled for, where their LDS
// allows more workgroups per CU than their registers otherwise would.
template <typename R, int L, bool MIRROR> constexpr int strided_min_waves() {
    return (sizeof(R) == 8 && MIRROR) ? (L == 512 ? 4 : (L == 768 ? 3 : 1)) : 1;
}

template <typename R, int L, int T, int SG, bool MIRROR, class Ld, class St>
__global__ void __launch_bounds__(T *col_threads<R>(L), (strided_min_waves<R, L, MIRROR>()))
k_strided(Ld ld, St st, const cx<R> *__restrict__ tw, int64_t inner) {
    strided_tile<R, L, T, SG, MIRROR>(ld, st, tw, inner, blockIdx.x, blockIdx.y);
}

// Multi-task launch (batches): the pass of several problems of the same
// transform length in one grid.  Task k owns blocks [first_k, first_{k+1});
// its tile (bx, o) follows from the block's offset in that range.  Each
// task's arguments are read once per workgroup (uniform loads).
template <typename R, int L, int T, int SG, bool SC>
__global__ void __launch_bounds__(T *col_threads<R>(L))
k_strided_multi(const StridedTaskArgs *__restrict__ tasks, int ntasks, const cx<R> *__restrict__ tw) {
    const int64_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < ntasks && tasks[k + 1].first <= b) ++k;
    const StridedTaskArgs a = tasks[k];
    const int64_t local = b - a.first;
    LdPlain<R, L> ld{static_cast<const cx<R> *>(a.in), a.in_os, a.in_ms, a.n_in, 0};
    StPlain<R, R, SC> st{static_cast<cx<R> *>(a.out), a.out_os, a.out_ms, a.n_out, (R)a.scale};
    strided_tile<R, L, T, SG, false>(ld, st, tw, a.inner, local % a.tiles, local / a.tiles);
}

// Forward x pass with the source build fused in front, direct form: each
// thread first writes f_n for its share of the column's Nx voxels into the
// column's LDS slot (a rolled loop, so the interpolation code exists once),
// then the FFT reads its first stage from there.  Column col = iy * Nz + iz.
template <typename R, int L, int T, int K, class St>
__global__ void __launch_bounds__(T *col_threads<R>(L))
k_xsrc(LdSource<R, K> src, St st, const cx<R> *__restrict__ tw, int64_t inner) {
    using F = Fft<R, L>;
    constexpr int NT = plan_tw_len(L, false);
    constexpr bool TWL = tw_fits<R>((size_t)T * L, NT);
    cx<R> *lds = reinterpret_cast<cx<R> *>(nvp_smem);
    cx<R> *twl = lds + T * L;
    if constexpr (TWL) stage_table<R>(twl, tw, NT);
    auto twf = [&](int e) { return TWL ? twl[e] : tw[e]; };
    const int tid = threadIdx.x, c = tid % T, t = tid / T;
    const int64_t col = (int64_t)blockIdx.x * T + c;
    const bool act = col < inner;
    const int iy = act ? (int)(col / src.Nz) : 0, iz = act ? (int)(col % src.Nz) : 0;
    const int Nx = src.Nx;
#pragma unroll 1
    for (int m = t; m < Nx; m += F::P) lds[m * T + c] = act ? src.value(m, iy, iz) : czero<R>();
    __syncthreads();
    F::template run<-1, true, true>(
        t, twf, [&](int m) { return m < Nx ? lds[m * T + c] : czero<R>(); },
        [&](int m, cx<R> v) {
            if (act) st(0, col, m, v);
        },
        [&](int m) -> cx<R> & { return lds[m * T + c]; });
}

// The same pass with the transfer split by axis.  Per chunk of target x
// indices [ix0, ix1): (A) for every field that needs interpolating, the y-z
// interpolation of the source x-rows the chunk touches is staged, per column,
// in the upper part of the column's LDS slot (rows Nx .. L-1, which the
// zero-padded transform never reads); (B) each target voxel then needs only
// K x-taps per field from LDS before the products of the source term are
// written to rows 0 .. Nx-1.  The host picks `chunk` so that the staged rows
// of all fields fit in L - Nx rows.
template <typename R, int L, int T, int K, class St>
__global__ void __launch_bounds__(T *col_threads<R>(L))
k_xsrc_staged(LdSource<R, K> src, St st, const cx<R> *__restrict__ tw, int64_t inner, int chunk) {
    using F = Fft<R, L>;
    constexpr int P = F::P;
    constexpr int NT = plan_tw_len(L, false);
    constexpr bool TWL = tw_fits<R>((size_t)T * L, NT);
    cx<R> *lds = reinterpret_cast<cx<R> *>(nvp_smem);
    const int tid = threadIdx.x, c = tid % T, t = tid / T;
    const int64_t col = (int64_t)blockIdx.x * T + c;
    const bool act = col < inner;
    const int iy = act ? (int)(col / src.Nz) : 0, iz = act ? (int)(col % src.Nz) : 0;
    const int Nx = src.Nx;
    cx<R> *stage = lds + (int64_t)Nx * T;
    cx<R> *twl = lds + T * L;
    if constexpr (TWL) stage_table<R>(twl, tw, NT);
    auto twf = [&](int e) { return TWL ? twl[e] : tw[e]; };
#pragma unroll 1
    for (int ix0 = 0; ix0 < Nx; ix0 += chunk) {
        const int ix1 = ix0 + chunk < Nx ? ix0 + chunk : Nx;
        int lo[NVP_MAX_FIELDS], off[NVP_MAX_FIELDS];
        int rows = 0;
#pragma unroll
        for (int i = 0; i < NVP_MAX_FIELDS; ++i) {
            lo[i] = 0;
            off[i] = rows;
            if (i < src.nf && !src.f[i].identity) {
                const FieldDev<R> &g = src.f[i];
                const int r0 = g.b[0][ix0], r1 = g.b[0][ix1 - 1] + K;
                lo[i] = r0;
                const cx<R> *colbase = g.p + (int64_t)r0 * g.s0 + (int64_t)g.b[1][iy] * g.s1 + g.b[2][iz];
                R wy[K], wz[K];
#pragma unroll
                for (int a = 0; a < K; ++a) {
                    wy[a] = g.w[1][iy * K + a];
                    wz[a] = g.w[2][iz * K + a];
                }
#pragma unroll 4
                for (int r = t; r < r1 - r0; r += P) {
                    cx<R> acc = czero<R>();
                    if (act) {
                        const cx<R> *rp = colbase + (int64_t)r * g.s0;
#pragma unroll
                        for (int b = 0; b < K; ++b) {
                            cx<R> az = czero<R>();
#pragma unroll
                            for (int d = 0; d < K; ++d) az = cadd<R>(az, cscale<R>(rp[b * g.s1 + d], wz[d]));
                            acc = cadd<R>(acc, cscale<R>(az, wy[b]));
                        }
                    }
                    stage[(rows + r) * T + c] = acc;
                }
                rows += r1 - r0;
            }
        }
        __syncthreads();
#pragma unroll 2
        for (int ix = ix0 + t; ix < ix1; ix += P) {
            cx<R> v[NVP_MAX_FIELDS];
#pragma unroll
            for (int i = 0; i < NVP_MAX_FIELDS; ++i) {
                v[i] = czero<R>();
                if (i < src.nf) {
                    const FieldDev<R> &g = src.f[i];
                    if (g.identity) {
                        if (act) v[i] = g.p[ix * g.s0 + (int64_t)iy * g.s1 + iz];
                    } else {
                        const int r = off[i] + g.b[0][ix] - lo[i];
#pragma unroll
                        for (int a = 0; a < K; ++a)
                            v[i] = cadd<R>(v[i], cscale<R>(stage[(r + a) * T + c], g.w[0][ix * K + a]));
                    }
                }
            }
            lds[ix * T + c] = src.products(v);
        }
        __syncthreads();
    }
    F::template run<-1, true, true>(
        t, twf, [&](int m) { return m < Nx ? lds[m * T + c] : czero<R>(); },
        [&](int m, cx<R> v) {
            if (act) st(0, col, m, v);
        },
        [&](int m) -> cx<R> & { return lds[m * T + c]; });
}

// The z pass of the convolution.  A quad = the up-to-four pencils
// (kx, ky), (Mx-kx, ky), (kx, My-ky), (Mx-kx, My-ky) that share one row of the
// kernel spectrum's octant (the embedded kernel is even on every axis, so
// K^(k) = K^(M - k)).  A workgroup takes SLOTS consecutive pencils of the
// quad sequence (pencil 4 q + j is member j of quad q): SLOTS = 4 or 8 keeps
// whole quads together; long transforms, whose pencils do not all fit the
// LDS at once, take 2 or 1.  Each pencil: Nz inputs -> forward FFT of length
// Mz -> times K^ -> inverse FFT -> first Nz outputs written back in place.
// Where a pencil's threads lie in one wavefront the waves run without
// workgroup barriers; twiddles come through the caches from the global table
// (staging them in LDS cost occupancy and was slower).  The inverse runs the
// radix plan in reverse order, so the forward outputs feed it straight from
// registers, where the product with K^ is taken.
template <typename R, int L, int SLOTS>
__device__ __forceinline__ void zconv_block(cx<R> *__restrict__ buf, const cx<R> *__restrict__ khat, int64_t Mx,
                                            int64_t My, int Nz, int64_t Hy, int64_t n_quads,
                                            const cx<R> *__restrict__ tw, int64_t block) {
    constexpr bool WL = wave_local<R>(L);
    using F = Fft<R, L, false, WL>;
    using G = Fft<R, L, true, WL>;
    constexpr int EO = F::EOUT;
    constexpr int SL = slot_len<R>(L);
    cx<R> *lds = reinterpret_cast<cx<R> *>(nvp_smem);
    const int tid = threadIdx.x, t = tid % F::P, slot = tid / F::P;
    // The workgroup's first pencil v0 = block SLOTS lies in quad q0 = v0 / 4,
    // split into (kx, ky) once, with a 32-bit division on workgroup-uniform
    // values (the host keeps the pencil count below 2^31); a slot's own quad
    // is at most two further on and follows with one carry, since Hy >= 9.
    // The mirrored index M - k needs no division either: k = 0 mirrors onto
    // itself.
    const uint32_t hy = (uint32_t)Hy, v0 = (uint32_t)block * (uint32_t)SLOTS, q0 = v0 >> 2;
    const uint32_t vs = v0 + (uint32_t)slot, sq = (vs >> 2) - q0;
    const int j = (int)(vs & 3u);
    const uint32_t kx0 = q0 / hy;
    const bool valid = (int64_t)(q0 + sq) < n_quads;
    uint32_t ukx = kx0, uky = q0 - kx0 * hy + sq;
    if (uky >= hy) uky -= hy, ++ukx;
    const int64_t kx = valid ? ukx : 0, ky = valid ? uky : 0;
    const int64_t px = ((j & 1) && kx) ? Mx - kx : kx;
    const int64_t py = ((j & 2) && ky) ? My - ky : ky;
    const bool act = valid && !(((j & 1) && px == kx) || ((j & 2) && py == ky));
    cx<R> *pen = buf + (px * My + py) * (int64_t)Nz;
    const cx<R> *krow = khat + (kx * Hy + ky) * octant_row(L);
    cx<R> *my = lds + slot * SL;
    const PencilSlot<R> ref{my};
    cx<R> v[F::E];
    // the pencil's upper half is zero (Mz >= 2 Nz - 1) and only its lower half
    // is kept.  Loads need no guard but m < Nz: a pencil past the last maps to
    // pencil (0, 0) and kernel row (0, 0), which exist, and an inactive
    // pencil's results are never stored.  With an even first radix the first
    // stage reads only elements below L/2, so for Nz = L/2 none is guarded.
    constexpr bool EVEN0 = 2 * F::K0 == plan_for(L).r[0];
    if (EVEN0 && Nz == L / 2)
        F::template load0<true>(v, t, [&](int m) { return pen[m]; });
    else
        F::template load0<true>(v, t, [&](int m) { return m < Nz ? pen[m] : czero<R>(); });
    // the spectrum values this thread multiplies by, loaded before the forward
    // transform so that their latency overlaps it (where registers allow)
    constexpr bool KPRE = sizeof(R) == 4 || EO <= 32;
    auto kval = [&](int i) {
        const int k = F::out_index(t, i);
        return F::out_valid(t, i) ? krow[k <= L / 2 ? k : L - k] : czero<R>();
    };
    cx<R> kv[KPRE ? EO : 1];
    if constexpr (KPRE) {
#pragma unroll
        for (int i = 0; i < EO; ++i) kv[i] = kval(i);
    }
    auto twf = [&](int e) { return tw[e]; };
    F::template compute_keep<-1, true>(v, t, twf, ref);
#pragma unroll
    for (int i = 0; i < EO; ++i) v[i] = cmul<R>(v[i], KPRE ? kv[i] : kval(i));
    G::template compute<1, false, true>(v, t, twf,
                           [&](int m, cx<R> x) {
                               if (act && m < Nz) pen[m] = x;
                           },
                           ref);
}

template <typename R, int L, int SLOTS>
__global__ void __launch_bounds__(SLOTS *col_threads<R>(L))
k_zconv(cx<R> *__restrict__ buf, const cx<R> *__restrict__ khat, int64_t Mx, int64_t My, int Nz, int64_t Hy,
        int64_t n_quads, const cx<R> *__restrict__ tw) {
    zconv_block<R, L, SLOTS>(buf, khat, Mx, My, Nz, Hy, n_quads, tw, blockIdx.x);
}

// Multi-task z pass (batches), laid out like k_strided_multi.
template <typename R, int L, int SLOTS>
__global__ void __launch_bounds__(SLOTS *col_threads<R>(L))
k_zconv_multi(const ZconvTaskArgs *__restrict__ tasks, int ntasks, const cx<R> *__restrict__ tw) {
    const int64_t b = blockIdx.x;
    int k = 0;
    while (k + 1 < ntasks && tasks[k + 1].first <= b) ++k;
    const ZconvTaskArgs a = tasks[k];
    zconv_block<R, L, SLOTS>(static_cast<cx<R> *>(a.buf), static_cast<const cx<R> *>(a.khat), a.Mx, a.My, a.Nz,
                             a.Hy, a.n_quads, tw, b - a.first);
}

// First pass of the kernel spectrum, fused with the kernel's tabulation: one
// octant row (i, j) per pencil.  The row's Hz = L/2+1 values of K at offsets
// (i, j, k) -- ktab[i^2 + j^2 + k^2] (h^3 G_k(|d| h) of equation "quad", the
// self value at the origin), zero for k >= Nz or beyond the grid in x or y (the
// embedding is exact for M >= 2N - 1) -- are gathered into LDS in FP64, then
// the FFT of the even extension to length L is written back as the row's first
// Hz outputs.
template <int L, int PW, bool TWL>
__global__ void __launch_bounds__(PW *kz_threads(L))
k_kz(double2 *__restrict__ out, int64_t Hx, int64_t Hy, int64_t Nx, int64_t Ny, int64_t Nz,
     const double2 *__restrict__ ktab, const double2 *__restrict__ tw, int64_t ntasks) {
    constexpr bool WL = wave_local_p(kz_threads(L));
    using F = Fft<double, L, false, WL, kz_threads(L)>;
    constexpr int HZ = L / 2 + 1;
    constexpr int SL = slot_len<double>(L);
    constexpr int NT = plan_tw_len(L, false);
    cx<double> *lds = reinterpret_cast<cx<double> *>(nvp_smem);
    const int tid = threadIdx.x, t = tid % F::P, c = tid / F::P;
    // the slot's task: one octant row, or the rows (i, j) and (j, i) of the
    // square of nonzero rows, which hold the same values
    const int64_t q = (int64_t)blockIdx.x * PW + c;
    const bool act = q < ntasks;
    const KzTask tk = kz_task(act ? q : 0, Hx, Hy, Nx < Ny ? Nx : Ny);
    const int64_t i = tk.i, jj = tk.j;
    cx<double> *my = lds + c * SL;
    cx<double> *twl = lds + PW * SL;  // the twiddle table, staged when it fits (TWL)
    if constexpr (TWL) {
        stage_table<double>(twl, tw, NT);
        __syncthreads();
    }
    auto twf = [&](int e) { return TWL ? twl[e] : tw[e]; };
    // all of this thread's gathers in flight before the first store
    constexpr int NK = (HZ + F::P - 1) / F::P;
    double2 g[NK];
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        const int k = t + q * F::P;
        g[q] = (act && i < Nx && jj < Ny && k < Nz && k < HZ) ? ktab[i * i + jj * jj + (int64_t)k * k]
                                                             : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        const int k = t + q * F::P;
        if (k < HZ) my[padded<double>(k)] = g[q];
    }
    if constexpr (WL) wave_sync();
    else __syncthreads();
    F::template run<-1, true>(
        t, twf, [&](int m) { return my[padded<double>(m <= L / 2 ? m : L - m)]; },
        [&](int m, cx<double> v) {
            if (act && m < HZ) {
                out[tk.r0 * octant_row(L) + m] = v;
                if (tk.r1 != tk.r0) out[tk.r1 * octant_row(L) + m] = v;
            }
        },
        PencilSlot<double>{my});
}

}  // namespace nvp
