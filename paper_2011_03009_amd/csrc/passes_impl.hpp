// Launcher templates shared by the per-length translation units.
#pragma once

#include "kernels.hpp"

namespace nvp {

// Columns per workgroup of the strided kernels: at least 128 contiguous bytes
// per row access, about 256 threads per workgroup.
template <typename R> constexpr int strided_cols(int L) {
    const int lo = sizeof(R) == 4 ? 16 : 8, hi = sizeof(R) == 4 ? 64 : 32;
    const int t = 256 / col_threads<R>(L);
    int c = t < lo ? lo : (t > hi ? hi : t);
    // the workgroup's columns must fit the 160 KiB of LDS and 1024 threads
    while (c > 1 && ((size_t)c * L * sizeof(cx<R>) > 163840 || c * col_threads<R>(L) > 1024)) c /= 2;
    return c;
}

// Whether the contiguous FP64 kernel stages its twiddle table in LDS: when
// the table and one pencil fit 128 KiB, up to 1024 points.  (Beyond, the
// staged table leaves room for only one workgroup of four rows per CU.)
template <typename R> constexpr bool contig_tw_lds(int L) {
    return L <= 1024 && (size_t)(twiddle_table_len(L) + slot_len<R>(L)) * sizeof(cx<R>) <= 131072;
}

// Pencils per workgroup of the contiguous FP64 kernel: about 256 threads,
// LDS <= 128 KiB (with the staged twiddles), and whole wavefronts (a multiple
// of 64 / P pencils where a pencil is wave-local).
template <typename R> constexpr int contig_pencils(int L) {
    const int P = kz_threads(L);
    const int by_threads = 256 / P > 0 ? 256 / P : 1;
    const int tw = contig_tw_lds<R>(L) ? twiddle_table_len(L) * (int)sizeof(cx<R>) : 0;
    const int by_lds = (int)((131072 - tw) / (slot_len<R>(L) * (int)sizeof(cx<R>)));
    int p = by_threads < by_lds ? by_threads : by_lds;
    const int unit = wave_local_p(P) ? 64 / P : 1;
    p = (p / unit) * unit;
    return p > 0 ? p : unit;
}

template <class K> inline hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <typename R, int L, int T, bool MIRROR> constexpr size_t strided_lds() {
    constexpr size_t data = strided_data_bytes<R, L, T, MIRROR>();
    return data + (tw_fits<R>(data / sizeof(cx<R>), plan_tw_len(L, false)) ? plan_tw_len(L, false) : 0) *
                      sizeof(cx<R>);
}

// The fused source passes keep complex columns of L entries in LDS.
template <typename R, int L, int T> constexpr size_t xsrc_lds() {
    return ((size_t)T * L + (tw_fits<R>((size_t)T * L, plan_tw_len(L, false)) ? plan_tw_len(L, false) : 0)) *
           sizeof(cx<R>);
}

template <typename R, typename Rout, int L, int SG, bool SC, bool MIRROR, int T = strided_cols<R>(L)>
hipError_t strided_v(const StridedArgs &a, const void *tw, hipStream_t s) {
    using Ld = LdPlain<R, L>;
    using St = StPlain<R, Rout, SC>;
    Ld ld{static_cast<const cx<R> *>(a.in), a.in_os, a.in_ms, a.n_in, a.mirror};
    St st{static_cast<cx<Rout> *>(a.out), a.out_os, a.out_ms, a.n_out, (R)a.scale};
    auto kern = k_strided<R, L, T, SG, MIRROR, Ld, St>;
    constexpr size_t lds = strided_lds<R, L, T, MIRROR>();
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    dim3 grid((unsigned)((a.inner + T - 1) / T), (unsigned)a.outer);
    hipLaunchKernelGGL(kern, grid, dim3(T * col_threads<R>(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                       a.inner);
    return hipGetLastError();
}

// Half the default column count: the tile-width alternative of the autotuner.
template <typename R> constexpr int strided_cols_half(int L) {
    const int t = strided_cols<R>(L) / 2;
    return t < 4 ? 4 : t;
}

template <typename R, typename Rout, int L, int SG, bool SC>
hipError_t strided_tiles(const StridedArgs &a, const void *tw, hipStream_t s) {
    if (a.tile == 1) return strided_v<R, Rout, L, SG, SC, false, strided_cols_half<R>(L)>(a, tw, s);
    return strided_v<R, Rout, L, SG, SC, false>(a, tw, s);
}

// Variants in use: forward, inverse, inverse with the epilogue scale (each at
// the default or half tile width), and (FP64 only) forward on mirrored even
// sequences.
template <typename R, typename Rout, int L>
hipError_t strided_impl(const StridedArgs &a, const void *tw, hipStream_t s) {
    if (a.mirror) {
        if constexpr (sizeof(R) == 8) {
            if (a.sign < 0 && a.scale == 1.0) return strided_v<R, Rout, L, -1, false, true>(a, tw, s);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (sizeof(R) == sizeof(Rout)) {
        if (a.sign < 0 && a.scale == 1.0) return strided_tiles<R, Rout, L, -1, false>(a, tw, s);
        if (a.sign > 0 && a.scale == 1.0) return strided_tiles<R, Rout, L, 1, false>(a, tw, s);
        if (a.sign > 0) return strided_tiles<R, Rout, L, 1, true>(a, tw, s);
    }
    return hipErrorInvalidValue;
}

template <typename R, int L, int K> hipError_t xsrc_impl_k(const SourceArgs &a, const void *tw, hipStream_t s) {
    constexpr int T = strided_cols<R>(L);
    using Ld = LdSource<R, K>;
    using St = StPlain<R, R, false>;
    Ld ld;
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
    St st{static_cast<cx<R> *>(a.out), 0, a.out_ms, L, R(1)};
    constexpr size_t lds = xsrc_lds<R, L, T>();
    dim3 grid((unsigned)((a.inner + T - 1) / T), 1);
    if (a.chunk > 0) {
        auto kern = k_xsrc_staged<R, L, T, K, St>;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(kern, grid, dim3(T * col_threads<R>(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                           a.inner, a.chunk);
    } else {
        auto kern = k_xsrc<R, L, T, K, St>;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(kern, grid, dim3(T * col_threads<R>(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                           a.inner);
    }
    return hipGetLastError();
}

template <typename R, int L> hipError_t xsrc_impl(const SourceArgs &a, const void *tw, hipStream_t s) {
    if (a.order == 1) return xsrc_impl_k<R, L, 2>(a, tw, s);
    if (a.order == 3) return xsrc_impl_k<R, L, 4>(a, tw, s);
    return hipErrorInvalidValue;
}

template <typename R, int L, int SLOTS>
hipError_t zconv_slots(void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw, hipStream_t s) {
    auto kern = k_zconv<R, L, SLOTS>;
    constexpr size_t lds = (size_t)SLOTS * slot_len<R>(L) * sizeof(cx<R>);
    static_assert(lds <= 163840 && SLOTS * col_threads<R>(L) <= 1024, "z-pass workgroup too large");
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    const int64_t Hx = Mx / 2 + 1, Hy = My / 2 + 1, nq = Hx * Hy;
    if (4 * nq > 0x7fffffff - SLOTS) return hipErrorInvalidValue;  // pencil indices are 32-bit in the kernel
    hipLaunchKernelGGL(kern, dim3((unsigned)((4 * nq + SLOTS - 1) / SLOTS)), dim3(SLOTS * col_threads<R>(L)), lds, s,
                       static_cast<cx<R> *>(buf), static_cast<const cx<R> *>(khat), Mx, My, Nz, Hy, nq,
                       static_cast<const cx<R> *>(tw));
    return hipGetLastError();
}

// Pencils per z-pass workgroup that fit: `slots` pencils of slot_len entries
// of esz bytes within `lds_cap` bytes and `thr_cap` threads.
constexpr bool zconv_fits(int L, size_t esz, int slots, size_t lds_cap, int thr_cap) {
    const size_t slot = (size_t)(esz == sizeof(float2) ? slot_len<float>(L) : slot_len<double>(L)) * esz;
    const int P = esz == sizeof(float2) ? col_threads<float>(L) : col_threads<double>(L);
    return (size_t)slots * slot <= lds_cap && slots * P <= thr_cap;
}

// Pencils per z-pass workgroup by default: two quads (8) when that keeps the
// workgroup within 128 threads and 80 KiB of LDS, else one quad (4);
// transforms too long for a quad in 160 KiB take 2 or 1.
constexpr int zconv_slots_for(int L, size_t esz) {
    return 4 * (esz == sizeof(float2) ? col_threads<float>(L) : col_threads<double>(L)) <= 128 &&
                   zconv_fits(L, esz, 8, 81920, 1024)
               ? 8
         : zconv_fits(L, esz, 4, 163840, 1024) ? 4
         : zconv_fits(L, esz, 2, 163840, 1024) ? 2 : 1;
}
template <typename R, int L> constexpr int zconv_default_slots() { return zconv_slots_for(L, sizeof(cx<R>)); }

// quads: pencil quads per workgroup, 0 for the default, or 1 / 2 forced
// (where a whole quad fits; otherwise the default).
template <typename R, int L>
hipError_t zconv_impl(void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw, int quads,
                      hipStream_t s) {
    constexpr int SD = zconv_default_slots<R, L>();
    if constexpr (SD >= 4) {
        if (quads == 1 || zconv_quads_override() == 1) return zconv_slots<R, L, 4>(buf, khat, Mx, My, Nz, tw, s);
    }
    return zconv_slots<R, L, SD>(buf, khat, Mx, My, Nz, tw, s);
}

template <int L>
hipError_t kz_impl(double2 *out, const int64_t H[3], const int64_t N[3], const double2 *ktab, const void *tw,
                   hipStream_t s) {
    constexpr int PW = contig_pencils<double>(L);
    constexpr bool TWL = contig_tw_lds<double>(L);
    auto kern = k_kz<L, PW, TWL>;
    constexpr size_t lds = ((size_t)PW * slot_len<double>(L) + (TWL ? plan_tw_len(L, false) : 0)) * sizeof(double2);
    static_assert(lds <= 163840 && PW * kz_threads(L) <= 1024, "kernel-spectrum workgroup too large");
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    // one task per octant row, except the mirror pairs (i, j), (j, i) of the nonzero square
    const int64_t ntasks = kz_task_count(H[0], H[1], N[0] < N[1] ? N[0] : N[1]);
    if (ntasks > 0x7fffffff - PW || N[0] > H[0] || N[1] > H[1]) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)((ntasks + PW - 1) / PW)), dim3(PW * kz_threads(L)), lds, s, out, H[0],
                       H[1], N[0], N[1], N[2], ktab, static_cast<const double2 *>(tw), ntasks);
    return hipGetLastError();
}

template <typename R, int L, int SG, bool SC>
hipError_t strided_multi_v(const StridedTaskArgs *tasks, int ntasks, int64_t blocks, const void *tw, hipStream_t s) {
    constexpr int T = strided_cols<R>(L);
    auto kern = k_strided_multi<R, L, T, SG, SC>;
    constexpr size_t lds = strided_lds<R, L, T, false>();
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(T * col_threads<R>(L)), lds, s, tasks, ntasks,
                       static_cast<const cx<R> *>(tw));
    return hipGetLastError();
}

template <typename R, int L>
hipError_t strided_multi_impl(const StridedTaskArgs *tasks, int ntasks, int64_t blocks, int sign, int scaled,
                              const void *tw, hipStream_t s) {
    if (ntasks < 1 || blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (sign < 0) return strided_multi_v<R, L, -1, false>(tasks, ntasks, blocks, tw, s);
    if (!scaled) return strided_multi_v<R, L, 1, false>(tasks, ntasks, blocks, tw, s);
    return strided_multi_v<R, L, 1, true>(tasks, ntasks, blocks, tw, s);
}

template <typename R, int L>
hipError_t zconv_multi_impl(const ZconvTaskArgs *tasks, int ntasks, int64_t blocks, const void *tw, hipStream_t s) {
    if (ntasks < 1 || blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
    constexpr int SLOTS = zconv_default_slots<R, L>();
    auto kern = k_zconv_multi<R, L, SLOTS>;
    constexpr size_t lds = (size_t)SLOTS * slot_len<R>(L) * sizeof(cx<R>);
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(SLOTS * col_threads<R>(L)), lds, s, tasks, ntasks,
                       static_cast<const cx<R> *>(tw));
    return hipGetLastError();
}

}  // namespace nvp
