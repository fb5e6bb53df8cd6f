// Launcher templates shared by the per-precision translation units.
#pragma once

#include "kernels.hpp"

namespace nvp {

// Columns per workgroup of the strided kernels: at least 128 contiguous bytes
// per row access, about 256 threads per workgroup.
template <typename R> constexpr int strided_cols(int L) {
    const int lo = sizeof(R) == 4 ? 16 : 8, hi = sizeof(R) == 4 ? 64 : 32;
    const int t = 256 / plan_threads(L);
    return t < lo ? lo : (t > hi ? hi : t);
}

// Pencils per workgroup of the contiguous kernel: about 256 threads, LDS <= 128 KiB.
template <typename R> constexpr int contig_pencils(int L) {
    const int by_threads = 256 / plan_threads(L) > 0 ? 256 / plan_threads(L) : 1;
    const int by_lds = (int)((131072 - L * (int)sizeof(cx<R>)) / (slot_len(L) * (int)sizeof(cx<R>)));
    const int p = by_threads < by_lds ? by_threads : by_lds;
    return p > 0 ? p : 1;
}

template <class K> inline hipError_t allow_lds(K kern, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// A column count is usable if the workgroup stays within 1024 threads and 160 KiB of LDS.
template <typename R, int L, int T> constexpr bool cols_ok() {
    return T * plan_threads(L) <= 1024 && (size_t)T * L * sizeof(cx<R>) <= 163840;
}

template <typename R, typename Rout, int L, int T>
hipError_t strided_t(const StridedArgs &a, const void *tw, hipStream_t s) {
    using Ld = LdPlain<R, L>;
    using St = StPlain<R, Rout>;
    Ld ld{static_cast<const cx<R> *>(a.in), a.in_os, a.in_ms, a.n_in, a.mirror};
    St st{static_cast<cx<Rout> *>(a.out), a.out_os, a.out_ms, a.n_out, (R)a.scale};
    const size_t lds = ((size_t)T * L + (tw_fits<R, L>((size_t)T * L) ? L : 0)) * sizeof(cx<R>);
    dim3 grid((unsigned)((a.inner + T - 1) / T), (unsigned)a.outer);
    if constexpr (sizeof(R) == 8) {
        if (a.mirror) {
            auto kern = k_strided<R, L, T, true, Ld, St>;
            static const hipError_t attr = allow_lds(kern, lds);
            if (attr != hipSuccess) return attr;
            hipLaunchKernelGGL(kern, grid, dim3(T * plan_threads(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                               (R)a.sign, a.inner);
            return hipGetLastError();
        }
    } else if (a.mirror) {
        return hipErrorInvalidValue;
    }
    auto kern = k_strided<R, L, T, false, Ld, St>;
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(kern, grid, dim3(T * plan_threads(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                       (R)a.sign, a.inner);
    return hipGetLastError();
}

// Column-count variants (complex64 passes): a.cols = 8, 16 or 32, else the default.
template <typename R, typename Rout, int L>
hipError_t strided_impl(const StridedArgs &a, const void *tw, hipStream_t s) {
    constexpr int T0 = strided_cols<R>(L);
    if constexpr (sizeof(R) == 4) {
        if (a.cols == 8 && T0 != 8) {
            if constexpr (cols_ok<R, L, 8>()) return strided_t<R, Rout, L, 8>(a, tw, s);
        }
        if (a.cols == 16 && T0 != 16) {
            if constexpr (cols_ok<R, L, 16>()) return strided_t<R, Rout, L, 16>(a, tw, s);
        }
        if (a.cols == 32 && T0 != 32) {
            if constexpr (cols_ok<R, L, 32>()) return strided_t<R, Rout, L, 32>(a, tw, s);
        }
    }
    return strided_t<R, Rout, L, T0>(a, tw, s);
}

template <typename R, int L, int K, int T> hipError_t xsrc_impl_k(const SourceArgs &a, const void *tw, hipStream_t s) {
    using Ld = LdSource<R, K>;
    using St = StPlain<R, R>;
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
    const size_t lds = ((size_t)T * L + (tw_fits<R, L>((size_t)T * L) ? L : 0)) * sizeof(cx<R>);
    dim3 grid((unsigned)((a.inner + T - 1) / T), 1);
    if (a.chunk > 0) {
        auto kern = k_xsrc_staged<R, L, T, K, St>;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(kern, grid, dim3(T * plan_threads(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                           a.inner, a.chunk);
    } else {
        auto kern = k_xsrc<R, L, T, K, St>;
        static const hipError_t attr = allow_lds(kern, lds);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(kern, grid, dim3(T * plan_threads(L)), lds, s, ld, st, static_cast<const cx<R> *>(tw),
                           a.inner);
    }
    return hipGetLastError();
}

template <typename R, int L, int T> hipError_t xsrc_impl_t(const SourceArgs &a, const void *tw, hipStream_t s) {
    if (a.order == 1) return xsrc_impl_k<R, L, 2, T>(a, tw, s);
    if (a.order == 3) return xsrc_impl_k<R, L, 4, T>(a, tw, s);
    return hipErrorInvalidValue;
}

template <typename R, int L> hipError_t xsrc_impl(const SourceArgs &a, const void *tw, hipStream_t s) {
    constexpr int T0 = strided_cols<R>(L);
    if constexpr (sizeof(R) == 4) {
        if (a.cols == 8 && T0 != 8) {
            if constexpr (cols_ok<R, L, 8>()) return xsrc_impl_t<R, L, 8>(a, tw, s);
        }
        if (a.cols == 32 && T0 != 32) {
            if constexpr (cols_ok<R, L, 32>()) return xsrc_impl_t<R, L, 32>(a, tw, s);
        }
    }
    return xsrc_impl_t<R, L, T0>(a, tw, s);
}

template <typename R, int L, int QW>
hipError_t zconv_qw(void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw, hipStream_t s) {
    auto kern = k_zconv<R, L, QW>;
    const size_t lds = ((size_t)4 * QW * slot_len(L) + L) * sizeof(cx<R>);
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    const int64_t Hx = Mx / 2 + 1, Hy = My / 2 + 1, nq = Hx * Hy;
    hipLaunchKernelGGL(kern, dim3((unsigned)((nq + QW - 1) / QW)), dim3(4 * QW * plan_threads(L)), lds, s,
                       static_cast<cx<R> *>(buf), static_cast<const cx<R> *>(khat), Mx, My, Nz, Hy, nq,
                       static_cast<const cx<R> *>(tw));
    return hipGetLastError();
}

template <typename R, int L>
hipError_t zconv_impl(void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw, hipStream_t s) {
    // quads per workgroup: up to 256 threads and 80 KiB of LDS
    constexpr int QW = (4 * plan_threads(L) <= 128 && (8 * slot_len(L) + L) * (int)sizeof(cx<R>) <= 81920) ? 2 : 1;
    if (zconv_quads_override() == 1) return zconv_qw<R, L, 1>(buf, khat, Mx, My, Nz, tw, s);
    return zconv_qw<R, L, QW>(buf, khat, Mx, My, Nz, tw, s);
}

template <int L>
hipError_t kz_impl(double2 *out, const int64_t H[3], const int64_t N[3], double h, double kr, double ki,
                   double self_re, double self_im, const void *tw, hipStream_t s) {
    constexpr int PW = contig_pencils<double>(L);
    auto kern = k_kz<L, PW>;
    const size_t lds = ((size_t)PW * slot_len(L) + L) * sizeof(double2);
    static const hipError_t attr = allow_lds(kern, lds);
    if (attr != hipSuccess) return attr;
    const int64_t rows = H[0] * H[1];
    hipLaunchKernelGGL(kern, dim3((unsigned)((rows + PW - 1) / PW)), dim3(PW * plan_threads(L)), lds, s, out, H[0],
                       H[1], N[0], N[1], N[2], h, kr, ki, make_double2(self_re, self_im),
                       static_cast<const double2 *>(tw));
    return hipGetLastError();
}

}  // namespace nvp
