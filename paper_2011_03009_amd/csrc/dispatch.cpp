// Length dispatch of the pass launchers.
#include "impl_decl.hpp"

namespace nvp {

#define NVP_DISPATCH(call)                         \
    switch (L) {                                   \
        NVP_FOR_EACH_LENGTH(X)                     \
    default: return hipErrorInvalidValue;          \
    }

hipError_t launch_strided_c64(int L, const StridedArgs &a, const void *tw, hipStream_t s) {
#define X(n) case n: return strided_impl<float, float, n>(a, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_strided_c128(int L, const StridedArgs &a, const void *tw, hipStream_t s) {
#define X(n) case n: return strided_impl<double, double, n>(a, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_strided_f64_c64(int L, const StridedArgs &a, const void *tw, hipStream_t s) {
#define X(n) case n: return strided_impl<double, float, n>(a, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_xsrc_c64(int L, const SourceArgs &a, const void *tw, hipStream_t s) {
#define X(n) case n: return xsrc_impl<float, n>(a, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_xsrc_c128(int L, const SourceArgs &a, const void *tw, hipStream_t s) {
#define X(n) case n: return xsrc_impl<double, n>(a, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_zconv_c64(int L, void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw,
                            int quads, hipStream_t s) {
#define X(n) case n: return zconv_impl<float, n>(buf, khat, Mx, My, Nz, tw, quads, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_zconv_c128(int L, void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw,
                             int quads, hipStream_t s) {
#define X(n) case n: return zconv_impl<double, n>(buf, khat, Mx, My, Nz, tw, quads, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_kz(int L, double2 *out, const int64_t H[3], const int64_t N[3], const double2 *ktab,
                     const void *tw, hipStream_t s) {
#define X(n) case n: return kz_impl<n>(out, H, N, ktab, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_strided_multi_c64(int L, const StridedTaskArgs *tasks, int ntasks, int64_t blocks, int sign,
                                    int scaled, const void *tw, hipStream_t s) {
#define X(n) case n: return strided_multi_impl<float, n>(tasks, ntasks, blocks, sign, scaled, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_strided_multi_c128(int L, const StridedTaskArgs *tasks, int ntasks, int64_t blocks, int sign,
                                     int scaled, const void *tw, hipStream_t s) {
#define X(n) case n: return strided_multi_impl<double, n>(tasks, ntasks, blocks, sign, scaled, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_zconv_multi_c64(int L, const ZconvTaskArgs *tasks, int ntasks, int64_t blocks, const void *tw,
                                  hipStream_t s) {
#define X(n) case n: return zconv_multi_impl<float, n>(tasks, ntasks, blocks, tw, s);
    NVP_DISPATCH()
#undef X
}

hipError_t launch_zconv_multi_c128(int L, const ZconvTaskArgs *tasks, int ntasks, int64_t blocks, const void *tw,
                                   hipStream_t s) {
#define X(n) case n: return zconv_multi_impl<double, n>(tasks, ntasks, blocks, tw, s);
    NVP_DISPATCH()
#undef X
}

}  // namespace nvp
