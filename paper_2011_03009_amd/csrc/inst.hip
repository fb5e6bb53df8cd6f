// Instantiates every pass kernel for one transform length, NVP_L.
#include "passes_impl.hpp"

#ifndef NVP_L
#error "compile with -DNVP_L=<transform length>"
#endif

namespace nvp {

template hipError_t strided_impl<float, float, NVP_L>(const StridedArgs &, const void *, hipStream_t);
template hipError_t strided_impl<double, double, NVP_L>(const StridedArgs &, const void *, hipStream_t);
template hipError_t strided_impl<double, float, NVP_L>(const StridedArgs &, const void *, hipStream_t);
template hipError_t xsrc_impl<float, NVP_L>(const SourceArgs &, const void *, hipStream_t);
template hipError_t xsrc_impl<double, NVP_L>(const SourceArgs &, const void *, hipStream_t);
template hipError_t zconv_impl<float, NVP_L>(void *, const void *, int64_t, int64_t, int, const void *, int,
                                             hipStream_t);
template hipError_t zconv_impl<double, NVP_L>(void *, const void *, int64_t, int64_t, int, const void *, int,
                                              hipStream_t);

template hipError_t strided_multi_impl<float, NVP_L>(const StridedTaskArgs *, int, int64_t, int, int, const void *,
                                                    hipStream_t);
template hipError_t strided_multi_impl<double, NVP_L>(const StridedTaskArgs *, int, int64_t, int, int, const void *,
                                                     hipStream_t);
template hipError_t zconv_multi_impl<float, NVP_L>(const ZconvTaskArgs *, int, int64_t, const void *, hipStream_t);
template hipError_t zconv_multi_impl<double, NVP_L>(const ZconvTaskArgs *, int, int64_t, const void *, hipStream_t);

template hipError_t kz_impl<NVP_L>(double2 *, const int64_t[3], const int64_t[3], const double2 *, const void *,
                                   hipStream_t);

}  // namespace nvp
