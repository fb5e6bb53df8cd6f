// Declarations of the per-length launcher templates.  Each length's
// instantiations live in their own translation unit (inst.hip compiled with
// -DNVP_L=<length>), so the kernels build in parallel.
#pragma once

#include "launch.hpp"

namespace nvp {

template <typename R, typename Rout, int L> hipError_t strided_impl(const StridedArgs &, const void *, hipStream_t);
template <typename R, int L> hipError_t xsrc_impl(const SourceArgs &, const void *, hipStream_t);
template <typename R, int L>
hipError_t zconv_impl(void *, const void *, int64_t, int64_t, int, const void *, int, hipStream_t);

template <typename R, int L>
hipError_t strided_multi_impl(const StridedTaskArgs *, int, int64_t, int, int, const void *, hipStream_t);
template <typename R, int L>
hipError_t zconv_multi_impl(const ZconvTaskArgs *, int, int64_t, const void *, hipStream_t);

template <int L>
hipError_t kz_impl(double2 *, const int64_t[3], const int64_t[3], const double2 *, const void *, hipStream_t);

}  // namespace nvp
