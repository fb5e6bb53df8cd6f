// Truncation-box reductions of a source term (qbox.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define NVP_QBOX_MAX 32
#define NVP_BOXSUM_BLOCKS 512

namespace nvp {

// frac_dev[count] = 10^(2 Q0); work: 1025 doubles; box_dev: count * 6 ints.
hipError_t qbox_launch(const void *f, bool dbl, const int64_t n[3], int count, const double *frac_dev, double *work,
                       int *box_dev, hipStream_t s);
// Potential at voxel t restricted to each of count boxes (box_dev: count * 6
// ints lo[3], hi[3], each box inside the grid; an empty box sums to 0);
// (s_re, s_im): the self-voxel kernel value; (f_re, f_im): added to the
// kernel at the six face neighbours (zero for the paper's rule); work:
// NVP_BOXSUM_BLOCKS * count double2; out_dev: count double2.
hipError_t boxsum_launch(const void *f, bool dbl, const int64_t n[3], const int t[3], double h, double kr, double ki,
                         double s_re, double s_im, double f_re, double f_im, const int *box_dev, int count,
                         double2 *work, double2 *out_dev, hipStream_t s);

}  // namespace nvp
