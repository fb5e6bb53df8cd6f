// Stand-in for the HIP runtime header when the FFT engine (fft_core.hpp) or the source kernel (source.hpp) is
// compiled for the host by the harnesses in tests/fft_host: the device
// qualifiers vanish, the vector types are plain structs, and __syncthreads is
// the harness's barrier over the host threads that play one column's lanes.
#pragma once
#include <stdint.h>

#define __host__
#define __device__
#define __forceinline__ inline
#define __global__
#define __launch_bounds__(x)

struct float2 {
    float x, y;
};
struct double2 {
    double x, y;
};

void __syncthreads();

template <typename T> inline T min(T a, T b) { return b < a ? b : a; }
template <typename T> inline T max(T a, T b) { return a < b ? b : a; }
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
