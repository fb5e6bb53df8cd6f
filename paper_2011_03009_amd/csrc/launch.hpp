// Host-side launchers of the pass kernels (defined in the *.hip files).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

// Transform lengths with a compiled radix plan.
#define NVP_FOR_EACH_LENGTH(X) \
    X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(144) X(160) X(192) X(224) X(256) X(288) X(320) X(336) \
    X(360) X(384) X(432) X(448) X(480) X(512) X(576) X(640) X(720) X(768) X(864) X(896) X(960) X(1024) X(1152) X(1280) \
    X(1344) X(1440) X(1536) X(1728) X(1792) X(1920) X(2048) X(2304) X(2560) X(2880) X(3072) X(3456) X(3840) \
    X(4096) X(4608) X(5120) X(5760) X(6144) X(6912) X(7680) X(8192)

namespace nvp {

bool length_supported(int L);
// Tuning switch read once from the environment (NVP_ZCONV_QUADS): 1 forces one
// pencil quad per z-pass workgroup; anything else keeps the default.
int zconv_quads_override();

// Generic strided pass: element m of column (o, col) is read at
// in[o*in_os + m*in_ms + col] and written to out[o*out_os + m*out_ms + col],
// col in [0, inner), o in [0, outer).  Inputs: the first n_in (zero beyond),
// or, with mirror, entries 0..L/2 of an even sequence.  Outputs: the first
// n_out, times `scale`.  sign = -1 forward, +1 inverse.
struct StridedArgs {
    const void *in;
    int64_t in_os, in_ms;
    int n_in;
    int mirror;
    void *out;
    int64_t out_os, out_ms;
    int n_out;
    double scale;
    int64_t inner, outer;
    int sign;
    int tile;  // 0: default columns per workgroup, 1: half as many (not for mirror or mixed precision)
};

// One problem's strided pass in a multi-task launch (batches): the
// StridedArgs of that pass, its column tiles per outer index and its first
// block in the grid (tasks sorted by first; the launch has sum tiles * outer
// blocks).
struct StridedTaskArgs {
    const void *in;
    int64_t in_os, in_ms;
    int n_in;
    void *out;
    int64_t out_os, out_ms;
    int n_out;
    double scale;
    int64_t inner, tiles, first;
};

// One problem's z pass in a multi-task launch.
struct ZconvTaskArgs {
    void *buf;
    const void *khat;
    int64_t Mx, My, Hy, n_quads, first;
    int Nz;
};

// Field of the fused source build (see LdSource).
struct FieldArgs {
    const void *p;
    int64_t s0, s1;
    const int *b[3];
    const void *w[3];  // weights in the working precision
    int identity;
};

struct SourceArgs {
    FieldArgs f[NVP_MAX_FIELDS];
    int nf;
    int order;  // 1 or 3
    int Nx, Nz;
    void *out;  // A [Mx][Ny][Nz]
    int64_t out_ms;  // Ny * Nz
    int64_t inner;   // Ny * Nz
    int chunk;       // > 0: staged separable transfer with this x-chunk; 0: direct gathers
};

hipError_t launch_strided_c64(int L, const StridedArgs &a, const void *tw, hipStream_t s);
hipError_t launch_strided_c128(int L, const StridedArgs &a, const void *tw, hipStream_t s);
// FP64 in, complex64 out (the downcast of the kernel spectrum).
hipError_t launch_strided_f64_c64(int L, const StridedArgs &a, const void *tw, hipStream_t s);

hipError_t launch_xsrc_c64(int L, const SourceArgs &a, const void *tw, hipStream_t s);
hipError_t launch_xsrc_c128(int L, const SourceArgs &a, const void *tw, hipStream_t s);

// Transfer + source build (k_source): f_n written to `out` [Nx][Ny][Nz];
// workgroups of SRC_TY x SRC_TZ threads, each thread owning source_rows target
// rows (y) of a tile and loading up to source_pre entries of a source plane's
// block, walking cx <= SRC_CXM x planes.
#define NVP_SRC_TY 8
#define NVP_SRC_TZ 32
#define NVP_SRC_CXM 64
#ifndef NVP_SRC_RY32
#define NVP_SRC_RY32 1
#endif
// Target rows per thread and block entries per thread, for reals of rsize bytes.
constexpr int source_rows(size_t rsize) { return rsize == 4 ? NVP_SRC_RY32 : 1; }
constexpr int source_pre(size_t rsize) { return source_rows(rsize) == 2 ? 3 : 2; }
// 1: the source kernel with one wavefront per field (k_source_wf): tiles of
// 8 x 32 columns, blocks of up to 64 NVP_SRC_PREW entries and 16 rows.
#ifndef NVP_SRC_WF
#define NVP_SRC_WF 1
#endif
#define NVP_SRC_PREW 7
// Whether the source kernel of reals of rsize bytes is k_source_wf (complex64).
constexpr bool source_wf(size_t rsize) { return NVP_SRC_WF && rsize == 4; }
// LDS bytes of a launch for nf fields, K-point stencils and reals of rsize
// bytes (4 or 8): the kernel's fixed layout.
constexpr size_t source_lds_bytes(int nf, int K, size_t rsize) {
    if (source_wf(rsize))
        return (size_t)nf * (((size_t)NVP_SRC_PREW * 64 + 16 * 32 + 2 * 256) * 2 * rsize +
                             (size_t)NVP_SRC_CXM * K * rsize + (size_t)NVP_SRC_CXM * sizeof(int));
    const size_t nt = (size_t)NVP_SRC_TY * NVP_SRC_TZ, ry = (size_t)source_rows(rsize);
    return (size_t)nf * (((size_t)source_pre(rsize) * nt + 2 * ry * nt) * 2 * rsize +
                         ((size_t)(NVP_SRC_TZ + ry * NVP_SRC_TY) * K + (size_t)NVP_SRC_CXM * K) * rsize +
                         (size_t)NVP_SRC_CXM * sizeof(int));
}
hipError_t launch_source_c64(const SourceArgs &a, void *out, int Ny, int cx, hipStream_t s);
hipError_t launch_source_c128(const SourceArgs &a, void *out, int Ny, int cx, hipStream_t s);

// quads: pencil quads per workgroup (0 default, 1 or 2).
hipError_t launch_zconv_c64(int L, void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw,
                            int quads, hipStream_t s);
hipError_t launch_zconv_c128(int L, void *buf, const void *khat, int64_t Mx, int64_t My, int Nz, const void *tw,
                             int quads, hipStream_t s);

// Multi-task launches (tasks_dev: device array of ntasks entries; blocks: the
// grid size they cover).  sign -1 forward, +1 inverse; scaled: inverse with
// the per-task scale.
hipError_t launch_strided_multi_c64(int L, const StridedTaskArgs *tasks_dev, int ntasks, int64_t blocks, int sign,
                                    int scaled, const void *tw, hipStream_t s);
hipError_t launch_strided_multi_c128(int L, const StridedTaskArgs *tasks_dev, int ntasks, int64_t blocks, int sign,
                                     int scaled, const void *tw, hipStream_t s);
hipError_t launch_zconv_multi_c64(int L, const ZconvTaskArgs *tasks_dev, int ntasks, int64_t blocks, const void *tw,
                                  hipStream_t s);
hipError_t launch_zconv_multi_c128(int L, const ZconvTaskArgs *tasks_dev, int ntasks, int64_t blocks, const void *tw,
                                   hipStream_t s);
// Launch geometry of the default variants: columns per strided workgroup and
// pencils per z-pass workgroup.
int strided_tile_cols(int L, int dbl);
int zconv_slots_per_block(int L, int dbl);

// The kernel by squared integer distance: ktab[q], q < n (see k_kradial);
// (face_re, face_im) is added to the entry q = 1 (zero for the paper's rule).
hipError_t launch_kradial(double2 *ktab, int64_t n, double h, double kr, double ki, double self_re, double self_im,
                          double face_re, double face_im, hipStream_t s);
// Kernel tabulation (gathered from ktab) fused with the first (z) FP64 pass of
// the kernel spectrum; writes the octant [Hx][Hy][Hz] (rows octant_row(L)
// apart) at `out`.
hipError_t launch_kz(int L, double2 *out, const int64_t H[3], const int64_t N[3], const double2 *ktab,
                     const void *tw, hipStream_t s);

}  // namespace nvp
