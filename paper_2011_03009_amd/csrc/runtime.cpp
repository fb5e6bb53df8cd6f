// Host runtime behind the C ABI of include/nvp.h: contexts, plans, grids,
// transfer tables, kernel spectra and the launch sequence of each harmonic.
//
// Built with -ffp-contract=off: the transfer tables decide integer stencil
// positions from floating-point coordinates, and that decision is made with
// plain IEEE double operations in the order written here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/nvp.h"
#include "fft_core.hpp"
#include "launch.hpp"

namespace nvp {
hipError_t launch_box_mask(const void *f, void *out, bool dbl, const int64_t n[3], const int64_t box[6],
                           hipStream_t s);
}  // namespace nvp

using nvp::FieldArgs;
using nvp::SourceArgs;
using nvp::StridedArgs;

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Twiddle {
    int L;
    int dbl;
    void *dev;
};

struct VpCache {
    bool valid = false;
    int quad = -1;
    double kr = 0, ki = 0;
    nvp_grid g{};
    int prec = -1;
    int64_t M[3]{};
    void *khat = nullptr, *A = nullptr, *B = nullptr;
};

}  // namespace

struct nvp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<Twiddle> tw;  // tables of every compiled length, inside tw_blob
    void *tw_blob = nullptr;
    VpCache vp;
    size_t max_lds = 0;
    int quad = NVP_QUAD_BALL;  // quadrature rule of plans and potentials created from now on
    int users = 0;             // live plans, batches and networks made with this context
};

namespace {

struct HarmField {
    int identity = 0;
    size_t off_b[3]{}, off_w[3]{};  // byte offsets in the plan's table blob
};

// Launch choices of one harmonic (the autotuner's search space).
struct Tune {
    int x_tile = 0, y_tile = 0;  // strided passes: 0 default columns per workgroup, 1 half
    int quads = 0;               // z pass: pencil quads per workgroup (0 default, 1, 2)
    int src = -1;                // source build: -1 default, 1 its own kernel, 0 fused into the x pass
    int src_cx = 0;              // source kernel: target x planes per workgroup (0 default)
};

struct Harm {
    Tune tune;
    int n = 0;
    nvp_grid g{};
    int64_t M[3]{};
    double kr = 0, ki = 0, Cn = 0;
    void *khat = nullptr;
    size_t khat_cap = 0;  // bytes allocated at khat
    bool khat_ok = false;
    int chunk = 0;  // x-chunk of the staged source build (0: direct gathers)
    int64_t src_lds = 0;  // > 0: the separate source kernel applies, with this many bytes of LDS
    int src_cx = 0;       // and this many target x planes per workgroup
    HarmField f[NVP_MAX_FIELDS];
};

// The source kernel's x chunk of harmonic h: the tuned one, else the default.
int src_cx_of(const Harm &h) { return h.tune.src_cx > 0 ? h.tune.src_cx : h.src_cx; }

struct TimedEvent {
    int kind;
    hipEvent_t a, b;
};

}  // namespace

struct nvp_plan {
    nvp_ctx *ctx = nullptr;
    int quad = NVP_QUAD_BALL;  // the context's rule when the plan was made
    nvp_prec prec = NVP_C64;
    int order = 1;
    nvp_medium med{};
    double f0 = 0;
    int n_harm = 0;
    nvp_grid g1{};
    std::vector<Harm> h;
    void *A = nullptr, *B = nullptr, *tables = nullptr;
    size_t bytes_A = 0, bytes_B = 0, bytes_tables = 0, bytes_khat = 0;
    bool cache = true;
    bool use_source_kernel = true;  // NVP_FUSED_SOURCE=1 selects the source build fused into the x pass
    bool timing = false;
    std::vector<TimedEvent> events;
    std::vector<hipEvent_t> pool;
    // Kernel spectra computed on a side stream, concurrently with the
    // convolutions (nvp_execute_cascade, spectra not cached, timing off).
    bool overlap = true;
    hipStream_t side = nullptr;
    hipEvent_t ev_start = nullptr;
    std::vector<hipEvent_t> ev_k;
    void *kscr = nullptr, *ktab = nullptr;  // FP64 octant scratch and distance table of the side stream
    size_t bytes_side = 0;
    // false: A, B, kscr and ktab live in a caller-owned workspace
    bool own_work = true;
};

namespace {

const char *g_create_err = "";
std::string g_create_err_buf;

nvp_status fail(nvp_ctx *ctx, nvp_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    else {
        g_create_err_buf = msg;
        g_create_err = g_create_err_buf.c_str();
    }
    return s;
}

// Device allocations of the runtime.  Fault injection for tests: with
// NVP_DEVICE_ALLOC_LIMIT set (bytes), any single allocation larger than that
// fails as out of memory, so that every allocation failure path can be
// exercised with valid sizes.
hipError_t dev_malloc(void **p, size_t bytes) {
    if (const char *lim = getenv("NVP_DEVICE_ALLOC_LIMIT")) {
        char *end = nullptr;
        const unsigned long long cap = strtoull(lim, &end, 10);
        if (end != lim && bytes > cap) {
            *p = nullptr;
            return hipErrorOutOfMemory;
        }
    }
    return hipMalloc(p, bytes);
}

nvp_status hip_fail(nvp_ctx *ctx, const char *what, hipError_t e) {
    return fail(ctx, e == hipErrorOutOfMemory ? NVP_E_NOMEM : NVP_E_HIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define NVP_HIP(ctx, call)                                       \
    do {                                                         \
        hipError_t _e = (call);                                  \
        if (_e != hipSuccess) return hip_fail((ctx), #call, _e); \
    } while (0)

size_t csize(nvp_prec p) { return p == NVP_C64 ? 8 : 16; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

bool grid_ok(const nvp_grid *g) {
    if (!g || !finite_pos(g->h)) return false;
    for (int a = 0; a < 3; ++a)
        if (g->n[a] < 1 || !std::isfinite(g->origin[a])) return false;
    return true;
}

bool medium_ok(const nvp_medium *m) {
    return m && finite_pos(m->c0) && finite_pos(m->rho0) && std::isfinite(m->beta) && std::isfinite(m->alpha0_db) &&
           m->alpha0_db >= 0 && std::isfinite(m->eta);
}

int64_t nint(double x) { return (int64_t)std::floor(x + 0.5); }

const int kLengths[] = {
#define X(n) n,
    NVP_FOR_EACH_LENGTH(X)
#undef X
};

int64_t circulant_len(int64_t n) {
    for (int L : kLengths)
        if (L >= 2 * n - 1) return L;
    return -1;
}

// Per-stage twiddle tables of length L: for the radix plan run forward and
// then in reverse order, stage s >= 1 (radix r, Ns = product of the earlier
// radices) holds exp(-2 pi i j q / (Ns r)) at [j][q-1], j < Ns, 1 <= q < r;
// computed in extended precision and rounded once.  The tables of every
// compiled length, in both precisions, are made once per context, in one
// device allocation at nvp_ctx_create, so that no later call allocates them.
void twiddle_values(int L, std::vector<double> &hd) {
    const int n = nvp::twiddle_table_len(L);
    hd.assign(2 * (size_t)(n > 0 ? n : 1), 0.0);
    size_t e = 0;
    for (int rev = 0; rev < 2; ++rev) {
        const int S = nvp::plan_for(L).S;
        for (int st = 1; st < S; ++st) {
            const int Ns = nvp::plan_ns(L, rev, st), r = nvp::plan_rad(L, rev, st);
            for (int j = 0; j < Ns; ++j)
                for (int q = 1; q < r; ++q, ++e) {
                    long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)(j * q) /
                                      (long double)(Ns * r);
                    hd[2 * e] = (double)cosl(ang);
                    hd[2 * e + 1] = (double)-sinl(ang);
                }
        }
    }
}

nvp_status make_twiddles(nvp_ctx *ctx) {
    std::vector<unsigned char> blob;
    std::vector<std::pair<size_t, std::pair<int, int>>> at;  // offset, (L, dbl)
    std::vector<double> hd;
    for (int L : kLengths) {
        twiddle_values(L, hd);
        for (int dbl = 0; dbl < 2; ++dbl) {
            const size_t off = (blob.size() + 255) / 256 * 256;
            const size_t bytes = hd.size() / 2 * (dbl ? 16 : 8);
            blob.resize(off + bytes);
            if (dbl) {
                std::memcpy(blob.data() + off, hd.data(), bytes);
            } else {
                float *f = reinterpret_cast<float *>(blob.data() + off);
                for (size_t i = 0; i < hd.size(); ++i) f[i] = (float)hd[i];
            }
            at.push_back({off, {L, dbl}});
        }
    }
    void *dev = nullptr;
    hipError_t e = dev_malloc(&dev, blob.size());
    if (e != hipSuccess) return hip_fail(ctx, "twiddle tables", e);
    e = hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(ctx, "twiddle upload", e);
    }
    ctx->tw_blob = dev;
    for (auto &a : at) ctx->tw.push_back({a.second.first, a.second.second, static_cast<unsigned char *>(dev) + a.first});
    return NVP_OK;
}

nvp_status twiddles(nvp_ctx *ctx, int L, bool dbl, const void **out) {
    for (auto &t : ctx->tw)
        if (t.L == L && t.dbl == (int)dbl) {
            *out = t.dev;
            return NVP_OK;
        }
    return fail(ctx, NVP_E_UNSUPPORTED, "no compiled transform of length " + std::to_string(L));
}

void self_cell(double kr, double ki, double h, double *re, double *im) {
    // (e^{ika} (1 - ika) - 1) / k^2 with a = (3 / (4 pi))^(1/3) h
    const double a = std::cbrt(3.0 / (4.0 * kPi)) * h;
    const double ar = kr * a, ai = ki * a;
    const double mag = std::exp(-ai);
    const double er = mag * std::cos(ar), ei = mag * std::sin(ar);
    const double br = 1.0 + ai, bi = -ar;
    const double nr = er * br - ei * bi - 1.0, ni = er * bi + ei * br;
    const double k2r = kr * kr - ki * ki, k2i = 2.0 * kr * ki;
    const double den = k2r * k2r + k2i * k2i;
    *re = (nr * k2r + ni * k2i) / den;
    *im = (ni * k2r - nr * k2i) / den;
}

// Epstein zeta function of the cubic lattice, Z(s) = sum over n in Z^3 \ {0}
// of |n|^{-2s} (continued analytically), at s = 1/2 and s = -1/2.
constexpr double kZetaHalf = -2.8372974794806196;
constexpr double kZetaMinusHalf = -0.26659627871839353;

// Self-voxel kernel value and the addition at the six face neighbours of
// quadrature rule `rule`: the paper's equal-volume ball (equation "quad",
// nothing added at the faces), or the corrected lattice rule.  The corrected
// rule keeps the midpoint sum over the other voxels and removes the error of
// G's singular Taylor terms 1/(4 pi r) and -k^2 r/(8 pi) (and restores the
// constant term ik/(4 pi) at the target) by the lattice-zeta weights
//   self = h^2 (Z(-1/2) - Z(1/2)) / (4 pi) + i k h^3 / (4 pi) + k^2 h^4 Z(-1/2) / (8 pi),
//   face = -h^2 Z(-1/2) / (24 pi)
// (a corrected trapezoidal rule for singular integrands; the face weight is
// the 7-point Laplacian of the h^4 term).
void quad_weights(int rule, double kr, double ki, double h, double *sr, double *si, double *fr, double *fi) {
    if (rule != NVP_QUAD_CORRECTED) {
        self_cell(kr, ki, h, sr, si);
        *fr = *fi = 0.0;
        return;
    }
    const std::complex<double> k(kr, ki), I(0.0, 1.0);
    const double h2 = h * h, c4 = 4.0 * kPi;
    const std::complex<double> w = h2 * (kZetaMinusHalf - kZetaHalf) / c4 + I * k * (h2 * h) / c4 +
                                   k * k * (h2 * h2) * kZetaMinusHalf / (2.0 * c4);
    *sr = w.real();
    *si = w.imag();
    *fr = -h2 * kZetaMinusHalf / (6.0 * c4);
    *fi = 0.0;
}

nvp_status check_grid_lengths(nvp_ctx *ctx, const nvp_grid *g, int64_t M[3]) {
    for (int a = 0; a < 3; ++a) {
        M[a] = circulant_len(g->n[a]);
        if (M[a] < 0)
            return fail(ctx, NVP_E_UNSUPPORTED,
                        "axis of " + std::to_string(g->n[a]) + " voxels: the longest transform is " +
                            std::to_string(kLengths[sizeof kLengths / sizeof kLengths[0] - 1]) +
                            ", so axes are limited to " +
                            std::to_string((kLengths[sizeof kLengths / sizeof kLengths[0] - 1] + 1) / 2) + " voxels");
    }
    return NVP_OK;
}

// ------------------------------------------------------------------ timing

struct Timer {
    nvp_plan *p;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(nvp_plan *plan, int k) : p(plan), kind(k) {
        if (!p || !p->timing) return;
        a = take();
        b = take();
        if (a && b) (void)hipEventRecord(a, p->ctx->stream);
    }
    hipEvent_t take() {
        if (!p->pool.empty()) {
            hipEvent_t e = p->pool.back();
            p->pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~Timer() {
        if (!p || !p->timing || !a || !b) return;
        (void)hipEventRecord(b, p->ctx->stream);
        p->events.push_back({kind, a, b});
    }
};

// ------------------------------------------------------------------ kernel spectrum

// Entries of the kernel-by-squared-distance table of grid g: every |d|^2 of
// an offset inside the grid.
int64_t radial_entries(const nvp_grid *g) {
    return (g->n[0] - 1) * (g->n[0] - 1) + (g->n[1] - 1) * (g->n[1] - 1) + (g->n[2] - 1) * (g->n[2] - 1) + 1;
}

// Octant of the FP64 DFT of the circulant-embedded kernel, stored as
// [Mx/2+1][My/2+1][Mz/2+1] (rows padded to octant_row(Mz)) in the plan
// precision at `khat`.  `scratch` holds the FP64 octant during the three
// passes, `ktab` the kernel by squared distance (radial_entries(g) FP64 values).
nvp_status kernel_spectrum(nvp_ctx *ctx, nvp_plan *timed, int quad, double kr, double ki, const nvp_grid *g,
                           const int64_t M[3], nvp_prec prec, void *khat, void *scratch, void *ktab) {
    const int64_t H[3] = {M[0] / 2 + 1, M[1] / 2 + 1, M[2] / 2 + 1};
    double sr, si, fr, fi;  // self voxel, face-neighbour addition
    quad_weights(quad, kr, ki, g->h, &sr, &si, &fr, &fi);
    const void *tw;
    nvp_status st;
    // z: tabulation fused with the FFT of the even extension of each octant row
    if ((st = twiddles(ctx, (int)M[2], true, &tw))) return st;
    {
        Timer t(timed, NVP_T_KTAB);
        NVP_HIP(ctx, nvp::launch_kradial(static_cast<double2 *>(ktab), radial_entries(g), g->h, kr, ki, sr, si, fr,
                                         fi, ctx->stream));
        NVP_HIP(ctx, nvp::launch_kz((int)M[2], static_cast<double2 *>(scratch), H, g->n,
                                    static_cast<const double2 *>(ktab), tw, ctx->stream));
    }
    Timer t(timed, NVP_T_KFFT);
    const int64_t HZS = nvp::octant_row(M[2]);  // padded row stride along z
    StridedArgs a{};
    // y
    if ((st = twiddles(ctx, (int)M[1], true, &tw))) return st;
    a.in = scratch; a.in_os = H[1] * HZS; a.in_ms = HZS; a.mirror = 1;
    a.out = scratch; a.out_os = H[1] * HZS; a.out_ms = HZS; a.n_out = (int)H[1];
    a.scale = 1.0; a.inner = H[2]; a.outer = H[0]; a.sign = -1;
    NVP_HIP(ctx, nvp::launch_strided_c128((int)M[1], a, tw, ctx->stream));
    // x, written in the plan precision; columns (y, z) as outer y, inner z
    if ((st = twiddles(ctx, (int)M[0], true, &tw))) return st;
    a = StridedArgs{};
    a.in = scratch; a.in_os = HZS; a.in_ms = H[1] * HZS; a.mirror = 1;
    a.out = khat; a.out_os = HZS; a.out_ms = H[1] * HZS; a.n_out = (int)H[0];
    a.scale = 1.0; a.inner = H[2]; a.outer = H[1]; a.sign = -1;
    if (prec == NVP_C64) NVP_HIP(ctx, nvp::launch_strided_f64_c64((int)M[0], a, tw, ctx->stream));
    else NVP_HIP(ctx, nvp::launch_strided_c128((int)M[0], a, tw, ctx->stream));
    return NVP_OK;
}

size_t khat_bytes(const int64_t M[3], nvp_prec prec) {
    return (size_t)(M[0] / 2 + 1) * (M[1] / 2 + 1) * nvp::octant_row(M[2]) * csize(prec);
}
size_t kscratch_bytes(const int64_t M[3]) {
    return (size_t)(M[0] / 2 + 1) * (M[1] / 2 + 1) * nvp::octant_row(M[2]) * 16;
}

// ------------------------------------------------------------------ the five passes

// x fwd (either from `f` directly or from the fused source), y fwd, z conv,
// y inv, x inv with `scale` into u.
nvp_status convolve(nvp_ctx *ctx, nvp_plan *timed, nvp_prec prec, const nvp_grid *g, const int64_t M[3],
                    const void *khat, void *A, void *B, const void *f, const SourceArgs *src, void *u,
                    double scale, int src_cx = 0, const Tune &tn = Tune{}, hipEvent_t kready = nullptr) {
    const int64_t Nx = g->n[0], Ny = g->n[1], Nz = g->n[2];
    const int64_t Mx = M[0], My = M[1], Mz = M[2];
    const bool dbl = prec == NVP_C128;
    const void *twx, *twy, *twz;
    nvp_status st;
    if ((st = twiddles(ctx, (int)Mx, dbl, &twx))) return st;
    if ((st = twiddles(ctx, (int)My, dbl, &twy))) return st;
    if ((st = twiddles(ctx, (int)Mz, dbl, &twz))) return st;
    auto strided = dbl ? nvp::launch_strided_c128 : nvp::launch_strided_c64;
    if (src && src_cx > 0) {
        // transfer + source into the first Nx rows of A, then the x pass in place
        {
            Timer t(timed, NVP_T_SRC);
            NVP_HIP(ctx, (dbl ? nvp::launch_source_c128 : nvp::launch_source_c64)(*src, A, (int)Ny, src_cx,
                                                                                ctx->stream));
        }
        f = A;
        src = nullptr;
    }
    {
        Timer t(timed, NVP_T_XFWD);
        if (src) {
            SourceArgs s = *src;
            s.out = A;
            s.out_ms = Ny * Nz;
            s.inner = Ny * Nz;
            NVP_HIP(ctx, (dbl ? nvp::launch_xsrc_c128 : nvp::launch_xsrc_c64)((int)Mx, s, twx, ctx->stream));
        } else {
            StridedArgs a{};
            a.in = f; a.in_os = 0; a.in_ms = Ny * Nz; a.n_in = (int)Nx;
            a.out = A; a.out_os = 0; a.out_ms = Ny * Nz; a.n_out = (int)Mx;
            a.scale = 1.0; a.inner = Ny * Nz; a.outer = 1; a.sign = -1; a.tile = tn.x_tile;
            NVP_HIP(ctx, strided((int)Mx, a, twx, ctx->stream));
        }
    }
    {
        Timer t(timed, NVP_T_YFWD);
        StridedArgs a{};
        a.in = A; a.in_os = Ny * Nz; a.in_ms = Nz; a.n_in = (int)Ny;
        a.out = B; a.out_os = My * Nz; a.out_ms = Nz; a.n_out = (int)My;
        a.scale = 1.0; a.inner = Nz; a.outer = Mx; a.sign = -1; a.tile = tn.y_tile;
        NVP_HIP(ctx, strided((int)My, a, twy, ctx->stream));
    }
    if (kready) NVP_HIP(ctx, hipStreamWaitEvent(ctx->stream, kready, 0));  // the kernel spectrum's side stream
    {
        Timer t(timed, NVP_T_ZCONV);
        NVP_HIP(ctx, (dbl ? nvp::launch_zconv_c128 : nvp::launch_zconv_c64)((int)Mz, B, khat, Mx, My, (int)Nz, twz,
                                                                          tn.quads, ctx->stream));
    }
    {
        Timer t(timed, NVP_T_YINV);
        StridedArgs a{};
        a.in = B; a.in_os = My * Nz; a.in_ms = Nz; a.n_in = (int)My;
        a.out = A; a.out_os = Ny * Nz; a.out_ms = Nz; a.n_out = (int)Ny;
        a.scale = 1.0; a.inner = Nz; a.outer = Mx; a.sign = 1; a.tile = tn.y_tile;
        NVP_HIP(ctx, strided((int)My, a, twy, ctx->stream));
    }
    {
        Timer t(timed, NVP_T_XINV);
        StridedArgs a{};
        a.in = A; a.in_os = 0; a.in_ms = Ny * Nz; a.n_in = (int)Mx;
        a.out = u; a.out_os = 0; a.out_ms = Ny * Nz; a.n_out = (int)Nx;
        a.scale = scale; a.inner = Ny * Nz; a.outer = 1; a.sign = 1; a.tile = tn.x_tile;
        NVP_HIP(ctx, strided((int)Mx, a, twx, ctx->stream));
    }
    return NVP_OK;
}

// Buffer A: the x-pass buffer [Mx][Ny][Nz]; before the convolution it holds
// the kernel-by-squared-distance table of the kernel spectrum.
size_t bytesA(const nvp_grid *g, const int64_t M[3], nvp_prec p) {
    const size_t a = (size_t)M[0] * g->n[1] * g->n[2] * csize(p), t = (size_t)radial_entries(g) * 16;
    return a > t ? a : t;
}
size_t bytesB(const nvp_grid *g, const int64_t M[3], nvp_prec p) {
    size_t b = (size_t)M[0] * M[1] * g->n[2] * csize(p);
    size_t k = kscratch_bytes(M);
    return b > k ? b : k;
}

bool same_grid(const nvp_grid &a, const nvp_grid &b) {
    return std::memcmp(a.origin, b.origin, sizeof a.origin) == 0 && a.h == b.h &&
           std::memcmp(a.n, b.n, sizeof a.n) == 0;
}

// The context's volume-potential buffers and kernel spectrum for (rule, k, g,
// prec): kept from the last call when they match, else made again.
nvp_status vp_prepare(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const int64_t M[3], nvp_prec prec) {
    VpCache &c = ctx->vp;
    const bool hit = c.valid && c.quad == ctx->quad && c.kr == k_re && c.ki == k_im && c.prec == (int)prec &&
                     same_grid(c.g, *g);
    if (hit) return NVP_OK;
    // same grid and precision: keep the buffers, remake only the spectrum
    if (c.khat && c.prec == (int)prec && same_grid(c.g, *g)) {
        c.valid = false;
        nvp_status st = kernel_spectrum(ctx, nullptr, ctx->quad, k_re, k_im, g, M, prec, c.khat, c.B, c.A);
        if (st) return st;
        c.valid = true;
        c.quad = ctx->quad;
        c.kr = k_re;
        c.ki = k_im;
        return NVP_OK;
    }
    NVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (c.khat) (void)hipFree(c.khat);
    if (c.A) (void)hipFree(c.A);
    if (c.B) (void)hipFree(c.B);
    c = VpCache{};
    hipError_t e1 = dev_malloc((void **)&c.khat, khat_bytes(M, prec));
    hipError_t e2 = dev_malloc((void **)&c.A, bytesA(g, M, prec));
    hipError_t e3 = dev_malloc((void **)&c.B, bytesB(g, M, prec));
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        if (c.khat) (void)hipFree(c.khat);
        if (c.A) (void)hipFree(c.A);
        if (c.B) (void)hipFree(c.B);
        c = VpCache{};
        return fail(ctx, NVP_E_NOMEM, "volume potential: device allocation failed");
    }
    nvp_status st = kernel_spectrum(ctx, nullptr, ctx->quad, k_re, k_im, g, M, prec, c.khat, c.B, c.A);
    if (st) {
        c.valid = false;
        return st;
    }
    c.valid = true;
    c.quad = ctx->quad;
    c.kr = k_re;
    c.ki = k_im;
    c.g = *g;
    c.prec = (int)prec;
    std::memcpy(c.M, M, sizeof M);
    return NVP_OK;
}

// 1-D interpolation of a source axis at the target centres (clamped into the
// source hull): order 1 linear, order 3 four-point Lagrange with the stencil
// shifted inward at the edges.
void axis_table(double dst_o, double dst_h, int64_t dst_n, double src_o, double src_h, int64_t src_n, int order,
                int *base, double *w) {
    const int K = order + 1;
    for (int64_t i = 0; i < dst_n; ++i) {
        const double x = dst_o + (double)i * dst_h;
        double s = (x - src_o) / src_h;
        s = std::fmin(std::fmax(s, 0.0), (double)(src_n - 1));
        const double i0 = std::fmin(std::floor(s), (double)(src_n - 2));
        if (order == 1) {
            const double t = s - i0;
            base[i] = (int)i0;
            w[i * K] = 1.0 - t;
            w[i * K + 1] = t;
        } else {
            const double b = std::fmin(std::fmax(i0 - 1.0, 0.0), (double)(src_n - 4));
            const double u = s - b;
            base[i] = (int)b;
            w[i * K] = -(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0;
            w[i * K + 1] = u * (u - 2.0) * (u - 3.0) / 2.0;
            w[i * K + 2] = -u * (u - 1.0) * (u - 3.0) / 2.0;
            w[i * K + 3] = u * (u - 1.0) * (u - 2.0) / 6.0;
        }
    }
}

// The transient work buffers: the two pass buffers and the second stream's
// spectrum scratch (freed here only when the plan owns them).
void release_work(nvp_plan *p) {
    if (p->own_work) {
        if (p->kscr) (void)hipFree(p->kscr);
        if (p->ktab) (void)hipFree(p->ktab);
        if (p->A) (void)hipFree(p->A);
        if (p->B) (void)hipFree(p->B);
    }
    p->kscr = p->ktab = p->A = p->B = nullptr;
    p->bytes_side = 0;
    p->own_work = true;
}

// Sizes of the second stream's FP64 octant scratch and distance table.
void side_sizes(const nvp_plan *p, size_t *ks, size_t *kt) {
    *ks = *kt = 0;
    for (auto &h : p->h) {
        *ks = std::max(*ks, kscratch_bytes(h.M));
        *kt = std::max(*kt, (size_t)radial_entries(&h.g) * 16);
    }
}

// Offsets of A, B, kscr and ktab inside a caller workspace; returns its size.
size_t work_layout(const nvp_plan *p, size_t off[4]) {
    size_t ks, kt;
    side_sizes(p, &ks, &kt);
    const size_t sz[4] = {p->bytes_A, p->bytes_B, ks, kt};
    size_t o = 0;
    for (int i = 0; i < 4; ++i) {
        off[i] = o;
        o += (sz[i] + 255) / 256 * 256;
    }
    return o;
}

void free_plan_memory(nvp_plan *p) {
    if (p->side) {
        (void)hipStreamSynchronize(p->side);
        (void)hipStreamDestroy(p->side);
        p->side = nullptr;
    }
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    p->ev_start = nullptr;
    for (auto e : p->ev_k) (void)hipEventDestroy(e);
    p->ev_k.clear();
    release_work(p);
    for (auto &h : p->h)
        if (h.khat) (void)hipFree(h.khat), h.khat = nullptr;
    if (p->tables) (void)hipFree(p->tables);
    p->tables = nullptr;
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    p->events.clear();
    for (auto e : p->pool) (void)hipEventDestroy(e);
    p->pool.clear();
}

// Transfer + source arguments of harmonic n from fields[m-1] = p_m.
SourceArgs source_args(const nvp_plan *plan, int n, const void *const *fields) {
    const Harm &h = plan->h[n - 2];
    SourceArgs src{};
    src.nf = n - 1;
    src.order = plan->order;
    src.Nx = (int)h.g.n[0];
    src.Nz = (int)h.g.n[2];
    src.chunk = h.chunk;
    const unsigned char *tb = static_cast<const unsigned char *>(plan->tables);
    for (int m = 1; m < n; ++m) {
        const nvp_grid &sg = m == 1 ? plan->g1 : plan->h[m - 2].g;
        FieldArgs &fa = src.f[m - 1];
        const HarmField &hf = h.f[m - 1];
        fa.p = fields[m - 1];
        fa.s0 = sg.n[1] * sg.n[2];
        fa.s1 = sg.n[2];
        fa.identity = hf.identity;
        for (int ax = 0; ax < 3; ++ax) {
            fa.b[ax] = hf.identity ? nullptr : reinterpret_cast<const int *>(tb + hf.off_b[ax]);
            fa.w[ax] = hf.identity ? nullptr : static_cast<const void *>(tb + hf.off_w[ax]);
        }
    }
    return src;
}

}  // namespace

// =================================================================== C ABI

namespace nvp {

// Looks up the fixed scratch array of nvp_volume_potential_noalloc on the
// context's device (noalloc.hip).
nvp_status noalloc_setup(nvp_ctx *ctx);

// Context access for the other translation units behind the C ABI.
int ctx_device(const nvp_ctx *c) { return c->device; }
void ctx_attach(nvp_ctx *c) { ++c->users; }
void ctx_detach(nvp_ctx *c) { --c->users; }
hipStream_t ctx_stream(const nvp_ctx *c) { return c->stream; }
nvp_status ctx_fail(nvp_ctx *c, nvp_status s, const char *msg) { return fail(c, s, msg); }
nvp_status ctx_hip_fail(nvp_ctx *c, const char *what, hipError_t e) { return hip_fail(c, what, e); }
void ctx_quad_weights(const nvp_ctx *c, double kr, double ki, double h, double *sr, double *si, double *fr,
                      double *fi) {
    quad_weights(c->quad, kr, ki, h, sr, si, fr, fi);
}

// The volume potential of nvp_volume_potential in buffers the caller places:
// checks the arguments, reports the bytes of the three buffers (kernel-spectrum
// octant, pass buffer A, pass buffer B), and, when the buffers are given,
// computes the kernel spectrum into them and convolves, with the same kernels,
// tables and launch choices as nvp_volume_potential (no cache: the spectrum is
// made on every call).  Allocates nothing.
nvp_status vp_buffers(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev, void *u_dev,
                      nvp_prec prec, size_t bytes[3], void *khat, void *A, void *B) {
    if (!ctx) return NVP_E_INVALID;
    if (!grid_ok(g) || !f_dev || !u_dev || f_dev == u_dev || (prec != NVP_C64 && prec != NVP_C128) ||
        !std::isfinite(k_re) || !std::isfinite(k_im) || k_im < 0 || (k_re == 0 && k_im == 0))
        return fail(ctx, NVP_E_INVALID, "volume potential: bad argument");
    int64_t M[3];
    nvp_status st = check_grid_lengths(ctx, g, M);
    if (st) return st;
    bytes[0] = khat_bytes(M, prec);
    bytes[1] = bytesA(g, M, prec);
    bytes[2] = bytesB(g, M, prec);
    if (!khat || !A || !B) return NVP_OK;
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    if ((st = kernel_spectrum(ctx, nullptr, ctx->quad, k_re, k_im, g, M, prec, khat, B, A))) return st;
    const double scale = -1.0 / ((double)M[0] * (double)M[1] * (double)M[2]);
    return convolve(ctx, nullptr, prec, g, M, khat, A, B, f_dev, nullptr, u_dev, scale);
}

}  // namespace nvp

extern "C" {

const char *nvp_status_str(nvp_status s) {
    switch (s) {
    case NVP_OK: return "ok";
    case NVP_E_INVALID: return "invalid argument";
    case NVP_E_NOMEM: return "out of memory";
    case NVP_E_HIP: return "HIP error";
    case NVP_E_UNSUPPORTED: return "unsupported";
    case NVP_E_STATE: return "bad state";
    default: return "unknown status";
    }
}

const char *nvp_last_error(const nvp_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err; }

nvp_status nvp_ctx_create(int device, void *hip_stream, nvp_ctx **out) {
    if (!out) return fail(nullptr, NVP_E_INVALID, "out is null");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(nullptr, "hipGetDeviceCount", e);
    if (device < 0 || device >= count) return fail(nullptr, NVP_E_INVALID, "no such device");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, "hipSetDevice", e);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(nullptr, "hipGetDeviceProperties", e);
    nvp_ctx *c = new (std::nothrow) nvp_ctx;
    if (!c) return fail(nullptr, NVP_E_NOMEM, "context allocation");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->max_lds = prop.sharedMemPerBlock;
    nvp_status st = make_twiddles(c);
    if (!st) st = nvp::noalloc_setup(c);
    if (st) {
        g_create_err_buf = c->err;
        g_create_err = g_create_err_buf.c_str();
        delete c;
        return st;
    }
    *out = c;
    return NVP_OK;
}

nvp_status nvp_ctx_set_quadrature(nvp_ctx *ctx, int rule) {
    if (!ctx) return NVP_E_INVALID;
    if (rule != NVP_QUAD_BALL && rule != NVP_QUAD_CORRECTED)
        return fail(ctx, NVP_E_INVALID, "nvp_ctx_set_quadrature: unknown rule");
    ctx->quad = rule;
    return NVP_OK;
}

nvp_status nvp_quadrature_weights(int rule, double k_re, double k_im, double h, double w[4]) {
    if (!w || (rule != NVP_QUAD_BALL && rule != NVP_QUAD_CORRECTED) || !std::isfinite(k_re) ||
        !std::isfinite(k_im) || (k_re == 0 && k_im == 0) || !finite_pos(h))
        return NVP_E_INVALID;
    quad_weights(rule, k_re, k_im, h, &w[0], &w[1], &w[2], &w[3]);
    return NVP_OK;
}

nvp_status nvp_ctx_destroy(nvp_ctx *ctx) {
    if (!ctx) return NVP_E_INVALID;
    if (ctx->users > 0)  // their destroy calls still reach the context
        return fail(ctx, NVP_E_STATE,
                    "nvp_ctx_destroy: " + std::to_string(ctx->users) + " plans, batches or networks still use this context");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->tw_blob) (void)hipFree(ctx->tw_blob);
    if (ctx->vp.khat) (void)hipFree(ctx->vp.khat);
    if (ctx->vp.A) (void)hipFree(ctx->vp.A);
    if (ctx->vp.B) (void)hipFree(ctx->vp.B);
    delete ctx;
    return NVP_OK;
}

nvp_status nvp_ctx_sync(nvp_ctx *ctx) {
    if (!ctx) return NVP_E_INVALID;
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    NVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    NVP_HIP(ctx, hipGetLastError());
    return NVP_OK;
}

nvp_status nvp_wavenumber(const nvp_medium *med, double f0, int n, double *k_re, double *k_im) {
    if (!medium_ok(med) || !finite_pos(f0) || n < 1 || !k_re || !k_im) return NVP_E_INVALID;
    const double f = n * f0;
    *k_re = 2.0 * kPi * f / med->c0;
    // alpha0 in dB/m at 1 MHz, eta the frequency exponent; dB -> Np: / (20 log10 e)
    *k_im = med->alpha0_db * std::pow(f / 1.0e6, med->eta) / (20.0 * std::log10(std::exp(1.0)));
    return NVP_OK;
}

nvp_status nvp_cascade_constant(const nvp_medium *med, double f0, int n, double *c) {
    if (!medium_ok(med) || !finite_pos(f0) || n < 1 || !c) return NVP_E_INVALID;
    const double w = 2.0 * kPi * f0;
    const double c2 = med->c0 * med->c0;
    *c = -med->beta * w * w * (double)n * (double)n / (2.0 * med->rho0 * c2 * c2);
    return NVP_OK;
}

nvp_status nvp_spacing(const nvp_medium *med, double f0, int n, int n_w, double *h) {
    if (!medium_ok(med) || !finite_pos(f0) || n < 1 || n_w < 1 || !h) return NVP_E_INVALID;
    *h = med->c0 / (n * f0) / n_w;
    return NVP_OK;
}

nvp_status nvp_grid_from_counts(const double focus[3], double h, const int64_t n[3], const int64_t i_f[3],
                                nvp_grid *out) {
    if (!focus || !n || !i_f || !out || !finite_pos(h)) return NVP_E_INVALID;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1 || !std::isfinite(focus[a])) return NVP_E_INVALID;
        out->origin[a] = focus[a] - (double)i_f[a] * h;
        out->n[a] = n[a];
    }
    out->h = h;
    return NVP_OK;
}

nvp_status nvp_grid_from_box(const double focus[3], const double lo[3], const double hi[3], double h, nvp_grid *out,
                             int64_t i_f_out[3]) {
    if (!focus || !lo || !hi || !out || !finite_pos(h)) return NVP_E_INVALID;
    int64_t n[3], i_f[3];
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] >= lo[a])) return NVP_E_INVALID;
        const int64_t c = nint((hi[a] - lo[a]) / h);
        n[a] = c > 1 ? c : 1;
        i_f[a] = nint((focus[a] - lo[a]) / h);
        if (i_f_out) i_f_out[a] = i_f[a];
    }
    return nvp_grid_from_counts(focus, h, n, i_f, out);
}

nvp_status nvp_rule_of_thumb_box(int n, double l, double R, double d, double eps, double lo[3], double hi[3]) {
    if (n < 2 || !finite_pos(l) || !finite_pos(R) || !(R < l) || !(d >= 0) || !(eps >= 0) || !lo || !hi)
        return NVP_E_INVALID;
    const double L = std::sqrt(l * l - R * R) - eps;
    const double s = 2.0 / n;  // lambda_n / lambda_2
    lo[0] = l - s * L;
    lo[1] = -s * R;
    lo[2] = -s * R;
    hi[0] = l + d;
    hi[1] = s * R;
    hi[2] = s * R;
    return NVP_OK;
}

nvp_status nvp_transfer_axis(double dst_origin, double dst_h, int64_t dst_n, double src_origin, double src_h,
                             int64_t src_n, int order, int32_t *base, double *w) {
    if ((order != 1 && order != 3) || dst_n < 1 || src_n < order + 1 || !base || !w || !finite_pos(dst_h) ||
        !finite_pos(src_h) || !std::isfinite(dst_origin) || !std::isfinite(src_origin))
        return NVP_E_INVALID;
    std::vector<int> b((size_t)dst_n);
    axis_table(dst_origin, dst_h, dst_n, src_origin, src_h, src_n, order, b.data(), w);
    for (int64_t i = 0; i < dst_n; ++i) base[i] = b[i];
    return NVP_OK;
}

nvp_status nvp_circulant_size(int64_t n, int64_t *m) {
    if (n < 1 || !m) return NVP_E_INVALID;
    *m = circulant_len(n);
    return *m < 0 ? NVP_E_UNSUPPORTED : NVP_OK;
}

nvp_status nvp_transform_lengths(int32_t *lengths, int capacity, int *count) {
    if (!count || capacity < 0 || (capacity > 0 && !lengths)) return NVP_E_INVALID;
    const int n = (int)(sizeof kLengths / sizeof kLengths[0]);
    *count = n;
    for (int i = 0; i < n && i < capacity; ++i) lengths[i] = kLengths[i];
    return NVP_OK;
}

nvp_status nvp_volume_potential(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev,
                                void *u_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    if (!grid_ok(g) || !f_dev || !u_dev || f_dev == u_dev || (prec != NVP_C64 && prec != NVP_C128) ||
        !std::isfinite(k_re) || !std::isfinite(k_im) || k_im < 0 || (k_re == 0 && k_im == 0))
        return fail(ctx, NVP_E_INVALID, "nvp_volume_potential: bad argument");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    int64_t M[3];
    nvp_status st = check_grid_lengths(ctx, g, M);
    if (st) return st;
    if ((st = vp_prepare(ctx, k_re, k_im, g, M, prec))) return st;
    const double scale = -1.0 / ((double)M[0] * (double)M[1] * (double)M[2]);
    return convolve(ctx, nullptr, prec, g, M, ctx->vp.khat, ctx->vp.A, ctx->vp.B, f_dev, nullptr, u_dev, scale);
}

nvp_status nvp_volume_potential_box(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev,
                                    const int64_t *box, double scale, void *u_dev, nvp_prec prec) {
    if (!ctx) return NVP_E_INVALID;
    if (!grid_ok(g) || !f_dev || !u_dev || f_dev == u_dev || (prec != NVP_C64 && prec != NVP_C128) ||
        !std::isfinite(k_re) || !std::isfinite(k_im) || k_im < 0 || (k_re == 0 && k_im == 0) ||
        !std::isfinite(scale))
        return fail(ctx, NVP_E_INVALID, "nvp_volume_potential_box: bad argument");
    if (box)
        for (int a = 0; a < 3; ++a)
            if (box[a] < 0 || box[a] > box[a + 3] || box[a + 3] >= g->n[a])
                return fail(ctx, NVP_E_INVALID, "nvp_volume_potential_box: box outside the grid or empty");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    int64_t M[3];
    nvp_status st = check_grid_lengths(ctx, g, M);
    if (st) return st;
    if ((st = vp_prepare(ctx, k_re, k_im, g, M, prec))) return st;
    VpCache &c = ctx->vp;
    const void *f = f_dev;
    if (box) {
        // the source restricted to the box, in the first Nx rows of the x-pass buffer (the x pass
        // then runs in place there; the kernel spectrum no longer needs that buffer)
        NVP_HIP(ctx, nvp::launch_box_mask(f_dev, c.A, prec == NVP_C128, g->n, box, ctx->stream));
        f = c.A;
    }
    const double sc = scale / ((double)M[0] * (double)M[1] * (double)M[2]);
    return convolve(ctx, nullptr, prec, g, M, c.khat, c.A, c.B, f, nullptr, u_dev, sc);
}

// Target x planes per source-kernel workgroup: enough x chunks for about
// `want` workgroups per launch (0: 2048, or the environment variable
// NVP_SRC_WGS, read once), and at most SRC_CXM planes.
int source_chunk(const int64_t n[3], size_t rsize, int64_t want = 0, int nf = 4) {
    static const int64_t dflt = [] {
        const char *e = getenv("NVP_SRC_WGS");
        const long v = e ? atol(e) : 0;
        return v > 0 ? (int64_t)v : (int64_t)2048;
    }();
    if (want <= 0) want = nvp::source_wf(rsize) ? dflt * 4 / std::max(1, nf) : dflt;  // about 8192 wavefronts
    const int64_t ty = (int64_t)NVP_SRC_TY * nvp::source_rows(rsize);
    const int64_t tiles = ((n[1] + ty - 1) / ty) * ((n[2] + NVP_SRC_TZ - 1) / NVP_SRC_TZ);
    int64_t chunks = std::max<int64_t>(1, std::min<int64_t>((want + tiles - 1) / tiles, n[0]));
    chunks = std::max<int64_t>(chunks, (n[0] + NVP_SRC_CXM - 1) / NVP_SRC_CXM);  // at most SRC_CXM planes each
    return (int)((n[0] + chunks - 1) / chunks);
}


// Grids, constants, transfer tables (built on the host into `host`) and
// source-build choices of every harmonic of plan p for the harmonic grids gn,
// and the sizes of its pass buffers.  Sets no device memory.
nvp_status plan_layout(nvp_ctx *ctx, nvp_plan *p, const nvp_grid *gn, std::vector<unsigned char> &host,
                       size_t *tbytes_out, size_t *maxA_out, size_t *maxB_out) {
    const int K = p->order + 1;
    const size_t rs = p->prec == NVP_C64 ? 4 : 8;
    size_t maxA = 0, maxB = 0, tbytes = 0;
    auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
    for (int i = 0; i < p->n_harm - 1; ++i) {
        Harm &h = p->h[i];
        h.n = i + 2;
        h.g = gn[i];
        nvp_status st = check_grid_lengths(ctx, &h.g, h.M);
        if (st) return st;
        nvp_wavenumber(&p->med, p->f0, h.n, &h.kr, &h.ki);
        nvp_cascade_constant(&p->med, p->f0, h.n, &h.Cn);
        size_t a = bytesA(&h.g, h.M, p->prec), b = bytesB(&h.g, h.M, p->prec);
        maxA = a > maxA ? a : maxA;
        maxB = b > maxB ? b : maxB;
        for (int m = 1; m < h.n; ++m) {
            const nvp_grid &src = m == 1 ? p->g1 : gn[m - 2];
            HarmField &f = h.f[m - 1];
            f.identity = same_grid(src, h.g) ? 1 : 0;
            if (f.identity) continue;
            for (int ax = 0; ax < 3; ++ax) {
                if (src.n[ax] < K)
                    return fail(ctx, NVP_E_INVALID, "a source grid axis is shorter than the transfer stencil");
                f.off_b[ax] = tbytes;
                tbytes = align(tbytes + (size_t)h.g.n[ax] * sizeof(int));
                f.off_w[ax] = tbytes;
                tbytes = align(tbytes + (size_t)h.g.n[ax] * K * rs);
            }
        }
    }
    // tables on the host, then one upload
    host.assign(tbytes ? tbytes : 1, 0);
    for (auto &h : p->h) {
        for (int m = 1; m < h.n; ++m) {
            const nvp_grid &src = m == 1 ? p->g1 : gn[m - 2];
            HarmField &f = h.f[m - 1];
            if (f.identity) continue;
            for (int ax = 0; ax < 3; ++ax) {
                std::vector<double> w((size_t)h.g.n[ax] * K);
                int *base = reinterpret_cast<int *>(host.data() + f.off_b[ax]);
                axis_table(h.g.origin[ax], h.g.h, h.g.n[ax], src.origin[ax], src.h, src.n[ax], p->order, base,
                           w.data());
                if (rs == 8) std::memcpy(host.data() + f.off_w[ax], w.data(), w.size() * 8);
                else {
                    float *wf = reinterpret_cast<float *>(host.data() + f.off_w[ax]);
                    for (size_t j = 0; j < w.size(); ++j) wf[j] = (float)w[j];
                }
            }
        }
    }
    // Chunk of the staged source build: the largest x-chunk whose source rows
    // (K-point stencils of every interpolated field) fit in the Mx - Nx rows
    // of the x pass's LDS slot that the zero-padded transform leaves unused.
    for (auto &h : p->h) {
        const int64_t Nx = h.g.n[0], cap = h.M[0] - Nx;
        std::vector<const int *> bx;
        for (int m = 1; m < h.n; ++m)
            if (!h.f[m - 1].identity) bx.push_back(reinterpret_cast<const int *>(host.data() + h.f[m - 1].off_b[0]));
        h.chunk = 0;
        if (bx.empty()) {
            h.chunk = (int)Nx;
            continue;
        }
        for (int64_t c = Nx; c >= 1 && !h.chunk; --c) {
            bool ok = true;
            for (int64_t i0 = 0; i0 < Nx && ok; i0 += c) {
                const int64_t i1 = i0 + c < Nx ? i0 + c : Nx;
                int64_t rows = 0;
                for (const int *b : bx) rows += b[i1 - 1] + K - b[i0];
                ok = rows <= cap;
            }
            if (ok) h.chunk = (int)c;
        }
    }
    // Source kernel: per field, the largest source block (SY x SZ) that a tile
    // of (SRC_TY source_rows) x SRC_TZ target columns touches; used when every
    // block fits the kernel's per-thread loads and z rows, its LDS fits 96 KiB
    // and every grid involved has fewer than 2^32 elements.
    const size_t rsize = csize(p->prec) / 2;
    for (auto &h : p->h) {
        const int64_t TY = NVP_SRC_TY * nvp::source_rows(rsize), TZ = NVP_SRC_TZ;
        bool small = true;  // 32-bit offsets
        for (int m = 1; m <= h.n; ++m) {
            const nvp_grid &gm = m == 1 ? p->g1 : p->h[m - 2].g;
            small = small && gm.n[0] * gm.n[1] * gm.n[2] < (int64_t(1) << 32);
        }
        int64_t msy = 0, mblk = 0;
        for (int m = 1; m < h.n; ++m) {
            if (h.f[m - 1].identity) continue;
            int64_t span[3] = {0, 0, 0};
            const int64_t T[3] = {1, TY, TZ};
            for (int ax = 1; ax < 3; ++ax) {
                const int *b = reinterpret_cast<const int *>(host.data() + h.f[m - 1].off_b[ax]);
                const int64_t n = h.g.n[ax];
                for (int64_t i0 = 0; i0 < n; i0 += T[ax]) {
                    const int64_t i1 = i0 + T[ax] < n ? i0 + T[ax] : n;
                    span[ax] = std::max(span[ax], (int64_t)b[i1 - 1] + K - b[i0]);
                }
            }
            msy = std::max(msy, span[1]);
            mblk = std::max(mblk, span[1] * span[2]);
        }
        const size_t lds = nvp::source_lds_bytes(h.n - 1, K, rsize);
        h.src_cx = source_chunk(h.g.n, rsize, 0, h.n - 1);
        const bool fits = nvp::source_wf(rsize) ? msy <= 16 && mblk <= 64 * NVP_SRC_PREW
                                     : msy <= 2 * TY && mblk <= nvp::source_pre(rsize) * NVP_SRC_TY * TZ;
        h.src_lds = small && fits && lds <= 98304 ? (int64_t)lds : 0;
    }
    *tbytes_out = tbytes;
    *maxA_out = maxA;
    *maxB_out = maxB;
    return NVP_OK;
}

nvp_status nvp_plan_cascade(nvp_ctx *ctx, const nvp_medium *med, double f0, int n_harm, const nvp_grid *g1,
                            const nvp_grid *gn, nvp_prec prec, int transfer_order, nvp_plan **out) {
    if (!ctx) return NVP_E_INVALID;
    if (!out) return fail(ctx, NVP_E_INVALID, "out is null");
    *out = nullptr;
    if (!medium_ok(med) || !finite_pos(f0) || !grid_ok(g1) || !gn || (prec != NVP_C64 && prec != NVP_C128))
        return fail(ctx, NVP_E_INVALID, "nvp_plan_cascade: bad argument");
    if (n_harm < 2 || n_harm > NVP_MAX_FIELDS + 1)
        return fail(ctx, n_harm < 2 ? NVP_E_INVALID : NVP_E_UNSUPPORTED, "nvp_plan_cascade: n_harm out of range");
    if (transfer_order != 1 && transfer_order != 3)
        return fail(ctx, NVP_E_UNSUPPORTED, "nvp_plan_cascade: transfer order must be 1 or 3");
    for (int i = 0; i < n_harm - 1; ++i)
        if (!grid_ok(&gn[i])) return fail(ctx, NVP_E_INVALID, "nvp_plan_cascade: bad harmonic grid");
    NVP_HIP(ctx, hipSetDevice(ctx->device));

    nvp_plan *p = new (std::nothrow) nvp_plan;
    if (!p) return fail(ctx, NVP_E_NOMEM, "plan allocation");
    p->ctx = ctx;
    p->quad = ctx->quad;
    p->prec = prec;
    p->order = transfer_order;
    p->med = *med;
    p->f0 = f0;
    p->n_harm = n_harm;
    p->g1 = *g1;
    p->h.resize(n_harm - 1);
    std::vector<unsigned char> host;
    size_t tbytes = 0, maxA = 0, maxB = 0;
    {
        nvp_status st = plan_layout(ctx, p, gn, host, &tbytes, &maxA, &maxB);
        if (st) {
            delete p;
            return st;
        }
    }
    hipError_t e = hipSuccess;
    if (tbytes) e = dev_malloc((void **)&p->tables, tbytes);
    if (e == hipSuccess) e = dev_malloc((void **)&p->A, maxA);
    if (e == hipSuccess) e = dev_malloc((void **)&p->B, maxB);
    for (auto &h : p->h) {
        if (e != hipSuccess) break;
        e = dev_malloc((void **)&h.khat, khat_bytes(h.M, prec));
        h.khat_cap = khat_bytes(h.M, prec);
        p->bytes_khat += h.khat_cap;
    }
    if (e == hipSuccess && tbytes) e = hipMemcpy(p->tables, host.data(), tbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_plan_memory(p);
        delete p;
        return hip_fail(ctx, "nvp_plan_cascade: allocation", e);
    }
    {
        const char *fs = getenv("NVP_FUSED_SOURCE");
        p->use_source_kernel = !(fs && atoi(fs) == 1);
    }
    p->bytes_A = maxA;
    p->bytes_B = maxB;
    p->bytes_tables = tbytes;
    ++ctx->users;
    *out = p;
    return NVP_OK;
}

nvp_status nvp_plan_regrid(nvp_plan *plan, int n, const nvp_grid *g) {
    if (!plan) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    if (n < 2 || n > plan->n_harm || !grid_ok(g)) return fail(ctx, NVP_E_INVALID, "nvp_plan_regrid: bad argument");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    // queued work of the plan may still read its tables and buffers
    NVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (plan->side) NVP_HIP(ctx, hipStreamSynchronize(plan->side));
    std::vector<nvp_grid> gn(plan->n_harm - 1);
    for (int i = 0; i < plan->n_harm - 1; ++i) gn[i] = plan->h[i].g;
    gn[n - 2] = *g;
    // lay out a copy first, so that a refused grid leaves the plan as it was
    nvp_plan q;
    q.ctx = ctx;
    q.order = plan->order;
    q.prec = plan->prec;
    q.med = plan->med;
    q.f0 = plan->f0;
    q.n_harm = plan->n_harm;
    q.g1 = plan->g1;
    q.h.resize(plan->n_harm - 1);
    std::vector<unsigned char> host;
    size_t tbytes = 0, maxA = 0, maxB = 0;
    nvp_status st = plan_layout(ctx, &q, gn.data(), host, &tbytes, &maxA, &maxB);
    if (st) return st;
    if (!plan->own_work && (maxA > plan->bytes_A || maxB > plan->bytes_B))
        return fail(ctx, NVP_E_INVALID, "nvp_plan_regrid: the caller workspace is too small for this grid");
    Harm &hn = q.h[n - 2];
    const size_t kb = khat_bytes(hn.M, plan->prec);
    // device memory that must grow
    void *tables = plan->tables, *khat = plan->h[n - 2].khat, *A = nullptr, *B = nullptr;
    hipError_t e = hipSuccess;
    if (tbytes > plan->bytes_tables) e = dev_malloc(&tables, tbytes);
    if (e == hipSuccess && kb > plan->h[n - 2].khat_cap) e = dev_malloc(&khat, kb);
    if (e == hipSuccess && plan->own_work && maxA > plan->bytes_A) e = dev_malloc(&A, maxA);
    if (e == hipSuccess && plan->own_work && maxB > plan->bytes_B) e = dev_malloc(&B, maxB);
    if (e == hipSuccess && tbytes) e = hipMemcpy(tables, host.data(), tbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (tables != plan->tables) (void)hipFree(tables);
        if (khat != plan->h[n - 2].khat) (void)hipFree(khat);
        if (A) (void)hipFree(A);
        if (B) (void)hipFree(B);
        return hip_fail(ctx, "nvp_plan_regrid: allocation", e);
    }
    if (tables != plan->tables) {
        (void)hipFree(plan->tables);
        plan->tables = tables;
        plan->bytes_tables = tbytes;
    }
    if (khat != plan->h[n - 2].khat) {
        (void)hipFree(plan->h[n - 2].khat);
        plan->bytes_khat += kb - plan->h[n - 2].khat_cap;
        plan->h[n - 2].khat = khat;
        plan->h[n - 2].khat_cap = kb;
    }
    if (A) {
        (void)hipFree(plan->A);
        plan->A = A;
        plan->bytes_A = maxA;
    }
    if (B) {
        (void)hipFree(plan->B);
        plan->B = B;
        plan->bytes_B = maxB;
    }
    // the side stream's scratch is sized for the grids: made again when next needed
    if (plan->own_work && plan->kscr) {
        size_t ks, kt;
        side_sizes(&q, &ks, &kt);
        if (ks + kt > plan->bytes_side) {
            (void)hipFree(plan->kscr);
            (void)hipFree(plan->ktab);
            plan->kscr = plan->ktab = nullptr;
            plan->bytes_side = 0;
        }
    }
    // every harmonic takes the new layout (later harmonics transfer from harmonic n's new grid);
    // harmonic n's spectrum and launch choices start afresh, the others keep theirs
    for (int i = 0; i < plan->n_harm - 1; ++i) {
        Harm &h = plan->h[i];
        const Harm &o = q.h[i];
        h.g = o.g;
        std::memcpy(h.M, o.M, sizeof h.M);
        h.kr = o.kr;
        h.ki = o.ki;
        h.Cn = o.Cn;
        h.chunk = o.chunk;
        h.src_lds = o.src_lds;
        h.src_cx = o.src_cx;
        std::memcpy(h.f, o.f, sizeof h.f);
        if (i == n - 2) {
            h.khat_ok = false;
            h.tune = Tune{};
        }
    }
    return NVP_OK;
}

nvp_status nvp_plan_workspace_bytes(const nvp_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return NVP_E_INVALID;
    *bytes = plan->bytes_tables + plan->bytes_khat;
    if (plan->own_work) *bytes += plan->bytes_A + plan->bytes_B + plan->bytes_side;
    return NVP_OK;
}

nvp_status nvp_plan_work_bytes(const nvp_plan *plan, size_t *bytes) {
    if (!plan || !bytes) return NVP_E_INVALID;
    size_t off[4];
    *bytes = work_layout(plan, off);
    return NVP_OK;
}

nvp_status nvp_plan_set_workspace(nvp_plan *plan, void *dev, size_t bytes) {
    if (!plan) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    size_t off[4];
    const size_t need = work_layout(plan, off);
    if (dev && bytes < need)
        return fail(ctx, NVP_E_INVALID, "nvp_plan_set_workspace: " + std::to_string(bytes) + " bytes, the plan needs " +
                                            std::to_string(need));
    if (dev && (reinterpret_cast<uintptr_t>(dev) & 255))
        return fail(ctx, NVP_E_INVALID, "nvp_plan_set_workspace: workspace not 256-byte aligned");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    // queued work of the plan may still use the current buffers
    NVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (plan->side) NVP_HIP(ctx, hipStreamSynchronize(plan->side));
    const size_t bA = plan->bytes_A, bB = plan->bytes_B;
    release_work(plan);
    if (dev) {
        char *w = static_cast<char *>(dev);
        plan->A = w + off[0];
        plan->B = w + off[1];
        plan->kscr = w + off[2];
        plan->ktab = w + off[3];
        plan->own_work = false;
        return NVP_OK;
    }
    hipError_t e = dev_malloc((void **)&plan->A, bA);
    if (e == hipSuccess) e = dev_malloc((void **)&plan->B, bB);
    if (e != hipSuccess) {
        if (plan->A) (void)hipFree(plan->A);
        plan->A = nullptr;
        return hip_fail(ctx, "nvp_plan_set_workspace: allocation", e);
    }
    return NVP_OK;
}

nvp_status nvp_plan_set_kernel_cache(nvp_plan *plan, int enable) {
    if (!plan) return NVP_E_INVALID;
    plan->cache = enable != 0;
    return NVP_OK;
}

nvp_status nvp_plan_set_overlap(nvp_plan *plan, int enable) {
    if (!plan) return NVP_E_INVALID;
    plan->overlap = enable != 0;
    return NVP_OK;
}

}  // extern "C"

namespace {

// Harmonic n with its kernel spectrum either computed here (kready null) or
// computed on the side stream, signalled by kready.
nvp_status run_harmonic(nvp_plan *plan, int n, const void *const *fields, void *pn_dev, hipEvent_t kready) {
    nvp_ctx *ctx = plan->ctx;
    Harm &h = plan->h[n - 2];
    nvp_status st;
    if (!kready && (!h.khat_ok || !plan->cache)) {
        if ((st = kernel_spectrum(ctx, plan, plan->quad, h.kr, h.ki, &h.g, h.M, plan->prec, h.khat, plan->B,
                                  plan->A)))
            return st;
        h.khat_ok = true;
    }
    SourceArgs src = source_args(plan, n, fields);
    const double scale = h.Cn / ((double)h.M[0] * (double)h.M[1] * (double)h.M[2]);
    const bool tiled_src = plan->use_source_kernel && h.tune.src != 0;
    return convolve(ctx, plan, plan->prec, &h.g, h.M, h.khat, plan->A, plan->B, nullptr, &src, pn_dev, scale,
                    tiled_src && h.src_lds > 0 ? src_cx_of(h) : 0, h.tune, kready);
}

// Side-stream resources of the overlapped spectra (created on first use).
nvp_status side_resources(nvp_plan *p) {
    nvp_ctx *ctx = p->ctx;
    if (!p->side) NVP_HIP(ctx, hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking));
    if (!p->ev_start) NVP_HIP(ctx, hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming));
    while ((int)p->ev_k.size() < p->n_harm - 1) {
        hipEvent_t e;
        NVP_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p->ev_k.push_back(e);
    }
    if (!p->kscr) {
        size_t ks, kt;
        side_sizes(p, &ks, &kt);
        NVP_HIP(ctx, dev_malloc((void **)&p->kscr, ks));
        hipError_t e = dev_malloc((void **)&p->ktab, kt);
        if (e != hipSuccess) {
            (void)hipFree(p->kscr);
            p->kscr = nullptr;
            return hip_fail(ctx, "side-stream scratch", e);
        }
        p->bytes_side = ks + kt;
    }
    return NVP_OK;
}

}  // namespace

extern "C" {

nvp_status nvp_execute_harmonic(nvp_plan *plan, int n, const void *const *fields, void *pn_dev) {
    if (!plan) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    if (n < 2 || n > plan->n_harm || !fields || !pn_dev)
        return fail(ctx, NVP_E_INVALID, "nvp_execute_harmonic: bad argument");
    for (int m = 1; m < n; ++m)
        if (!fields[m - 1] || fields[m - 1] == pn_dev)
            return fail(ctx, NVP_E_INVALID, "nvp_execute_harmonic: null or aliased field");
    if (!plan->A || !plan->B) return fail(ctx, NVP_E_STATE, "nvp_execute_harmonic: the plan has no work buffers");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    return run_harmonic(plan, n, fields, pn_dev, nullptr);
}

nvp_status nvp_execute_cascade(nvp_plan *plan, const void *p1_dev, void *const *pn_dev) {
    if (!plan) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    if (!p1_dev || !pn_dev) return fail(ctx, NVP_E_INVALID, "nvp_execute_cascade: null buffer");
    for (int n = 2; n <= plan->n_harm; ++n)
        if (!pn_dev[n - 2]) return fail(ctx, NVP_E_INVALID, "nvp_execute_cascade: null output");
        else if (pn_dev[n - 2] == p1_dev) return fail(ctx, NVP_E_INVALID, "nvp_execute_cascade: aliased output");
    if (!plan->A || !plan->B) return fail(ctx, NVP_E_STATE, "nvp_execute_cascade: the plan has no work buffers");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    bool need = false;
    for (auto &h : plan->h) need = need || !h.khat_ok || !plan->cache;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    NVP_HIP(ctx, hipStreamIsCapturing(ctx->stream, &cs));
    const bool ovl = plan->overlap && !plan->timing && need && cs == hipStreamCaptureStatusNone;
    if (ovl) {
        nvp_status st = side_resources(plan);
        if (st) return st;
    }
    std::vector<const void *> fields(plan->n_harm);
    fields[0] = p1_dev;
    for (int n = 2; n <= plan->n_harm; ++n) {
        Harm &h = plan->h[n - 2];
        hipEvent_t kready = nullptr;
        if (ovl && (!h.khat_ok || !plan->cache)) {
            // harmonic n's kernel spectrum on the side stream, from the moment the
            // context stream reaches harmonic n (after all its earlier work, which
            // may still read the spectrum), concurrently with the source build
            // and the forward x and y passes; the z pass waits for it
            NVP_HIP(ctx, hipEventRecord(plan->ev_start, ctx->stream));
            NVP_HIP(ctx, hipStreamWaitEvent(plan->side, plan->ev_start, 0));
            const hipStream_t user = ctx->stream;
            ctx->stream = plan->side;
            nvp_status st =
                kernel_spectrum(ctx, nullptr, plan->quad, h.kr, h.ki, &h.g, h.M, plan->prec, h.khat, plan->kscr,
                                plan->ktab);
            ctx->stream = user;
            if (st) return st;
            NVP_HIP(ctx, hipEventRecord(plan->ev_k[n - 2], plan->side));
            kready = plan->ev_k[n - 2];
            h.khat_ok = true;
        }
        nvp_status st = run_harmonic(plan, n, fields.data(), pn_dev[n - 2], kready);
        if (st) return st;
        fields[n - 1] = pn_dev[n - 2];
    }
    return NVP_OK;
}

nvp_status nvp_source_term(nvp_plan *plan, int n, const void *const *fields, void *f_dev) {
    if (!plan) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    if (n < 2 || n > plan->n_harm || !fields || !f_dev)
        return fail(ctx, NVP_E_INVALID, "nvp_source_term: bad argument");
    for (int m = 1; m < n; ++m)
        if (!fields[m - 1] || fields[m - 1] == f_dev)
            return fail(ctx, NVP_E_INVALID, "nvp_source_term: null or aliased field");
    const Harm &h = plan->h[n - 2];
    if (h.src_lds <= 0)
        return fail(ctx, NVP_E_UNSUPPORTED, "nvp_source_term: the source blocks of this grid pair do not fit the source kernel");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    const SourceArgs src = source_args(plan, n, fields);
    NVP_HIP(ctx, (plan->prec == NVP_C128 ? nvp::launch_source_c128 : nvp::launch_source_c64)(
                     src, f_dev, (int)h.g.n[1], src_cx_of(h), ctx->stream));
    return NVP_OK;
}

nvp_status nvp_plan_destroy(nvp_plan *plan) {
    if (!plan) return NVP_E_INVALID;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipStreamSynchronize(plan->ctx->stream);
    free_plan_memory(plan);
    --plan->ctx->users;
    delete plan;
    return NVP_OK;
}

nvp_status nvp_plan_set_timing(nvp_plan *plan, int enable) {
    if (!plan) return NVP_E_INVALID;
    plan->timing = enable != 0;
    return NVP_OK;
}

nvp_status nvp_plan_get_timing(nvp_plan *plan, double *ms, int64_t *count, int n_kinds) {
    if (!plan || !ms || !count || n_kinds < 1) return NVP_E_INVALID;
    nvp_ctx *ctx = plan->ctx;
    for (int k = 0; k < n_kinds; ++k) {
        ms[k] = 0;
        count[k] = 0;
    }
    for (auto &e : plan->events) {
        NVP_HIP(ctx, hipEventSynchronize(e.b));
        float t = 0;
        NVP_HIP(ctx, hipEventElapsedTime(&t, e.a, e.b));
        if (e.kind < n_kinds) {
            ms[e.kind] += t;
            count[e.kind] += 1;
        }
        plan->pool.push_back(e.a);
        plan->pool.push_back(e.b);
    }
    plan->events.clear();
    return NVP_OK;
}


// ------------------------------------------------------------------ autotuning

}  // extern "C"

namespace {

// Tuning-cache key of one harmonic: device, precision, transfer order and the
// shapes that decide the launches (target grid, circulant, source grids).
std::string tune_key(const nvp_plan *p, int n, const char *arch) {
    const Harm &h = p->h[n - 2];
    std::ostringstream k;
    k << arch << "|c" << (p->prec == NVP_C64 ? 64 : 128) << "|o" << p->order << "|N" << h.g.n[0] << "x" << h.g.n[1]
      << "x" << h.g.n[2] << "|M" << h.M[0] << "x" << h.M[1] << "x" << h.M[2] << "|S";
    for (int m = 1; m < n; ++m) {
        const nvp_grid &sg = m == 1 ? p->g1 : p->h[m - 2].g;
        k << (h.f[m - 1].identity ? "=" : "") << sg.n[0] << "x" << sg.n[1] << "x" << sg.n[2] << ";";
    }
    return k.str();
}

void read_tune_cache(const char *path, std::map<std::string, Tune> &out) {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        Tune t;
        if (ls >> key >> t.x_tile >> t.y_tile >> t.quads >> t.src) {
            if (!(ls >> t.src_cx) || t.src_cx < 0 || t.src_cx > NVP_SRC_CXM) t.src_cx = 0;  // older files: none
            out[key] = t;
        }
    }
}

bool write_tune_cache(const char *path, const std::map<std::string, Tune> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        if (!o) return false;
        for (const auto &kv : m)
            o << kv.first << " " << kv.second.x_tile << " " << kv.second.y_tile << " " << kv.second.quads << " "
              << kv.second.src << " " << kv.second.src_cx << "\n";
        if (!o) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

struct DevMem {
    std::vector<void *> p;
    ~DevMem() {
        for (void *q : p) (void)hipFree(q);
    }
};

// Times the launch choices of every harmonic of `plan` on zero-filled fields
// (the kernels have no data-dependent control flow) and keeps the fastest.
// Choices found in `cache` are taken without timing; new ones are added.
nvp_status autotune_plan(nvp_plan *plan, std::map<std::string, Tune> &cache, int reps) {
    nvp_ctx *ctx = plan->ctx;
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    NVP_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    const size_t cs = csize(plan->prec);
    DevMem mem;
    std::vector<const void *> fields(plan->n_harm);
    size_t out_elems = 1;
    for (int m = 1; m <= plan->n_harm; ++m) {
        const nvp_grid &g = m == 1 ? plan->g1 : plan->h[m - 2].g;
        const size_t elems = (size_t)g.n[0] * g.n[1] * g.n[2];
        if (m == plan->n_harm) {
            out_elems = std::max(out_elems, elems);
            break;
        }
        void *q = nullptr;
        NVP_HIP(ctx, dev_malloc((void **)&q, elems * cs));
        mem.p.push_back(q);
        NVP_HIP(ctx, hipMemsetAsync(q, 0, elems * cs, ctx->stream));
        fields[m - 1] = q;
        if (m >= 2) out_elems = std::max(out_elems, elems);
    }
    void *out = nullptr;
    NVP_HIP(ctx, dev_malloc((void **)&out, out_elems * cs));
    mem.p.push_back(out);
    hipEvent_t e0, e1;
    NVP_HIP(ctx, hipEventCreate(&e0));
    NVP_HIP(ctx, hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    const bool timing = plan->timing;
    plan->timing = false;
    nvp_status st = NVP_OK;
    for (int n = 2; n <= plan->n_harm && st == NVP_OK; ++n) {
        Harm &h = plan->h[n - 2];
        const std::string key = tune_key(plan, n, prop.gcnArchName);
        auto it = cache.find(key);
        if (it != cache.end()) {
            h.tune = it->second;
            continue;
        }
        float best = 1e30f;
        Tune best_t{};
        // one choice: a warm-up run, then reps timed runs
        auto try_choice = [&](const Tune &t) {
            h.tune = t;
            if ((st = nvp_execute_harmonic(plan, n, fields.data(), out))) return;
            if (hipEventRecord(e0, ctx->stream) != hipSuccess) {
                st = NVP_E_HIP;
                return;
            }
            for (int r = 0; r < reps && st == NVP_OK; ++r) st = nvp_execute_harmonic(plan, n, fields.data(), out);
            if (st) return;
            float ms = 0;
            if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = hip_fail(ctx, "autotune timing", hipGetLastError());
                return;
            }
            if (ms < best) {
                best = ms;
                best_t = t;
            }
        };
        const int src_opts = (plan->use_source_kernel && h.src_lds > 0) ? 2 : 1;
        for (int xt = 0; xt < 2 && st == NVP_OK; ++xt)
            for (int yt = 0; yt < 2 && st == NVP_OK; ++yt)
                for (int q = 1; q <= 2 && st == NVP_OK; ++q)
                    for (int so = 0; so < src_opts && st == NVP_OK; ++so) {
                        Tune t;
                        t.x_tile = xt;
                        t.y_tile = yt;
                        t.quads = q;
                        t.src = src_opts == 2 ? 1 - so : 0;
                        try_choice(t);
                    }
        // then, with the source kernel chosen, its x chunk: chunks for about a half
        // and twice the default number of workgroups
        if (st == NVP_OK && best_t.src == 1) {
            const Tune base = best_t;
            for (int64_t want : {(int64_t)1024, (int64_t)4096}) {
                Tune t = base;
                const size_t rs = csize(plan->prec) / 2;
                t.src_cx = source_chunk(h.g.n, rs, nvp::source_wf(rs) ? want * 4 / std::max(1, h.n - 1) : want,
                                        h.n - 1);
                if (t.src_cx != h.src_cx && st == NVP_OK) try_choice(t);
            }
        }
        h.tune = best_t;
        cache[key] = best_t;
    }
    plan->timing = timing;
    if (st == NVP_OK) NVP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return st;
}

}  // namespace

// ------------------------------------------------------------------ batches

struct nvp_batch {
    nvp_ctx *ctx = nullptr;
    std::vector<nvp_plan *> plans;
    std::vector<int64_t> off;  // first output slot of each problem
    int64_t n_out = 0;
    bool graph = true;
    int branches = 4;
    hipStream_t cap = nullptr;       // stream the graph is recorded from (the context stream may be the null stream)
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // fork, then one join event per branch
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    std::vector<const void *> cap_in;
    std::vector<void *> cap_out;
    bool warm = false;
    bool grouped = false;        // multi-task launches per pass and transform length
    void *tasks = nullptr;       // device task tables of the grouped schedule
    size_t tasks_bytes = 0;
};

namespace {

void drop_graph(nvp_batch *b) {
    if (b->ge) (void)hipGraphExecDestroy(b->ge);
    if (b->g) (void)hipGraphDestroy(b->g);
    b->ge = nullptr;
    b->g = nullptr;
    b->cap_in.clear();
    b->cap_out.clear();
}

void free_batch(nvp_batch *b) {
    drop_graph(b);
    if (b->tasks) (void)hipFree(b->tasks);
    b->tasks = nullptr;
    for (auto *p : b->plans) nvp_plan_destroy(p);
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->cap = nullptr;
    for (auto e : b->events) (void)hipEventDestroy(e);
    b->plans.clear();
    b->streams.clear();
    b->events.clear();
}

nvp_status run_eager(nvp_batch *b, const void *const *p1, void *const *pn) {
    for (size_t i = 0; i < b->plans.size(); ++i) {
        nvp_status st = nvp_execute_cascade(b->plans[i], p1[i], pn + b->off[i]);
        if (st) return st;
    }
    return NVP_OK;
}

// ------------------------------------------------------------------ grouped schedule

// One step of the grouped schedule: a problem's source build or whole
// harmonic, or one multi-task launch of a pass over the problems whose
// transform length along that pass's axis is L.
struct GroupStep {
    int kind = 0;  // 0 source build, 1 strided pass, 2 z pass, 3 whole harmonic (fused source path)
    int problem = 0, n = 0;
    int L = 0, sign = 0, scaled = 0;
    int ntasks = 0;
    int64_t blocks = 0;
    size_t offset = 0;  // byte offset of the step's tasks in the task buffer
};

// The pass kinds of one harmonic, in launch order.
enum { P_XFWD, P_YFWD, P_ZCONV, P_YINV, P_XINV };

// Builds the grouped schedule for the given buffers and uploads its task
// tables.  Level by level (harmonic n of every problem that has it): the
// source builds, then each pass as one launch per transform length.
nvp_status build_grouped(nvp_batch *b, const void *const *p1, void *const *pn, std::vector<GroupStep> &steps) {
    nvp_ctx *ctx = b->ctx;
    const bool dbl = b->plans[0]->prec == NVP_C128;
    int maxn = 0;
    for (auto *p : b->plans) maxn = std::max(maxn, p->n_harm);
    std::vector<unsigned char> host;
    auto push = [&](const void *data, size_t bytes) {
        const size_t o = (host.size() + 255) & ~(size_t)255;
        host.resize(o + bytes);
        std::memcpy(host.data() + o, data, bytes);
        return o;
    };
    for (int n = 2; n <= maxn; ++n) {
        std::vector<int> act;
        for (int i = 0; i < (int)b->plans.size(); ++i) {
            nvp_plan *p = b->plans[i];
            if (n > p->n_harm) continue;
            if (!p->use_source_kernel || p->h[n - 2].src_lds <= 0 || p->h[n - 2].tune.src == 0) {
                GroupStep g;
                g.kind = 3;
                g.problem = i;
                g.n = n;
                steps.push_back(g);
                continue;
            }
            act.push_back(i);
            GroupStep g;
            g.kind = 0;
            g.problem = i;
            g.n = n;
            steps.push_back(g);
        }
        for (int pass = P_XFWD; pass <= P_XINV; ++pass) {
            std::map<int, std::vector<int>> by_len;
            for (int i : act) {
                const Harm &h = b->plans[i]->h[n - 2];
                const int L = (int)(pass == P_XFWD || pass == P_XINV ? h.M[0] : pass == P_ZCONV ? h.M[2] : h.M[1]);
                by_len[L].push_back(i);
            }
            for (auto &kv : by_len) {
                const int L = kv.first;
                GroupStep g;
                g.L = L;
                g.ntasks = (int)kv.second.size();
                if (pass == P_ZCONV) {
                    g.kind = 2;
                    const int slots = nvp::zconv_slots_per_block(L, dbl);
                    std::vector<nvp::ZconvTaskArgs> t;
                    for (int i : kv.second) {
                        nvp_plan *p = b->plans[i];
                        const Harm &h = p->h[n - 2];
                        nvp::ZconvTaskArgs a{};
                        a.buf = p->B;
                        a.khat = h.khat;
                        a.Mx = h.M[0];
                        a.My = h.M[1];
                        a.Hy = h.M[1] / 2 + 1;
                        a.n_quads = (h.M[0] / 2 + 1) * a.Hy;
                        a.Nz = (int)h.g.n[2];
                        a.first = g.blocks;
                        g.blocks += (4 * a.n_quads + slots - 1) / slots;
                        t.push_back(a);
                    }
                    g.offset = push(t.data(), t.size() * sizeof(t[0]));
                } else {
                    g.kind = 1;
                    g.sign = pass <= P_YFWD ? -1 : 1;
                    g.scaled = pass == P_XINV;
                    const int T = nvp::strided_tile_cols(L, dbl);
                    std::vector<nvp::StridedTaskArgs> t;
                    for (int i : kv.second) {
                        nvp_plan *p = b->plans[i];
                        const Harm &h = p->h[n - 2];
                        const int64_t Nx = h.g.n[0], Ny = h.g.n[1], Nz = h.g.n[2];
                        const int64_t Mx = h.M[0], My = h.M[1];
                        nvp::StridedTaskArgs a{};
                        int64_t outer = 1;
                        a.scale = 1.0;
                        if (pass == P_XFWD) {
                            a.in = p->A; a.in_os = 0; a.in_ms = Ny * Nz; a.n_in = (int)Nx;
                            a.out = p->A; a.out_os = 0; a.out_ms = Ny * Nz; a.n_out = (int)Mx;
                            a.inner = Ny * Nz;
                        } else if (pass == P_YFWD) {
                            a.in = p->A; a.in_os = Ny * Nz; a.in_ms = Nz; a.n_in = (int)Ny;
                            a.out = p->B; a.out_os = My * Nz; a.out_ms = Nz; a.n_out = (int)My;
                            a.inner = Nz;
                            outer = Mx;
                        } else if (pass == P_YINV) {
                            a.in = p->B; a.in_os = My * Nz; a.in_ms = Nz; a.n_in = (int)My;
                            a.out = p->A; a.out_os = Ny * Nz; a.out_ms = Nz; a.n_out = (int)Ny;
                            a.inner = Nz;
                            outer = Mx;
                        } else {
                            a.in = p->A; a.in_os = 0; a.in_ms = Ny * Nz; a.n_in = (int)Mx;
                            a.out = pn[b->off[i] + n - 2]; a.out_os = 0; a.out_ms = Ny * Nz; a.n_out = (int)Nx;
                            a.scale = h.Cn / ((double)h.M[0] * (double)h.M[1] * (double)h.M[2]);
                            a.inner = Ny * Nz;
                        }
                        a.tiles = (a.inner + T - 1) / T;
                        a.first = g.blocks;
                        g.blocks += a.tiles * outer;
                        t.push_back(a);
                    }
                    g.offset = push(t.data(), t.size() * sizeof(t[0]));
                }
                if (g.blocks > 0x7fffffff) return fail(ctx, NVP_E_UNSUPPORTED, "grouped pass exceeds the grid limit");
                steps.push_back(g);
            }
        }
    }
    (void)p1;
    if (b->tasks && b->tasks_bytes < host.size()) {
        (void)hipFree(b->tasks);
        b->tasks = nullptr;
    }
    if (!b->tasks && !host.empty()) {
        NVP_HIP(ctx, dev_malloc((void **)&b->tasks, host.size()));
        b->tasks_bytes = host.size();
    }
    if (!host.empty()) NVP_HIP(ctx, hipMemcpy(b->tasks, host.data(), host.size(), hipMemcpyHostToDevice));
    return NVP_OK;
}

// Issues the grouped schedule on the context stream.
nvp_status run_grouped(nvp_batch *b, const std::vector<GroupStep> &steps, const void *const *p1, void *const *pn) {
    nvp_ctx *ctx = b->ctx;
    const bool dbl = b->plans[0]->prec == NVP_C128;
    const unsigned char *tb = static_cast<const unsigned char *>(b->tasks);
    for (const GroupStep &g : steps) {
        if (g.kind == 0 || g.kind == 3) {
            nvp_plan *p = b->plans[g.problem];
            std::vector<const void *> fields(g.n - 1);
            fields[0] = p1[g.problem];
            for (int m = 2; m < g.n; ++m) fields[m - 1] = pn[b->off[g.problem] + m - 2];
            if (g.kind == 3) {
                nvp_status st = nvp_execute_harmonic(p, g.n, fields.data(), pn[b->off[g.problem] + g.n - 2]);
                if (st) return st;
                continue;
            }
            const Harm &h = p->h[g.n - 2];
            const SourceArgs src = source_args(p, g.n, fields.data());
            NVP_HIP(ctx, (dbl ? nvp::launch_source_c128 : nvp::launch_source_c64)(src, p->A, (int)h.g.n[1], src_cx_of(h),
                                                                                ctx->stream));
            continue;
        }
        const void *tw;
        nvp_status st = twiddles(ctx, g.L, dbl, &tw);
        if (st) return st;
        if (g.kind == 1) {
            const auto *t = reinterpret_cast<const nvp::StridedTaskArgs *>(tb + g.offset);
            NVP_HIP(ctx, (dbl ? nvp::launch_strided_multi_c128 : nvp::launch_strided_multi_c64)(
                             g.L, t, g.ntasks, g.blocks, g.sign, g.scaled, tw, ctx->stream));
        } else {
            const auto *t = reinterpret_cast<const nvp::ZconvTaskArgs *>(tb + g.offset);
            NVP_HIP(ctx, (dbl ? nvp::launch_zconv_multi_c128 : nvp::launch_zconv_multi_c64)(g.L, t, g.ntasks, g.blocks,
                                                                                          tw, ctx->stream));
        }
    }
    return NVP_OK;
}

// Records every problem's cascade into one graph: problem i on branch
// i mod branches, each branch a stream forked from and joined back into the
// recording stream, so independent problems may run concurrently.
nvp_status capture_grouped(nvp_batch *b, const void *const *p1, void *const *pn);

nvp_status capture(nvp_batch *b, const void *const *p1, void *const *pn) {
    nvp_ctx *ctx = b->ctx;
    if (!b->cap) NVP_HIP(ctx, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    if (b->grouped) return capture_grouped(b, p1, pn);
    const int S = std::min<int>(b->branches, (int)b->plans.size());
    while ((int)b->streams.size() < S) {
        hipStream_t s;
        NVP_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->streams.push_back(s);
    }
    while ((int)b->events.size() < S + 1) {
        hipEvent_t e;
        NVP_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->events.push_back(e);
    }
    const hipStream_t user = ctx->stream, origin = b->cap;
    NVP_HIP(ctx, hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    nvp_status st = NVP_OK;
    hipError_t e = hipEventRecord(b->events[0], origin);
    for (int s = 0; s < S && e == hipSuccess; ++s) e = hipStreamWaitEvent(b->streams[s], b->events[0], 0);
    if (e != hipSuccess) st = hip_fail(ctx, "batch capture fork", e);
    for (size_t i = 0; i < b->plans.size() && st == NVP_OK; ++i) {
        ctx->stream = b->streams[i % S];
        st = nvp_execute_cascade(b->plans[i], p1[i], pn + b->off[i]);
        ctx->stream = user;
    }
    for (int s = 0; s < S && st == NVP_OK; ++s) {
        e = hipEventRecord(b->events[s + 1], b->streams[s]);
        if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->events[s + 1], 0);
        if (e != hipSuccess) st = hip_fail(ctx, "batch capture join", e);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(origin, &g);
    if (st == NVP_OK && e != hipSuccess) st = hip_fail(ctx, "hipStreamEndCapture", e);
    if (st != NVP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(ctx, "hipGraphInstantiate", e);
    }
    b->g = g;
    b->ge = ge;
    b->cap_in.assign(p1, p1 + b->plans.size());
    b->cap_out.assign(pn, pn + b->n_out);
    return NVP_OK;
}

// The grouped schedule recorded as one graph on the recording stream.
nvp_status capture_grouped(nvp_batch *b, const void *const *p1, void *const *pn) {
    nvp_ctx *ctx = b->ctx;
    std::vector<GroupStep> steps;
    nvp_status st = build_grouped(b, p1, pn, steps);
    if (st) return st;
    const hipStream_t user = ctx->stream;
    NVP_HIP(ctx, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    ctx->stream = b->cap;
    st = run_grouped(b, steps, p1, pn);
    ctx->stream = user;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (st == NVP_OK && e != hipSuccess) st = hip_fail(ctx, "hipStreamEndCapture", e);
    if (st != NVP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(ctx, "hipGraphInstantiate", e);
    }
    b->g = g;
    b->ge = ge;
    b->cap_in.assign(p1, p1 + b->plans.size());
    b->cap_out.assign(pn, pn + b->n_out);
    return NVP_OK;
}

}  // namespace

extern "C" {

nvp_status nvp_batch_set_grouped(nvp_batch *b, int enable) {
    if (!b) return NVP_E_INVALID;
    if ((enable != 0) != b->grouped) drop_graph(b);
    b->grouped = enable != 0;
    return NVP_OK;
}

nvp_status nvp_plan_autotune(nvp_plan *plan, const char *cache_path, int reps) {
    if (!plan) return NVP_E_INVALID;
    if (reps < 1 || reps > 100) return fail(plan->ctx, NVP_E_INVALID, "nvp_plan_autotune: reps out of range");
    std::map<std::string, Tune> cache;
    if (cache_path) read_tune_cache(cache_path, cache);
    nvp_status st = autotune_plan(plan, cache, reps);
    if (st == NVP_OK && cache_path && !write_tune_cache(cache_path, cache))
        return fail(plan->ctx, NVP_E_INVALID, std::string("nvp_plan_autotune: cannot write ") + cache_path);
    return st;
}

nvp_status nvp_plan_get_tuning(const nvp_plan *plan, int n, int *choice) {
    if (!plan || !choice || n < 2 || n > plan->n_harm) return NVP_E_INVALID;
    const Tune &t = plan->h[n - 2].tune;
    choice[0] = t.x_tile;
    choice[1] = t.y_tile;
    choice[2] = t.quads;
    choice[3] = t.src;
    choice[4] = t.src_cx;
    return NVP_OK;
}

nvp_status nvp_plan_set_tuning(nvp_plan *plan, int n, const int *choice) {
    if (!plan) return NVP_E_INVALID;
    if (!choice || n < 2 || n > plan->n_harm) return fail(plan->ctx, NVP_E_INVALID, "nvp_plan_set_tuning: bad argument");
    Tune t;
    t.x_tile = choice[0];
    t.y_tile = choice[1];
    t.quads = choice[2];
    t.src = choice[3];
    t.src_cx = choice[4];
    if ((t.x_tile | t.y_tile) & ~1 || t.quads < 0 || t.quads > 2 || t.src < -1 || t.src > 1 || t.src_cx < 0 ||
        t.src_cx > NVP_SRC_CXM)
        return fail(plan->ctx, NVP_E_INVALID, "nvp_plan_set_tuning: a choice out of range");
    if (t.src == 1 && (!plan->use_source_kernel || plan->h[n - 2].src_lds <= 0))
        return fail(plan->ctx, NVP_E_UNSUPPORTED,
                    "nvp_plan_set_tuning: the source kernel does not take this harmonic's grids");
    plan->h[n - 2].tune = t;
    return NVP_OK;
}

nvp_status nvp_batch_create(nvp_ctx *ctx, int count, const nvp_problem *problems, nvp_prec prec, int transfer_order,
                            nvp_batch **out) {
    if (!ctx) return NVP_E_INVALID;
    if (!out || !problems || count < 1) return fail(ctx, NVP_E_INVALID, "nvp_batch_create: bad argument");
    *out = nullptr;
    nvp_batch *b = new (std::nothrow) nvp_batch;
    if (!b) return fail(ctx, NVP_E_NOMEM, "batch allocation");
    b->ctx = ctx;
    for (int i = 0; i < count; ++i) {
        const nvp_problem &pr = problems[i];
        nvp_plan *p = nullptr;
        nvp_status st = nvp_plan_cascade(ctx, &pr.med, pr.f0, pr.n_harm, &pr.g1, pr.gn, prec, transfer_order, &p);
        if (st) {
            const std::string msg = "problem " + std::to_string(i) + ": " + ctx->err;
            free_batch(b);
            delete b;
            return fail(ctx, st, msg);
        }
        p->overlap = false;  // a batch overlaps whole problems on its own streams
        b->plans.push_back(p);
        b->off.push_back(b->n_out);
        b->n_out += pr.n_harm - 1;
    }
    ++ctx->users;
    *out = b;
    return NVP_OK;
}

nvp_status nvp_batch_outputs(const nvp_batch *b, int64_t *n_out) {
    if (!b || !n_out) return NVP_E_INVALID;
    *n_out = b->n_out;
    return NVP_OK;
}

nvp_status nvp_batch_set_graph(nvp_batch *b, int enable, int branches) {
    if (!b) return NVP_E_INVALID;
    if (branches < 1 || branches > 16) return fail(b->ctx, NVP_E_INVALID, "nvp_batch_set_graph: branches not in 1..16");
    if ((enable != 0) != b->graph || branches != b->branches) drop_graph(b);
    b->graph = enable != 0;
    b->branches = branches;
    return NVP_OK;
}

nvp_status nvp_batch_autotune(nvp_batch *b, const char *cache_path, int reps) {
    if (!b) return NVP_E_INVALID;
    if (reps < 1 || reps > 100) return fail(b->ctx, NVP_E_INVALID, "nvp_batch_autotune: reps out of range");
    std::map<std::string, Tune> cache;
    if (cache_path) read_tune_cache(cache_path, cache);
    for (auto *p : b->plans) {
        nvp_status st = autotune_plan(p, cache, reps);
        if (st) return st;
    }
    drop_graph(b);  // launch choices changed
    if (cache_path && !write_tune_cache(cache_path, cache))
        return fail(b->ctx, NVP_E_INVALID, std::string("nvp_batch_autotune: cannot write ") + cache_path);
    return NVP_OK;
}

nvp_status nvp_batch_execute(nvp_batch *b, const void *const *p1_dev, void *const *pn_dev) {
    if (!b) return NVP_E_INVALID;
    nvp_ctx *ctx = b->ctx;
    if (!p1_dev || !pn_dev) return fail(ctx, NVP_E_INVALID, "nvp_batch_execute: null buffer list");
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (!p1_dev[i]) return fail(ctx, NVP_E_INVALID, "nvp_batch_execute: null p1");
    for (int64_t i = 0; i < b->n_out; ++i)
        if (!pn_dev[i]) return fail(ctx, NVP_E_INVALID, "nvp_batch_execute: null output");
    NVP_HIP(ctx, hipSetDevice(ctx->device));
    if (!b->warm || (!b->graph && !b->grouped)) {
        // eager: also the first run of a graph or grouped batch, which computes and
        // caches every kernel spectrum and twiddle table so that later runs hold the
        // convolutions only
        nvp_status st = run_eager(b, p1_dev, pn_dev);
        if (st) return st;
        for (auto *p : b->plans)
            for (auto &h : p->h)
                if (!h.khat_ok || !p->cache) return NVP_OK;  // kernel cache off: stay eager
        b->warm = true;
        return NVP_OK;
    }
    if (!b->graph) {
        // grouped launches without a graph
        std::vector<GroupStep> steps;
        nvp_status st = build_grouped(b, p1_dev, pn_dev, steps);
        if (st) return st;
        return run_grouped(b, steps, p1_dev, pn_dev);
    }
    const bool same = b->ge && std::equal(b->cap_in.begin(), b->cap_in.end(), p1_dev) &&
                      std::equal(b->cap_out.begin(), b->cap_out.end(), pn_dev);
    if (!same) {
        drop_graph(b);
        nvp_status st = capture(b, p1_dev, pn_dev);
        if (st) return st;
    }
    NVP_HIP(ctx, hipGraphLaunch(b->ge, ctx->stream));
    return NVP_OK;
}

nvp_status nvp_batch_destroy(nvp_batch *b) {
    if (!b) return NVP_E_INVALID;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    free_batch(b);
    --b->ctx->users;
    delete b;
    return NVP_OK;
}

}  // extern "C"
