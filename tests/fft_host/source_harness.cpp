// Host emulation of the source kernels: the streamed one
// (paper_2011_03009_amd/csrc/source.hpp) and the one with a wavefront per
// field (source_wf.hpp).
//
// The kernel body is compiled for the host: every workgroup of the launch
// grid runs as host threads, one per work item, sharing a barrier (for
// __syncthreads), one barrier per 64 of them (for wave_sync) and
// an LDS array of exactly the size the launch gives it, filled with NaN so
// that a read of an entry not written before it is seen.  Random monotone axis
// tables (source planes advancing by 0, 1 or 2 per target voxel, clamped at
// both ends, as interpolation onto finer, equal or coarser grids makes them),
// random weights, fields on the target grid among them, ragged tiles in y and
// z and ragged x chunks, one or two target rows per thread of the streamed
// kernel, in FP32 and FP64,
// for K = 2 and 4 and 1 to 4 and 7
// fields.  Each output is compared with the separable transfer and the
// source product summed directly in long double, and must be written.  Built
// with AddressSanitizer: an index outside a field, a table, the output or the
// LDS aborts.  Prints "OK <cases>" or a diagnostic, and exits non-zero on
// failure.
#define NVP_HOST_EMULATION 1
#include <array>
#include <barrier>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <limits>
#include <memory>
#include <random>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

static thread_local std::barrier<> *tl_bar = nullptr;       // the workgroup's threads
static thread_local std::barrier<> *tl_wave_bar = nullptr;  // the wavefront's 64 threads
void __syncthreads() { tl_bar->arrive_and_wait(); }
namespace nvp {
inline void wave_sync() { tl_wave_bar->arrive_and_wait(); }
}  // namespace nvp

#include "source.hpp"
#include "source_wf.hpp"

using namespace nvp;
using cld = std::complex<long double>;

constexpr int TY = 8, TZ = 32, CXM = 16;  // threads along y and z; the largest x chunk

#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");        \
            std::abort();                      \
        }                                      \
    } while (0)

// 64-byte aligned storage, so that a voxel's K weights can be read as one aligned vector
template <typename T> struct Buf {
    T *p = nullptr;
    size_t n = 0;
    explicit Buf(size_t n_) : n(n_) {
        const size_t bytes = ((n * sizeof(T) + 63) / 64) * 64;
        p = static_cast<T *>(std::aligned_alloc(64, bytes ? bytes : 64));
    }
    Buf(const Buf &) = delete;
    Buf(Buf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; }
    ~Buf() { std::free(p); }
    T &operator[](size_t i) { return p[i]; }
};

// a non-decreasing table of base indices for n_t targets into n_s sources
std::vector<int> monotone_table(std::mt19937_64 &g, int n_t, int n_s, int K, double p0, double p2) {
    std::uniform_real_distribution<double> u(0, 1);
    std::vector<int> b(n_t);
    int v = (int)(u(g) * (n_s - K + 1));
    for (int i = 0; i < n_t; ++i) {
        const double x = u(g);
        if (i) v += x < p0 ? 0 : x < 1 - p2 ? 1 : 2;
        b[i] = std::min(std::max(v, 0), n_s - K);
    }
    return b;
}

// WF: the kernel with one wavefront per field (k_source_wf; PRE is its block
// entries per lane over 64 lanes); else the streamed kernel with RY rows per thread.
template <typename R, int K, int NF, int RY, int PRE, bool WF = false> struct Case {
    static constexpr int TYT = WF ? 8 : RY * TY;  // target rows of a tile
    static constexpr int NTH = WF ? NF * 64 : TY * TZ;  // threads of a workgroup
    int N[3];
    std::vector<int> identity;
    std::vector<std::array<int, 3>> ns;
    std::vector<Buf<cx<R>>> p;
    std::vector<std::array<std::vector<int>, 3>> b;
    std::vector<std::array<Buf<R> *, 3>> w;
    std::vector<Buf<R>> wstore;

    bool run(std::mt19937_64 &g, int cx_len, double p0, double p2, long double tol) {
        std::uniform_int_distribution<int> pick(0, 3);
        std::normal_distribution<double> nd;
        LdSource<R, K> src{};
        src.nf = NF;
        src.Nx = N[0];
        src.Nz = N[2];
        wstore.reserve(3 * NF);
        for (int i = 0; i < NF; ++i) {
            const bool id = pick(g) == 0;
            identity.push_back(id);
            std::array<int, 3> n{};
            std::array<std::vector<int>, 3> bi;
            for (int ax = 0; ax < 3; ++ax) {
                if (id) {
                    n[ax] = N[ax];
                    continue;
                }
                n[ax] = std::max(K, (int)(N[ax] * (1.0 - p0 + p2)) + 3);
                bi[ax] = monotone_table(g, N[ax], n[ax], K, p0, p2);
            }
            ns.push_back(n);
            b.push_back(bi);
            Buf<cx<R>> f((size_t)n[0] * n[1] * n[2]);
            for (size_t e = 0; e < f.n; ++e) {
                f[e].x = (R)nd(g);
                f[e].y = (R)nd(g);
            }
            p.push_back(std::move(f));
        }
        w.resize(NF);
        for (int i = 0; i < NF; ++i) {
            FieldDev<R> &d = src.f[i];
            d.p = p[i].p;
            d.s0 = (int64_t)ns[i][1] * ns[i][2];
            d.s1 = ns[i][2];
            d.identity = identity[i];
            for (int ax = 0; ax < 3; ++ax) {
                if (identity[i]) {
                    d.b[ax] = nullptr;
                    d.w[ax] = nullptr;
                    continue;
                }
                wstore.emplace_back((size_t)N[ax] * K);
                Buf<R> &ww = wstore.back();
                for (size_t e = 0; e < ww.n; ++e) ww[e] = (R)nd(g);
                w[i][ax] = &ww;
                d.b[ax] = b[i][ax].data();
                d.w[ax] = ww.p;
            }
        }
        // launch geometry, as the host chooses it
        int msy = 0, mblk = 0;
        for (int i = 0; i < NF; ++i) {
            if (identity[i]) continue;
            int sy = 0, sz = 0;
            for (int i0 = 0; i0 < N[1]; i0 += TYT) sy = std::max(sy, b[i][1][std::min(i0 + TYT, N[1]) - 1] + K - b[i][1][i0]);
            for (int i0 = 0; i0 < N[2]; i0 += TZ) sz = std::max(sz, b[i][2][std::min(i0 + TZ, N[2]) - 1] + K - b[i][2][i0]);
            msy = std::max(msy, sy);
            mblk = std::max(mblk, sy * sz);
        }
        // beyond the kernel's limits the host takes the fused path
        if (WF ? (msy > 16 || mblk > 64 * PRE) : (msy > 2 * TYT || mblk > PRE * TY * TZ)) return false;
        CHECK(cx_len <= CXM, "chunk %d beyond %d", cx_len, CXM);
        Buf<cx<R>> out((size_t)N[0] * N[1] * N[2]);
        const R nan = std::numeric_limits<R>::quiet_NaN();
        for (size_t e = 0; e < out.n; ++e) out[e].x = out[e].y = nan;
        const int gz = (N[2] + TZ - 1) / TZ, gy = (N[1] + TYT - 1) / TYT, gx = (N[0] + cx_len - 1) / cx_len;
        const size_t lds_n = WF ? SrcWfLds<R, K, NF, PRE, CXM>::BYTES : SrcLds<R, K, NF, TY, TZ, RY, PRE, CXM>::BYTES;
        for (int bx = 0; bx < gx; ++bx)
            for (int by = 0; by < gy; ++by)
                for (int bz = 0; bz < gz; ++bz) {
                    // NaN in every real and int of the LDS: a read before its write shows
                    Buf<unsigned char> lds(lds_n);
                    for (size_t e = 0; e < lds_n; ++e) lds[e] = 0xff;
                    std::barrier<> bar(NTH);
                    std::vector<std::unique_ptr<std::barrier<>>> wbar;
                    for (int v = 0; v < (NTH + 63) / 64; ++v) wbar.emplace_back(new std::barrier<>(64));
                    std::vector<std::thread> th;
                    for (int t = 0; t < NTH; ++t)
                        th.emplace_back([&, t] {
                            tl_bar = &bar;
                            tl_wave_bar = wbar[t / 64].get();
                            if constexpr (WF)
                                source_tile_wf<R, K, NF, PRE, CXM>(src, out.p, N[1], cx_len, lds.p, t, bz, by, bx);
                            else
                                source_tile<R, K, NF, TY, TZ, RY, PRE, CXM>(src, out.p, N[1], cx_len, lds.p, t, bz,
                                                                            by, bx);
                        });
                    for (auto &x : th) x.join();
                }
        // reference
        long double err = 0, ref2 = 0;
        for (int ix = 0; ix < N[0]; ++ix)
            for (int iy = 0; iy < N[1]; ++iy)
                for (int iz = 0; iz < N[2]; ++iz) {
                    const int idx[3] = {ix, iy, iz};
                    cld v[NF];
                    for (int i = 0; i < NF; ++i) {
                        const auto &n = ns[i];
                        if (identity[i]) {
                            const cx<R> e = p[i][((size_t)ix * n[1] + iy) * n[2] + iz];
                            v[i] = cld(e.x, e.y);
                            continue;
                        }
                        cld acc = 0;
                        for (int a = 0; a < K; ++a)
                            for (int c = 0; c < K; ++c)
                                for (int d = 0; d < K; ++d) {
                                    const int s[3] = {b[i][0][ix] + a, b[i][1][iy] + c, b[i][2][iz] + d};
                                    const cx<R> e = p[i][((size_t)s[0] * n[1] + s[1]) * n[2] + s[2]];
                                    const long double wt = (long double)(*w[i][0])[(size_t)idx[0] * K + a] *
                                                           (long double)(*w[i][1])[(size_t)idx[1] * K + c] *
                                                           (long double)(*w[i][2])[(size_t)idx[2] * K + d];
                                    acc += wt * cld(e.x, e.y);
                                }
                        v[i] = acc;
                    }
                    cld f = 0;
                    for (int a = 0; a < NF; ++a) f += v[a] * v[NF - 1 - a];
                    const cx<R> o = out[((size_t)ix * N[1] + iy) * N[2] + iz];
                    CHECK(!std::isnan((double)o.x) && !std::isnan((double)o.y),
                          "output (%d,%d,%d) not written (or NaN) N=%d,%d,%d NF=%d K=%d cx=%d", ix, iy, iz, N[0],
                          N[1], N[2], NF, K, cx_len);
                    err += std::norm(cld(o.x, o.y) - f);
                    ref2 += std::norm(f);
                }
        const long double rel = sqrtl(err / (ref2 > 0 ? ref2 : 1));
        CHECK(rel < tol, "FAIL %s K=%d NF=%d N=%d,%d,%d cx=%d p0=%.2f p2=%.2f rel err %.3Le",
              sizeof(R) == 8 ? "f64" : "f32", K, NF, N[0], N[1], N[2], cx_len, p0, p2, rel);
        return true;
    }
};

template <typename R, int K, int NF, int RY = 1, int PRE = 2, bool WF = false> int cases(unsigned seed) {
    std::mt19937_64 g(seed);
    const long double tol = sizeof(R) == 8 ? 1e-12L : 1e-5L;
    // (Nx, Ny, Nz, x chunk, P(no advance), P(advance by 2))
    struct Shape {
        int nx, ny, nz, cx;
        double p0, p2;
    };
    const Shape shapes[] = {
        {9, 17, 45, 4, 0.2, 0.0},   // coarser source grids (ratio 4/5), ragged tiles
        {12, 8, 32, 12, 0.8, 0.0},  // much coarser (ratio 1/5), whole tiles, one chunk
        {7, 13, 70, 3, 0.0, 0.0},   // equal spacing
        {10, 9, 33, 5, 0.1, 0.1},   // a little finer in places
        {5, 3, 5, 2, 0.5, 0.0},     // smaller than one tile
    };
    int ran = 0;
    for (const Shape &s : shapes) {
        Case<R, K, NF, RY, PRE, WF> c;
        c.N[0] = s.nx;
        c.N[1] = s.ny;
        c.N[2] = s.nz;
        ran += c.run(g, s.cx, s.p0, s.p2, tol) ? 1 : 0;
    }
    return ran;
}

int main() {
    int n = 0;
    n += cases<float, 4, 1>(1);
    n += cases<float, 4, 2>(2);
    n += cases<float, 4, 3>(3);
    n += cases<float, 4, 4>(4);
    n += cases<float, 4, 7>(5);
    n += cases<float, 2, 3>(6);
    n += cases<double, 4, 4>(7);
    n += cases<double, 2, 2>(8);
    n += cases<double, 4, 7>(9);
    // two target rows per thread
    n += cases<float, 4, 1, 2, 3>(11);
    n += cases<float, 4, 4, 2, 3>(12);
    n += cases<float, 2, 3, 2, 3>(13);
    n += cases<double, 4, 3, 2, 3>(14);
    // one wavefront per field
    n += cases<float, 4, 1, 1, 7, true>(21);
    n += cases<float, 4, 2, 1, 7, true>(22);
    n += cases<float, 4, 3, 1, 7, true>(23);
    n += cases<float, 4, 4, 1, 7, true>(24);
    n += cases<float, 4, 7, 1, 7, true>(25);
    n += cases<float, 2, 3, 1, 7, true>(26);
    n += cases<double, 4, 4, 1, 7, true>(27);
    n += cases<double, 2, 2, 1, 7, true>(28);
    CHECK(n >= 100, "only %d cases fit the kernel's limits", n);
    std::printf("OK %d\n", n);
    return 0;
}
