// Host emulation of the Stockham FFT engine (paper_2011_03009_amd/csrc/fft_core.hpp).
//
// The engine's own code is compiled for the host: each lane of a column is a
// host thread, a barrier over them stands in for __syncthreads and for the
// wave-local wave_sync, and the LDS is a host array.  Every transform length
// NVP_HOST_L runs, in FP64 and FP32, the ways the library's kernels use the
// engine, each compared with a direct DFT in long double:
//   fwd   forward transform of a column whose upper half is zero (x and y passes);
//   inv   inverse transform keeping the lower half (x and y inverse passes);
//   conv  forward transform kept in registers, a spectral product, and the
//         inverse in reverse radix order, through a padded pencil slot (z pass);
//   even  forward transform of an even sequence read from its first L/2+1
//         entries, exchanged through one real plane (FP64 kernel spectrum);
//   cols  the forward transform of three interleaved columns sharing one LDS
//         array (the strided passes' layout).
// Every load and store index is checked against the column, every output must
// be written exactly once, and the harness is built with AddressSanitizer so
// that an engine register or LDS index beyond its array aborts.
// Prints "OK <L>" or a diagnostic, and exits non-zero on failure.
#define NVP_HOST_EMULATION 1
#include <barrier>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <random>
#include <thread>
#include <vector>

#include "hip/hip_runtime.h"

static thread_local std::barrier<> *tl_bar = nullptr;
void __syncthreads() { tl_bar->arrive_and_wait(); }
namespace nvp {
inline void wave_sync() { tl_bar->arrive_and_wait(); }
}  // namespace nvp

#include "fft_core.hpp"

#ifndef NVP_HOST_L
#error "compile with -DNVP_HOST_L=<transform length>"
#endif

using namespace nvp;
using cld = std::complex<long double>;

static int g_fail = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");      \
            std::abort();                    \
        }                                    \
    } while (0)

// The library's twiddle table of length L (forward-order stages, then the
// reversed order), built by the same rule as the runtime: extended precision,
// rounded once.
template <typename R> std::vector<cx<R>> twiddle_table(int L) {
    std::vector<cx<R>> t;
    for (int rev = 0; rev < 2; ++rev)
        for (int st = 1; st < plan_for(L).S; ++st) {
            const int Ns = plan_ns(L, rev, st), r = plan_rad(L, rev, st);
            for (int j = 0; j < Ns; ++j)
                for (int q = 1; q < r; ++q) {
                    const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)(j * q) /
                                          (long double)(Ns * r);
                    cx<R> w;
                    w.x = (R)(double)cosl(a);
                    w.y = (R)(double)-sinl(a);
                    t.push_back(w);
                }
        }
    CHECK((int)t.size() == twiddle_table_len(L), "twiddle table length %zu != %d", t.size(), twiddle_table_len(L));
    return t;
}

// y_k = sum_m x_m exp(sg 2 pi i k m / L), long double
std::vector<cld> dft(const std::vector<cld> &x, int sg) {
    const int L = (int)x.size();
    std::vector<cld> w(L), y(L);
    for (int j = 0; j < L; ++j) {
        const long double a = 2.0L * 3.141592653589793238462643383279502884L * j / L;
        w[j] = cld(cosl(a), sg * sinl(a));
    }
    for (int k = 0; k < L; ++k) {
        cld s = 0;
        for (int m = 0; m < L; ++m) s += x[m] * w[(int64_t)k * m % L];
        y[k] = s;
    }
    return y;
}

template <typename R> cld C(cx<R> v) { return cld(v.x, v.y); }
template <typename R> cx<R> X(cld v) {
    cx<R> r;
    r.x = (R)v.real();
    r.y = (R)v.imag();
    return r;
}

// relative L2 error of got[m] against ref[m] over m in [0, n)
long double rel_err(const std::vector<cld> &got, const std::vector<cld> &ref, int n) {
    long double e = 0, s = 0;
    for (int m = 0; m < n; ++m) {
        e += std::norm(got[m] - ref[m]);
        s += std::norm(ref[m]);
    }
    return sqrtl(e / (s > 0 ? s : 1));
}

// Runs body(t) on `threads` host threads that share one barrier.
void lanes(int threads, const std::function<void(int)> &body) {
    std::barrier<> bar(threads);
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t)
        th.emplace_back([&, t] {
            tl_bar = &bar;
            body(t);
        });
    for (auto &x : th) x.join();
}

template <typename R> std::vector<cld> random_column(int L, int n, unsigned seed) {
    std::mt19937_64 g(seed);
    std::normal_distribution<double> d;
    std::vector<cld> x(L, cld(0));
    for (int m = 0; m < n; ++m) x[m] = C<R>(X<R>(cld(d(g), d(g))));  // representable in R
    return x;
}

template <typename R> struct Checker {
    static constexpr int L = NVP_HOST_L;
    const long double tol = sizeof(R) == 8 ? 1e-12L : 2e-6L;
    std::vector<cx<R>> tw = twiddle_table<R>(L);

    void report(const char *what, long double e) {
        if (!(e < tol)) {
            std::fprintf(stderr, "FAIL L=%d %s %s rel err %.3Le\n", L, sizeof(R) == 8 ? "f64" : "f32", what, e);
            ++g_fail;
        }
    }

    // forward, upper half zero, plain column-layout LDS (one column)
    void fwd() {
        using F = Fft<R, L>;
        auto x = random_column<R>(L, L / 2, 1);
        std::vector<cx<R>> lds(L), out(L);
        std::vector<int> writes(L, 0);
        lanes(F::P, [&](int t) {
            F::template run<-1, false, true, false>(
                t, [&](int e) { return tw[e]; },
                [&](int m) {
                    CHECK(m >= 0 && m < L, "fwd load %d", m);
                    return X<R>(x[m]);
                },
                [&](int m, cx<R> v) {
                    CHECK(m >= 0 && m < L, "fwd store %d", m);
                    out[m] = v;
                    __atomic_add_fetch(&writes[m], 1, __ATOMIC_RELAXED);
                },
                [&](int m) -> cx<R> & {
                    CHECK(m >= 0 && m < L, "fwd lds %d", m);
                    return lds[m];
                });
        });
        for (int m = 0; m < L; ++m) CHECK(writes[m] == 1, "fwd output %d written %d times", m, writes[m]);
        std::vector<cld> got(L);
        for (int m = 0; m < L; ++m) got[m] = C<R>(out[m]);
        report("fwd", rel_err(got, dft(x, -1), L));
    }

    // inverse, only the lower half kept
    void inv() {
        using F = Fft<R, L>;
        auto x = random_column<R>(L, L, 2);
        std::vector<cx<R>> lds(L), out(L);
        std::vector<int> writes(L, 0);
        lanes(F::P, [&](int t) {
            F::template run<1, false, false, true>(
                t, [&](int e) { return tw[e]; }, [&](int m) { return X<R>(x[m]); },
                [&](int m, cx<R> v) {
                    CHECK(m >= 0 && m < L, "inv store %d", m);
                    out[m] = v;
                    __atomic_add_fetch(&writes[m], 1, __ATOMIC_RELAXED);
                },
                [&](int m) -> cx<R> & {
                    CHECK(m >= 0 && m < L, "inv lds %d", m);
                    return lds[m];
                });
        });
        for (int m = 0; m < L / 2; ++m) CHECK(writes[m] == 1, "inv output %d written %d times", m, writes[m]);
        for (int m = L / 2; m < L; ++m) CHECK(writes[m] <= 1, "inv output %d written %d times", m, writes[m]);
        std::vector<cld> got(L);
        for (int m = 0; m < L; ++m) got[m] = C<R>(out[m]);
        report("inv", rel_err(got, dft(x, 1), L / 2));
    }

    // the z pass: forward kept in registers, product, reverse-order inverse
    void conv() {
        constexpr bool WL = wave_local<R>(L);
        using F = Fft<R, L, false, WL>;
        using G = Fft<R, L, true, WL>;
        auto x = random_column<R>(L, L / 2, 3);
        auto k = random_column<R>(L, L, 4);
        std::vector<cx<R>> slot(pencil_pad<R>(L) + 1), out(L);
        std::vector<int> writes(L, 0);
        lanes(F::P, [&](int t) {
            const PencilSlot<R> ref{slot.data()};
            cx<R> v[F::E];
            F::template load0<true>(v, t, [&](int m) {
                CHECK(m >= 0 && m < L / 2 + L / plan_for(L).r[0], "conv load %d", m);
                return X<R>(x[m]);
            });
            auto twf = [&](int e) { return tw[e]; };
            F::template compute_keep<-1, true>(v, t, twf, ref);
            for (int i = 0; i < F::EOUT; ++i)
                if (F::out_valid(t, i)) {
                    const int m = F::out_index(t, i);
                    CHECK(m >= 0 && m < L, "conv spectrum index %d", m);
                    v[i] = cmul<R>(v[i], X<R>(k[m]));
                }
            G::template compute<1, false, true>(v, t, twf,
                                                [&](int m, cx<R> y) {
                                                    CHECK(m >= 0 && m < L, "conv store %d", m);
                                                    out[m] = y;
                                                    __atomic_add_fetch(&writes[m], 1, __ATOMIC_RELAXED);
                                                },
                                                ref);
        });
        for (int m = 0; m < L / 2; ++m) CHECK(writes[m] == 1, "conv output %d written %d times", m, writes[m]);
        auto X_ = dft(x, -1);
        for (int m = 0; m < L; ++m) X_[m] *= k[m];
        auto y = dft(X_, 1);
        std::vector<cld> got(L);
        for (int m = 0; m < L; ++m) got[m] = C<R>(out[m]);
        report("conv", rel_err(got, y, L / 2));
    }

    // even sequence from its first L/2+1 entries, real-plane exchange (FP64 passes)
    void even() {
        using F = Fft<R, L>;
        auto h = random_column<R>(L, L / 2 + 1, 5);
        std::vector<cld> x(L);
        for (int m = 0; m < L; ++m) x[m] = h[m <= L / 2 ? m : L - m];
        std::vector<R> plane(L);
        std::vector<cx<R>> out(L);
        std::vector<int> writes(L, 0);
        lanes(F::P, [&](int t) {
            F::template run<-1, false>(
                t, [&](int e) { return tw[e]; },
                [&](int m) {
                    CHECK(m >= 0 && m < L, "even load %d", m);
                    return X<R>(h[m <= L / 2 ? m : L - m]);
                },
                [&](int m, cx<R> v) {
                    CHECK(m >= 0 && m < L, "even store %d", m);
                    out[m] = v;
                    __atomic_add_fetch(&writes[m], 1, __ATOMIC_RELAXED);
                },
                SplitCols<R, 1>{plane.data(), 0});
        });
        for (int m = 0; m < L; ++m) CHECK(writes[m] == 1, "even output %d written %d times", m, writes[m]);
        std::vector<cld> got(L);
        for (int m = 0; m < L; ++m) got[m] = C<R>(out[m]);
        report("even", rel_err(got, dft(x, -1), L));
    }

    // The FP64 kernel-spectrum passes as the kernels run them.  kz: one
    // octant row per pencil, its L/2+1 entries gathered into the padded
    // pencil slot, the transform reading its first stage from that same slot
    // (wave-local where the column fits a wavefront).  mirror: T columns whose
    // L/2+1 entries are staged as complex values, column-interleaved, in the
    // LDS array that the transform then reuses as one real plane per exchange.
    void kz() {
        constexpr int PK = sizeof(R) == 8 ? kz_threads(L) : col_threads<R>(L);
        constexpr bool WL = wave_local_p(PK);
        using F = Fft<R, L, false, WL, PK>;
        auto h = random_column<R>(L, L / 2 + 1, 6);
        std::vector<cld> x(L);
        for (int m = 0; m < L; ++m) x[m] = h[m <= L / 2 ? m : L - m];
        std::vector<cx<R>> slot(pencil_pad<R>(L) + 1), out(L / 2 + 1);
        lanes(F::P, [&](int t) {
            for (int k = t; k <= L / 2; k += F::P) slot[pencil_pad<R>(k)] = X<R>(h[k]);
            if (WL) wave_sync();
            else __syncthreads();
            F::template run<-1, true>(
                t, [&](int e) { return tw[e]; },
                [&](int m) {
                    CHECK(m >= 0 && m < L, "kz load %d", m);
                    return slot[pencil_pad<R>(m <= L / 2 ? m : L - m)];
                },
                [&](int m, cx<R> v) {
                    if (m <= L / 2) out[m] = v;
                },
                PencilSlot<R>{slot.data()});
        });
        std::vector<cld> got(L / 2 + 1);
        for (int m = 0; m <= L / 2; ++m) got[m] = C<R>(out[m]);
        report("kz", rel_err(got, dft(x, -1), L / 2 + 1));
    }

    template <int T> void mirror() {
        using F = Fft<R, L>;
        std::vector<std::vector<cld>> h, x;
        for (int c = 0; c < T; ++c) {
            h.push_back(random_column<R>(L, L / 2 + 1, 20 + c));
            std::vector<cld> e(L);
            for (int m = 0; m < L; ++m) e[m] = h[c][m <= L / 2 ? m : L - m];
            x.push_back(e);
        }
        const size_t a = (size_t)T * L * sizeof(R), b = (size_t)T * (L / 2 + 1) * sizeof(cx<R>);
        std::vector<unsigned char> mem(a > b ? a : b);
        cx<R> *lds = reinterpret_cast<cx<R> *>(mem.data());
        std::vector<std::vector<cx<R>>> out(T, std::vector<cx<R>>(L));
        lanes(T * F::P, [&](int tid) {
            const int c = tid % T, t = tid / T;
            for (int m = t; m <= L / 2; m += F::P) lds[(size_t)m * T + c] = X<R>(h[c][m]);
            __syncthreads();
            F::template run<-1, true>(
                t, [&](int e) { return tw[e]; },
                [&](int m) {
                    CHECK(m >= 0 && m < L, "mirror load %d", m);
                    return lds[(size_t)(m <= L / 2 ? m : L - m) * T + c];
                },
                [&](int m, cx<R> v) { out[c][m] = v; }, SplitCols<R, T>{reinterpret_cast<R *>(mem.data()), c});
        });
        for (int c = 0; c < T; ++c) {
            std::vector<cld> got(L);
            for (int m = 0; m < L; ++m) got[m] = C<R>(out[c][m]);
            report("mirror", rel_err(got, dft(x[c], -1), L));
        }
    }

    // three interleaved columns sharing one LDS array (lds[m T + c])
    void cols() {
        using F = Fft<R, L>;
        constexpr int T = 3;
        std::vector<std::vector<cld>> x;
        for (int c = 0; c < T; ++c) x.push_back(random_column<R>(L, L / 2, 10 + c));
        std::vector<cx<R>> lds((size_t)T * L);
        std::vector<std::vector<cx<R>>> out(T, std::vector<cx<R>>(L));
        lanes(T * F::P, [&](int tid) {
            const int c = tid % T, t = tid / T;
            F::template run<-1, false, true, false>(
                t, [&](int e) { return tw[e]; }, [&](int m) { return X<R>(x[c][m]); },
                [&](int m, cx<R> v) { out[c][m] = v; },
                [&](int m) -> cx<R> & {
                    CHECK(m >= 0 && m < L, "cols lds %d", m);
                    return lds[(size_t)m * T + c];
                });
        });
        for (int c = 0; c < T; ++c) {
            std::vector<cld> got(L);
            for (int m = 0; m < L; ++m) got[m] = C<R>(out[c][m]);
            report("cols", rel_err(got, dft(x[c], -1), L));
        }
    }
};

int main() {
    {
        Checker<double> c;
        c.fwd();
        c.inv();
        c.conv();
        c.even();
        c.kz();
        c.mirror<4>();
        c.cols();
    }
    {
        Checker<float> c;
        c.fwd();
        c.inv();
        c.conv();
        c.cols();
    }
    if (g_fail) return 1;
    std::printf("OK %d P=%d E=%d (FP64: P=%d E=%d; FP64 octant rows: P=%d E=%d)\n", NVP_HOST_L,
                Fft<float, NVP_HOST_L>::P, Fft<float, NVP_HOST_L>::E, Fft<double, NVP_HOST_L>::P,
                Fft<double, NVP_HOST_L>::E, kz_threads(NVP_HOST_L),
                Fft<double, NVP_HOST_L, false, false, kz_threads(NVP_HOST_L)>::E);
    return 0;
}
