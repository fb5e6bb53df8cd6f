// Stockham autosort mixed-radix FFT engine for gfx950 (64-wide wavefronts).
//
// One column of length L is transformed by P threads.  Stage s (radix r_s,
// Ns = r_0 ... r_{s-1}) has L / r_s butterflies; thread t does butterflies
// b = t + i P, i < ceil(L / (r_s P)) (the last one only where b < L / r_s),
// holding their r_s values each in registers.  Butterfly b
// reads its inputs at b + q L / r_s, twiddles input q by
// W^(j q L / (Ns r_s)) with j = b mod Ns and W = exp(-+ 2 pi i / L), does a
// radix-r_s DFT, and writes output p to (b / Ns) Ns r_s + j + p Ns.  That
// ordering is self-sorting: the last stage writes natural order, so its
// outputs go straight to global memory (or to a fused consumer), and the first
// stage reads straight from global memory (or from a fused producer).  Only
// the stages in between exchange data through LDS.
//
// Forward transforms use sign -1 (X_k = sum x_m e^{-2 pi i k m / L}), inverse
// +1, unnormalised; the sign is a compile-time parameter, so rotations by +-i
// and conjugated twiddles cost no instructions.  Twiddles come from per-stage
// tables [j][q-1] = exp(-2 pi i j q / (Ns r)) computed on the host in extended
// precision and rounded once; every access is a per-thread base plus a
// constant offset.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nvp {

template <typename R> struct cx_sel;
template <> struct cx_sel<float> { using type = float2; };
template <> struct cx_sel<double> { using type = double2; };
template <typename R> using cx = typename cx_sel<R>::type;

template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { cx<R> r; r.x = a; r.y = b; return r; }
template <typename R> __device__ __forceinline__ cx<R> czero() { return mk<R>(R(0), R(0)); }
template <typename R> __device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R> __device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename R> __device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }
// a * conj(b)
template <typename R> __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
    return mk<R>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// SG * i * a, SG = +-1 at compile time
template <int SG, typename R> __device__ __forceinline__ cx<R> crot(cx<R> a) {
    if constexpr (SG > 0) return mk<R>(-a.y, a.x);
    else return mk<R>(a.y, -a.x);
}
// a * (c + SG i s) for constants c, s
template <int SG, typename R> __device__ __forceinline__ cx<R> cmulk(cx<R> a, R c, R s) {
    return SG > 0 ? mk<R>(a.x * c - a.y * s, a.x * s + a.y * c) : mk<R>(a.x * c + a.y * s, a.y * c - a.x * s);
}

// ---------------------------------------------------------------- small DFTs
// y_p = sum_q v_q exp(SG 2 pi i p q / N), in place on v[0..N-1].

template <int N, typename R> struct Dft;

// run_lo<SG, K>: the same transform when only v[0..K-1] may be nonzero (the
// rest are taken as zero, whatever they hold), so no work is spent on them.

template <typename R> struct Dft<2, R> {
    template <int SG> static __device__ __forceinline__ void run(cx<R> *v) {
        cx<R> a = v[0], b = v[1];
        v[0] = cadd<R>(a, b);
        v[1] = csub<R>(a, b);
    }
    template <int SG, int K> static __device__ __forceinline__ void run_lo(cx<R> *v) {
        static_assert(K >= 1, "at least one nonzero input");
        if constexpr (K >= 2) run<SG>(v);
        else v[1] = v[0];
    }
};

template <typename R> struct Dft<4, R> {
    template <int SG> static __device__ __forceinline__ void run(cx<R> *v) {
        cx<R> a = cadd<R>(v[0], v[2]), b = csub<R>(v[0], v[2]);
        cx<R> c = cadd<R>(v[1], v[3]), d = crot<SG, R>(csub<R>(v[1], v[3]));
        v[0] = cadd<R>(a, c);
        v[2] = csub<R>(a, c);
        v[1] = cadd<R>(b, d);
        v[3] = csub<R>(b, d);
    }
    template <int SG, int K> static __device__ __forceinline__ void run_lo(cx<R> *v) {
        static_assert(K >= 1, "at least one nonzero input");
        if constexpr (K >= 4) {
            run<SG>(v);
        } else {
            const cx<R> a = K >= 3 ? cadd<R>(v[0], v[2]) : v[0], b = K >= 3 ? csub<R>(v[0], v[2]) : v[0];
            const cx<R> c = K >= 2 ? v[1] : czero<R>(), d = crot<SG, R>(c);
            if constexpr (K >= 2) {
                v[0] = cadd<R>(a, c);
                v[2] = csub<R>(a, c);
                v[1] = cadd<R>(b, d);
                v[3] = csub<R>(b, d);
            } else {
                v[1] = v[2] = v[3] = v[0];
            }
        }
    }
};

// Even/odd split: y_p = E_p + W^p O_p, y_{p+N/2} = E_p - W^p O_p.
template <typename R> struct Dft<8, R> {
    template <int SG> static __device__ __forceinline__ void run(cx<R> *v) { run_lo<SG, 8>(v); }
    template <int SG, int K> static __device__ __forceinline__ void run_lo(cx<R> *v) {
        cx<R> e[4] = {v[0], v[2], v[4], v[6]};
        cx<R> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, R>::template run_lo<SG, (K + 1) / 2>(e);
        Dft<4, R>::template run_lo<SG, K / 2>(o);
        const R c = R(0.707106781186547524400844362105);
        // W^1 = c (1 + SG i), W^3 = c (-1 + SG i)
        o[1] = SG > 0 ? mk<R>(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                      : mk<R>(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
        o[2] = crot<SG, R>(o[2]);
        o[3] = SG > 0 ? mk<R>(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                      : mk<R>(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            v[p] = cadd<R>(e[p], o[p]);
            v[p + 4] = csub<R>(e[p], o[p]);
        }
    }
};

template <typename R> struct Dft<16, R> {
    template <int SG> static __device__ __forceinline__ void run(cx<R> *v) { run_lo<SG, 16>(v); }
    template <int SG, int K> static __device__ __forceinline__ void run_lo(cx<R> *v) {
        cx<R> e[8], o[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<8, R>::template run_lo<SG, (K + 1) / 2>(e);
        Dft<8, R>::template run_lo<SG, K / 2>(o);
        const R c1 = R(0.923879532511286756128183189397);  // cos(pi/8)
        const R s1 = R(0.382683432365089771728459984030);  // sin(pi/8)
        const R c2 = R(0.707106781186547524400844362105);
        o[1] = cmulk<SG, R>(o[1], c1, s1);
        o[2] = SG > 0 ? mk<R>(c2 * (o[2].x - o[2].y), c2 * (o[2].x + o[2].y))
                      : mk<R>(c2 * (o[2].x + o[2].y), c2 * (o[2].y - o[2].x));
        o[3] = cmulk<SG, R>(o[3], s1, c1);
        o[4] = crot<SG, R>(o[4]);
        o[5] = cmulk<SG, R>(o[5], -s1, c1);
        o[6] = SG > 0 ? mk<R>(-c2 * (o[6].x + o[6].y), c2 * (o[6].x - o[6].y))
                      : mk<R>(c2 * (o[6].y - o[6].x), -c2 * (o[6].x + o[6].y));
        o[7] = cmulk<SG, R>(o[7], -c1, s1);
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            v[p] = cadd<R>(e[p], o[p]);
            v[p + 8] = csub<R>(e[p], o[p]);
        }
    }
};

// cos and sin of 2 pi k / N for k = 1..(N-1)/2 (N = 3, 5, 7, 9).
__host__ __device__ constexpr double odd_cos(int N, int k) {
    return N == 3 ? -0.5
         : N == 5 ? (k == 1 ? 0.309016994374947424102293417183 : -0.809016994374947424102293417183)
         : N == 7 ? (k == 1 ? 0.623489801858733530525004884004
                     : k == 2 ? -0.222520933956314404288902564497 : -0.900968867902419126236102319507)
         : (k == 1 ? 0.766044443118978035202392650555 : k == 2 ? 0.173648177666930348851716626769
            : k == 3 ? -0.5 : -0.939692620785908384054109277325);
}
__host__ __device__ constexpr double odd_sin(int N, int k) {
    return N == 3 ? 0.866025403784438646763723170753
         : N == 5 ? (k == 1 ? 0.951056516295153572116439333379 : 0.587785252292473129168705954639)
         : N == 7 ? (k == 1 ? 0.781831482468029808708444526674
                     : k == 2 ? 0.974927912181823607018131682994 : 0.433883739117558120475768332849)
         : (k == 1 ? 0.642787609686539326322643409907 : k == 2 ? 0.984807753012208059366743024590
            : k == 3 ? 0.866025403784438646763723170753 : 0.342020143325668733044099614682);
}

// Odd N (any, prime or not): pair v_q with v_{N-q}:  y_p = v_0 + sum_q a_q cos(2 pi p q / N) +- SG i sum_q b_q sin(...).
template <int N, typename R> struct DftOdd {
    template <int SG> static __device__ __forceinline__ void run(cx<R> *v) { run_lo<SG, N>(v); }
    template <int SG, int K> static __device__ __forceinline__ void run_lo(cx<R> *v) {
        static_assert(K > (N - 1) / 2, "inputs 1..(N-1)/2 are taken as nonzero");
        constexpr int H = (N - 1) / 2;
        cx<R> a[H], b[H];
        cx<R> y0 = v[0];
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            if (N - q < K) {
                a[q - 1] = cadd<R>(v[q], v[N - q]);
                b[q - 1] = csub<R>(v[q], v[N - q]);
            } else {
                a[q - 1] = b[q - 1] = v[q];
            }
            y0 = cadd<R>(y0, a[q - 1]);
        }
        cx<R> out[N];
#pragma unroll
        for (int p = 1; p <= H; ++p) {
            cx<R> A = v[0], B = czero<R>();
#pragma unroll
            for (int q = 1; q <= H; ++q) {
                const int idx = (p * q) % N;  // 0 where N is not prime (N = 9: p q = 3 * 3)
                const R cv = R(idx == 0 ? 1.0 : idx <= H ? odd_cos(N, idx) : odd_cos(N, N - idx));
                const R sv = R(idx == 0 ? 0.0 : idx <= H ? odd_sin(N, idx) : -odd_sin(N, N - idx));
                A = cadd<R>(A, cscale<R>(a[q - 1], cv));
                B = cadd<R>(B, cscale<R>(b[q - 1], sv));
            }
            cx<R> iB = crot<SG, R>(B);
            out[p] = cadd<R>(A, iB);
            out[N - p] = csub<R>(A, iB);
        }
        v[0] = y0;
#pragma unroll
        for (int p = 1; p < N; ++p) v[p] = out[p];
    }
};
template <typename R> struct Dft<3, R> : DftOdd<3, R> {};
template <typename R> struct Dft<5, R> : DftOdd<5, R> {};
template <typename R> struct Dft<7, R> : DftOdd<7, R> {};
template <typename R> struct Dft<9, R> : DftOdd<9, R> {};

// ---------------------------------------------------------------- octant layout

// Row stride (entries) of the kernel-spectrum octant [Mx/2+1][My/2+1][*] along
// z: Mz/2+1 rounded up to 16, so that every row starts on a 128-byte line in
// complex64 and a 256-byte boundary in complex128.
__host__ __device__ constexpr int64_t octant_row(int64_t Mz) { return (Mz / 2 + 1 + 15) / 16 * 16; }

// ---------------------------------------------------------------- plans

struct PlanDesc {
    int S;        // number of stages
    int r[6];     // radix of each stage
    int P;        // threads per column
    int P64 = 0;  // threads per column in FP64, where it differs from P
};

// Radix plans of the supported lengths.  The first stage reads global memory
// directly and the last writes it, so fewer stages mean fewer LDS round trips.
// A large even first radix prunes most: a forward input's upper half is zero,
// so half of that stage's butterfly inputs are, and the reversed (inverse)
// plan's last stage computes only the lower half.  (Orders measured at 640,
// 768 and 896 points: 8,4,4,5, 8,8,4,3 and 8,7,4,4 were the fastest tried.)
// A column's threads split each stage's butterflies as evenly as they can;
// where L / r is not a multiple of P, some threads of that stage have one
// butterfly fewer.  P is a power of two up to 64 where that keeps the
// registers per thread (the largest butterfly share times its radix) at 48
// complex values or fewer, so that the contiguous axis can run a column in
// one wavefront.
__host__ __device__ constexpr PlanDesc plan_for(int L) {
    switch (L) {
    case 16: return PlanDesc{1, {16, 0, 0, 0, 0, 0}, 1};
    case 32: return PlanDesc{2, {2, 16, 0, 0, 0, 0}, 2};
    case 48: return PlanDesc{3, {3, 4, 4, 0, 0, 0}, 4};
    case 64: return PlanDesc{2, {4, 16, 0, 0, 0, 0}, 4};
    case 80: return PlanDesc{3, {4, 4, 5, 0, 0, 0}, 4};
    case 96: return PlanDesc{3, {3, 4, 8, 0, 0, 0}, 4};
    case 112: return PlanDesc{3, {7, 4, 4, 0, 0, 0}, 4};
    case 128: return PlanDesc{2, {8, 16, 0, 0, 0, 0}, 8};
    case 144: return PlanDesc{3, {4, 9, 4, 0, 0, 0}, 4};
    case 160: return PlanDesc{3, {5, 4, 8, 0, 0, 0}, 4};
    case 192: return PlanDesc{3, {3, 8, 8, 0, 0, 0}, 8};
    case 224: return PlanDesc{3, {16, 7, 2, 0, 0, 0}, 8};
    case 256: return PlanDesc{2, {16, 16, 0, 0, 0, 0}, 16};
    case 288: return PlanDesc{3, {8, 9, 4, 0, 0, 0}, 16};
    case 320: return PlanDesc{3, {5, 8, 8, 0, 0, 0}, 8};
    case 336: return PlanDesc{3, {16, 7, 3, 0, 0, 0}, 16};
    case 360: return PlanDesc{3, {8, 9, 5, 0, 0, 0}, 16};
    case 384: return PlanDesc{4, {3, 8, 4, 4, 0, 0}, 16};
    case 432: return PlanDesc{3, {16, 9, 3, 0, 0, 0}, 16};
    case 448: return PlanDesc{4, {7, 4, 4, 4, 0, 0}, 16};
    case 480: return PlanDesc{4, {16, 5, 3, 2, 0, 0}, 16};
    case 512: return PlanDesc{3, {8, 8, 8, 0, 0, 0}, 32};
    case 576: return PlanDesc{3, {8, 9, 8, 0, 0, 0}, 16};
    case 640: return PlanDesc{4, {8, 4, 4, 5, 0, 0}, 64, 32};
    case 720: return PlanDesc{3, {16, 9, 5, 0, 0, 0}, 32};
    case 768: return PlanDesc{4, {8, 8, 4, 3, 0, 0}, 64, 32};
    case 864: return PlanDesc{4, {16, 9, 3, 2, 0, 0}, 32};
    case 896: return PlanDesc{4, {8, 7, 4, 4, 0, 0}, 64, 32};
    case 960: return PlanDesc{4, {16, 5, 3, 4, 0, 0}, 32};
    case 1024: return PlanDesc{3, {16, 8, 8, 0, 0, 0}, 32};
    case 1152: return PlanDesc{4, {8, 9, 4, 4, 0, 0}, 32};
    case 1280: return PlanDesc{4, {5, 8, 8, 4, 0, 0}, 32};
    case 1344: return PlanDesc{4, {8, 7, 3, 8, 0, 0}, 64};
    case 1440: return PlanDesc{4, {8, 9, 5, 4, 0, 0}, 64};
    case 1536: return PlanDesc{4, {3, 8, 8, 8, 0, 0}, 64};
    case 1728: return PlanDesc{4, {16, 9, 3, 4, 0, 0}, 64};
    case 1792: return PlanDesc{3, {16, 7, 16, 0, 0, 0}, 64};
    case 1920: return PlanDesc{4, {16, 5, 3, 8, 0, 0}, 64};
    case 2048: return PlanDesc{3, {16, 16, 8, 0, 0, 0}, 64};
    case 2304: return PlanDesc{4, {8, 9, 8, 4, 0, 0}, 64};
    case 2560: return PlanDesc{4, {8, 5, 8, 8, 0, 0}, 64};
    case 2880: return PlanDesc{4, {16, 9, 5, 4, 0, 0}, 64};
    case 3072: return PlanDesc{4, {16, 3, 16, 4, 0, 0}, 64};
    case 3456: return PlanDesc{4, {16, 9, 3, 8, 0, 0}, 128};
    case 3840: return PlanDesc{4, {16, 5, 3, 16, 0, 0}, 128};
    case 4096: return PlanDesc{3, {16, 16, 16, 0, 0, 0}, 128};
    case 4608: return PlanDesc{4, {8, 9, 8, 8, 0, 0}, 128};
    case 5120: return PlanDesc{4, {16, 5, 8, 8, 0, 0}, 256};
    case 5760: return PlanDesc{4, {16, 9, 5, 8, 0, 0}, 256};
    case 6144: return PlanDesc{4, {16, 3, 16, 8, 0, 0}, 256};
    case 6912: return PlanDesc{4, {16, 9, 3, 16, 0, 0}, 256};
    case 7680: return PlanDesc{5, {16, 5, 3, 16, 2, 0}, 256};
    case 8192: return PlanDesc{4, {16, 16, 16, 2, 0, 0}, 256};
    default: return PlanDesc{0, {0, 0, 0, 0, 0, 0}, 0};
    }
}

// Registers (complex values) per thread of the plan of length L run by P
// threads per column: the largest butterfly share times its radix.
__host__ __device__ constexpr int plan_regs(int L, int P) {
    const PlanDesc d = plan_for(L);
    int e = 0;
    for (int s = 0; s < d.S; ++s) {
        const int r = d.r[s], per = (L / r + P - 1) / P;
        e = per * r > e ? per * r : e;
    }
    return e;
}
__host__ __device__ constexpr int plan_rmax(int L) {
    const PlanDesc d = plan_for(L);
    int m = 0;
    for (int s = 0; s < d.S; ++s) m = d.r[s] > m ? d.r[s] : m;
    return m;
}

// Threads per column of the plan in precision R.  (At 640, 768 and 896 points
// a complex64 column takes a whole wavefront, so that more columns' waves fit a
// CU beside their LDS; the FP64 passes measured fastest on 32 threads.)
template <typename R> __host__ __device__ constexpr int col_threads(int L) {
    return sizeof(R) == 8 && plan_for(L).P64 ? plan_for(L).P64 : plan_for(L).P;
}
// Threads per column of the FP64 octant-row pass of the kernel spectrum (its
// first pass, fused with the tabulation): twice the plan's wherever a thread
// would otherwise hold more than 8 complex values and every thread keeps a
// butterfly in every stage, staying within one wavefront where the plan's
// column does.  (The FP64 strided passes measured faster on the plan's own.)
__host__ __device__ constexpr int kz_threads(int L) {
    const int P = col_threads<double>(L);
    return (plan_regs(L, P) > 8 && 2 * P <= L / plan_rmax(L) && (2 * P <= 64 || P > 64)) ? 2 * P : P;
}
// Whether P threads per column fit one wavefront with no column straddling two.
__host__ __device__ constexpr bool wave_local_p(int P) { return P > 0 && P <= 64 && 64 % P == 0; }
template <typename R> __host__ __device__ constexpr bool wave_local(int L) { return wave_local_p(col_threads<R>(L)); }

// Radix of stage s and product of the radices before it, for the plan run
// forward (rev = false) or in reverse radix order (rev = true).
__host__ __device__ constexpr int plan_rad(int L, bool rev, int s) {
    return rev ? plan_for(L).r[plan_for(L).S - 1 - s] : plan_for(L).r[s];
}
__host__ __device__ constexpr int plan_ns(int L, bool rev, int s) {
    int n = 1;
    for (int i = 0; i < s; ++i) n *= plan_rad(L, rev, i);
    return n;
}
// Offset of stage s's twiddles [j][q-1] (j < Ns, q = 1..r-1) in the table of
// one direction; stages 1..S-1 have twiddles.
__host__ __device__ constexpr int plan_tw_off(int L, bool rev, int s) {
    int o = 0;
    for (int i = 1; i < s; ++i) o += plan_ns(L, rev, i) * (plan_rad(L, rev, i) - 1);
    return o;
}
__host__ __device__ constexpr int plan_tw_len(int L, bool rev) { return plan_tw_off(L, rev, plan_for(L).S); }
// The table of length L holds the forward-order stages, then the reversed-order ones.
__host__ __device__ constexpr int twiddle_table_len(int L) { return plan_tw_len(L, false) + plan_tw_len(L, true); }

// ---------------------------------------------------------------- engine

// LDS slot of one contiguous pencil.  Pad elements spread the Stockham
// stages' strided writes and contiguous reads over the 64 four-byte banks:
// for complex64, two per 32 elements and one more per 128; for complex128,
// one per 16 (the layouts with the fewest conflicts in a model of the
// engine's access patterns over the compiled lengths).
template <typename R> __host__ __device__ constexpr int pencil_pad(int m) {
    if constexpr (sizeof(R) == 4) return m + 2 * (m >> 5) + (m >> 7);
    else return m + (m >> 4);
}

// Accessor of a padded pencil slot.  at(pad(B), c) addresses element B + c as
// pad(B) + pad(c): a per-thread base plus a compile-time offset, valid where
// the engine has checked pad(B + c) = pad(B) + pad(c) for every thread.
template <typename R> struct PencilSlot {
    cx<R> *p;
    static __host__ __device__ constexpr int pad(int m) { return pencil_pad<R>(m); }
    __device__ __forceinline__ cx<R> &operator()(int m) const { return p[pad(m)]; }
    __device__ __forceinline__ cx<R> &at(int pad_base, int c) const { return p[pad_base + pad(c)]; }
};
template <class T> struct is_pencil_slot { static constexpr bool value = false; };
template <typename R> struct is_pencil_slot<PencilSlot<R>> { static constexpr bool value = true; };

// Accessor of T interleaved columns holding one real plane: element m of
// column c at p[m T + c].  With it the engine exchanges real and imaginary
// parts in two rounds, so a column needs half the LDS (twice the columns per
// CU) for twice the barriers.
template <typename R, int T> struct SplitCols {
    R *p;
    int c;
    __device__ __forceinline__ R &re(int m) const { return p[m * T + c]; }
};
template <class T> struct is_split_cols { static constexpr bool value = false; };
template <typename R, int T> struct is_split_cols<SplitCols<R, T>> { static constexpr bool value = true; };

// Orders LDS traffic between the lanes of one wavefront.  A thread's own
// accesses on either side may provably not alias (so the compiler would be
// free to swap them), but other lanes' do: the memory clobber keeps every LDS
// access on its side, and the wait makes the writes complete before any lane
// reads.  (NVP_HOST_EMULATION: the engine compiled for the host by the
// CPU tests, which run a column's threads as host threads and supply their
// own wave_sync and __syncthreads.)
#ifndef NVP_HOST_EMULATION
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
#endif

// REV = true runs the stages in reverse radix order.  Its first stage then has
// the radix of the forward plan's last stage, so a forward transform's
// outputs, as left in registers by compute_keep(), are exactly the inputs the
// reversed transform's first stage expects in the same thread and slot.
// WAVE = true: each column's P <= 64 threads lie in one wavefront (and no
// other wave touches its LDS slot), so stages synchronise per wave instead of
// per workgroup.  Tw: tw(e) -> entry e of this direction's twiddle table.
// PT: threads per column, 0 for the plan's own.
template <typename R, int L, bool REV = false, bool WAVE = false, int PT = 0> struct Fft {
    static constexpr PlanDesc D = plan_for(L);
    static constexpr int S = D.S;
    static constexpr int P = PT ? PT : col_threads<R>(L);  // threads per column
    static_assert(S > 0, "unsupported FFT length");
    static_assert(!WAVE || (P <= 64 && 64 % P == 0), "a wave-local column needs at most 64 threads, 64 % P == 0");
    static constexpr int TW_BASE = REV ? plan_tw_len(L, false) : 0;  // offset in the two-direction table

    // (from the plan held in D, so that the compile-time checks below do not
    // look the plan up again for every index they check)
    static constexpr int rad(int s) { return REV ? D.r[S - 1 - s] : D.r[s]; }
    static constexpr int ns(int s) {
        int n = 1;
        for (int i = 0; i < s; ++i) n *= rad(i);
        return n;
    }
    // butterflies of stage s, and how many each thread takes (the last one
    // only where t + i P < nb(s): full(s) says every thread has all of them)
    static constexpr int nb(int s) { return L / rad(s); }
    static constexpr int per(int s) { return (nb(s) + P - 1) / P; }
    static constexpr bool full(int s) { return nb(s) % P == 0; }
    static constexpr int regs() {
        int e = 0;
        for (int s = 0; s < S; ++s) e = per(s) * rad(s) > e ? per(s) * rad(s) : e;
        return e;
    }
    static constexpr bool every_thread_busy() {
        for (int s = 0; s < S; ++s)
            if (nb(s) < P) return false;
        return true;
    }
    static_assert(every_thread_busy(), "each stage needs at least one butterfly per thread");
    static constexpr int E = regs();                      // complex values per thread
    static constexpr int EOUT = per(S - 1) * rad(S - 1);  // registers the last stage leaves (compute_keep)

    static __device__ __forceinline__ void sync() {
        if constexpr (WAVE) wave_sync();
        else __syncthreads();
    }

    template <int s> static __device__ __forceinline__ bool valid(int t, int i) {
        if constexpr (full(s)) return true;
        else return t + i * P < nb(s);
    }

    // Output index held in register `slot` (< EOUT) after the last stage, and
    // whether that register holds an output at all.
    static __device__ __forceinline__ int out_index(int t, int slot) {
        constexpr int r = rad(S - 1);
        return t + (slot / r) * P + (slot % r) * (L / r);
    }
    static __device__ __forceinline__ bool out_valid(int t, int slot) {
        return valid<S - 1>(t, slot / rad(S - 1));
    }

    // Butterflies of stage s on v (a thread's share; values of a missing last
    // butterfly are transformed too, and never stored).
    template <int s, int SG> static __device__ __forceinline__ void bflies(cx<R> *v) {
        constexpr int r = rad(s);
#pragma unroll
        for (int i = 0; i < per(s); ++i) Dft<r, R>::template run<SG>(v + i * r);
    }

    // Inputs at or beyond L/2 of a column whose upper half is zero: first-stage
    // slots q >= K0 (K0 = ceil(r0 / 2)) hold elements >= L/2 for every thread.
    static constexpr int K0 = (rad(0) + 1) / 2;
    template <int SG, bool ZH> static __device__ __forceinline__ void bflies0(cx<R> *v) {
        constexpr int r0 = rad(0);
        if constexpr (ZH) {
#pragma unroll
            for (int i = 0; i < per(0); ++i) Dft<r0, R>::template run_lo<SG, K0>(v + i * r0);
        } else {
            bflies<0, SG>(v);
        }
    }

    // Stockham destination of butterfly b = t + i P at stage s, written so
    // that it is a per-thread base plus a compile-time offset when possible.
    static __host__ __device__ constexpr int wr_idx(int s, int t, int i) {
        const int Ns = ns(s), r = rad(s);
        if (P % Ns == 0) return (t / Ns) * Ns * r + (t % Ns) + i * P * r;
        if (P * per(s) <= Ns) return t + i * P;
        const int b = t + i * P;
        return (b / Ns) * Ns * r + b % Ns;
    }
    template <int s> static __device__ __forceinline__ int wr_index(int t, int i) { return wr_idx(s, t, i); }
    // j = b mod Ns for b = t + i P, likewise.
    template <int s> static __device__ __forceinline__ int tw_j(int t, int i) {
        constexpr int Ns = ns(s);
        if constexpr (P % Ns == 0) return t % Ns;
        else if constexpr (P * per(s) <= Ns) return t + i * P;
        else return (t + i * P) % Ns;
    }

    // Whether the writes of stage s (element wr_idx(s, t, i) + p Ns) and the
    // reads of stage s (element t + i P + q L / r) may address a padded slot
    // as pad(base) + pad(offset) with the offset taken from thread 0, checked
    // for every thread and butterfly.
    static constexpr bool split_writes(int s) {
        const int Ns = ns(s), r = rad(s);
        if (!(P % Ns == 0 || P * per(s) <= Ns)) return false;
        for (int t = 0; t < P; ++t) {
            const int B = wr_idx(s, t, 0);
            for (int i = 0; i < per(s); ++i) {
                if (t + i * P >= nb(s)) continue;
                for (int p = 0; p < r; ++p) {
                    const int c = wr_idx(s, t, i) - B + p * Ns;
                    const int c0 = wr_idx(s, 0, i) - wr_idx(s, 0, 0) + p * Ns;
                    if (c != c0 || c < 0 || pencil_pad<R>(B + c) != pencil_pad<R>(B) + pencil_pad<R>(c)) return false;
                }
            }
        }
        return true;
    }
    static constexpr bool split_reads(int s) {
        const int r = rad(s);
        for (int t = 0; t < P; ++t)
            for (int i = 0; i < per(s); ++i) {
                if (t + i * P >= nb(s)) continue;
                for (int q = 0; q < r; ++q) {
                    const int c = i * P + q * (L / r);
                    if (pencil_pad<R>(t + c) != pencil_pad<R>(t) + pencil_pad<R>(c)) return false;
                }
            }
        return true;
    }

    // First-stage inputs: v[i r0 + q] = x[t + i P + q L / r0] for the
    // thread's butterflies (zero for a missing last one, which reads nothing).
    // ZH: the column's elements from L/2 on are zero and are not read.
    template <bool ZH = false, class Ld> static __device__ __forceinline__ void load0(cx<R> *v, int t, Ld ld) {
        constexpr int r0 = rad(0);
#pragma unroll
        for (int i = 0; i < per(0); ++i) {
            const int b = t + i * P;
            const bool ok = valid<0>(t, i);
#pragma unroll
            for (int q = 0; q < r0; ++q) {
                if ((!ZH || q < K0) && ok) v[i * r0 + q] = ld(b + q * (L / r0));
                else v[i * r0 + q] = czero<R>();
            }
        }
    }

    // All stages on v (loaded by load0); st(m, x) receives the outputs.
    // ZH: inputs from L/2 on are zero.  OH: only outputs below L/2 are stored.
    template <int SG, bool ZH = false, bool OH = false, class Tw, class St, class Lds>
    static __device__ __forceinline__ void compute(cx<R> *v, int t, Tw tw, St st, Lds lds) {
        bflies0<SG, ZH>(v);
        next<0, SG, true, OH>(v, t, tw, st, lds);
    }

    // All stages on v; the outputs stay in v (see out_index, out_valid).
    template <int SG, bool ZH = false, class Tw, class Lds>
    static __device__ __forceinline__ void compute_keep(cx<R> *v, int t, Tw tw, Lds lds) {
        bflies0<SG, ZH>(v);
        next<0, SG, false, false>(v, t, tw, [](int, cx<R>) {}, lds);
    }

    // Transform this thread's share of one column.
    //   ld(m)     -> input element m (first stage)
    //   st(m, x)  <- output element m (last stage, natural order)
    //   lds(m)    -> reference to element m of this column's LDS slot
    // LDS_IN: ld reads the same LDS slot, so wait before overwriting it.
    template <int SG, bool LDS_IN, bool ZH = false, bool OH = false, class Tw, class Ld, class St, class Lds>
    static __device__ __forceinline__ void run(int t, Tw tw, Ld ld, St st, Lds lds) {
        cx<R> v[E];
        load0<ZH>(v, t, ld);
        if constexpr (LDS_IN) sync();
        compute<SG, ZH, OH>(v, t, tw, st, lds);
    }

    // The LDS exchange after stage s through a single real plane: real parts,
    // then imaginary parts; the next stage's inputs come out twiddled.
    template <int s, int SG, class W, class Lds>
    static __device__ __forceinline__ void exchange_split(cx<R> *v, int t, W twq, Lds lds) {
        constexpr int r = rad(s), Ns = ns(s), r1 = rad(s + 1);
        R xr[E];
#pragma unroll
        for (int part = 0; part < 2; ++part) {
#pragma unroll
            for (int i = 0; i < per(s); ++i) {
                if (!valid<s>(t, i)) continue;
                const int w = wr_index<s>(t, i);
#pragma unroll
                for (int p = 0; p < r; ++p) lds.re(w + p * Ns) = part ? v[i * r + p].y : v[i * r + p].x;
            }
            sync();
#pragma unroll
            for (int i = 0; i < per(s + 1); ++i) {
                if (!valid<s + 1>(t, i)) continue;
                const int b = t + i * P;
#pragma unroll
                for (int q = 0; q < r1; ++q) {
                    const R y = lds.re(b + q * (L / r1));
                    if (part == 0) {
                        xr[i * r1 + q] = y;
                    } else {
                        const cx<R> x = mk<R>(xr[i * r1 + q], y);
                        if (q == 0) v[i * r1] = x;
                        else v[i * r1 + q] = SG < 0 ? cmul<R>(x, twq(i, q)) : cmulc<R>(x, twq(i, q));
                    }
                }
            }
            sync();
        }
    }

    template <int s, int SG, bool STORE, bool OH, class Tw, class St, class Lds>
    static __device__ __forceinline__ void next(cx<R> *v, int t, Tw tw, St st, Lds lds) {
        constexpr int r = rad(s);
        constexpr int Ns = ns(s);
        if constexpr (s == S - 1) {
            if constexpr (STORE) {
#pragma unroll
                for (int i = 0; i < per(s); ++i) {
                    if (!valid<s>(t, i)) continue;
                    const int b = t + i * P;
#pragma unroll
                    for (int p = 0; p < r; ++p)
                        if (!OH || p < (r + 1) / 2) st(b + p * (L / r), v[i * r + p]);
                }
            }
        } else {
            constexpr int r1 = rad(s + 1);
            constexpr int I1 = per(s + 1);
            constexpr int off = TW_BASE + plan_tw_off(L, REV, s + 1);
            // next stage's twiddles first, so that their loads are in flight during the
            // LDS exchange (complex64; complex128 values would cost too many registers)
            constexpr bool PRE = sizeof(R) == 4;
            cx<R> wv[I1][r1 - 1];
            if constexpr (PRE) {
#pragma unroll
                for (int i = 0; i < I1; ++i) {
                    if (!valid<s + 1>(t, i)) continue;
                    const int jb = off + tw_j<s + 1>(t, i) * (r1 - 1) - 1;
#pragma unroll
                    for (int q = 1; q < r1; ++q) wv[i][q - 1] = tw(jb + q);
                }
            }
            auto twq = [&](int i, int q) {
                if constexpr (PRE) return wv[i][q - 1];
                else return tw(off + tw_j<s + 1>(t, i) * (r1 - 1) - 1 + q);
            };
            if constexpr (is_split_cols<Lds>::value) {
                exchange_split<s, SG>(v, t, twq, lds);
            } else {
            constexpr bool WS = is_pencil_slot<Lds>::value && split_writes(s);
            const int pw = WS ? pencil_pad<R>(wr_index<s>(t, 0)) : 0;
#pragma unroll
            for (int i = 0; i < per(s); ++i) {
                if (!valid<s>(t, i)) continue;
                const int w = wr_index<s>(t, i);
#pragma unroll
                for (int p = 0; p < r; ++p) {
                    if constexpr (WS) lds.at(pw, wr_idx(s, 0, i) - wr_idx(s, 0, 0) + p * Ns) = v[i * r + p];
                    else lds(w + p * Ns) = v[i * r + p];
                }
            }
            sync();
            constexpr bool RS = is_pencil_slot<Lds>::value && split_reads(s + 1);
            const int pr = RS ? pencil_pad<R>(t) : 0;
#pragma unroll
            for (int i = 0; i < I1; ++i) {
                if (!valid<s + 1>(t, i)) continue;
                const int b = t + i * P;
                if constexpr (RS) v[i * r1] = lds.at(pr, i * P);
                else v[i * r1] = lds(b);
#pragma unroll
                for (int q = 1; q < r1; ++q) {
                    cx<R> x;
                    if constexpr (RS) x = lds.at(pr, i * P + q * (L / r1));
                    else x = lds(b + q * (L / r1));
                    const cx<R> w = twq(i, q);
                    v[i * r1 + q] = SG < 0 ? cmul<R>(x, w) : cmulc<R>(x, w);
                }
            }
            sync();
            }
            bflies<s + 1, SG>(v);
            next<s + 1, SG, STORE, OH>(v, t, tw, st, lds);
        }
    }
};

}  // namespace nvp
