// Device-side building blocks of the fused NsDLCT passes (gfx950).
//
//  * cplx<T>            interleaved complex value in registers
//  * dft_reg<R, S>      R-point DFT (R = 2^a 3^b up to 64) in registers, exponent
//                       sign S (-1 forward, +1 inverse), compile-time twiddles
//  * LineFFT<T, N, ...> an N-point line DFT spread over TPL threads of a
//                       workgroup: mixed-radix Stockham stages, each thread
//                       owning N/TPL samples in registers, LDS exchanges
//                       between stages.  The first and the last stage use the
//                       same radix, so a line DFT leaves every thread holding
//                       exactly the positions the next line DFT starts from:
//                       an FFT -> pointwise chirp -> IFFT sequence needs no
//                       exchange around the chirp.
//
// Stage s (radix R, Ns = product of the radices before it) computes, for every
// butterfly j in [0, N/R): inputs x[j + q N/R] (q < R), twiddle by
// W_{Ns R}^{q (j mod Ns)}, an R-point DFT, outputs to
// y[(j div Ns) Ns R + (j mod Ns) + q Ns].  After the last stage y is the DFT
// in natural order.  Thread t owns butterflies j = t + TPL*i.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nslct {

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * (S i) for S = +-1.
template <int S, typename T>
__device__ __forceinline__ cplx<T> mul_si(cplx<T> a) {
    if constexpr (S > 0)
        return {-a.im, a.re};
    else
        return {a.im, -a.re};
}

// cos(2 pi k / 192), k = 0..191 (sin(2 pi k/192) = entry (k + 144) mod 192).
// 192 = 3 * 64 covers every in-register twiddle of radices built from 2, 3, 4.
constexpr double kCos192[192] = {
    1.0, 0.9994645874763657, 0.9978589232386035, 0.9951847266721969,
    0.9914448613738104, 0.986643332084879, 0.9807852804032304, 0.9738769792773336,
    0.9659258262890683, 0.9569403357322088, 0.9469301294951057, 0.9359059267573258,
    0.9238795325112867, 0.9108638249211758, 0.8968727415326884, 0.881921264348355,
    0.8660254037844387, 0.8492021815265789, 0.8314696123025452, 0.8128466845916152,
    0.7933533402912352, 0.773010453362737, 0.7518398074789774, 0.7298640726978357,
    0.7071067811865476, 0.6835923020228712, 0.6593458151000688, 0.6343932841636455,
    0.6087614290087207, 0.5824776968678022, 0.5555702330196024, 0.5280678506503681,
    0.5000000000000001, 0.4713967368259976, 0.44228869021900125, 0.4127070298043947,
    0.38268343236508984, 0.3522500479212336, 0.3214394653031617, 0.2902846772544625,
    0.25881904510252074, 0.22707626303437345, 0.19509032201612833, 0.16289547339458882,
    0.1305261922200517, 0.09801714032956055, 0.06540312923014327, 0.032719082821776165,
    0.0, -0.03271908282177604, -0.06540312923014314, -0.09801714032956042,
    -0.1305261922200516, -0.1628954733945887, -0.1950903220161282, -0.2270762630343733,
    -0.25881904510252063, -0.29028467725446216, -0.3214394653031616, -0.3522500479212335,
    -0.3826834323650895, -0.4127070298043946, -0.44228869021900113, -0.4713967368259977,
    -0.4999999999999998, -0.528067850650368, -0.5555702330196023, -0.582477696867802,
    -0.6087614290087207, -0.6343932841636454, -0.6593458151000688, -0.6835923020228714,
    -0.7071067811865475, -0.7298640726978354, -0.7518398074789773, -0.773010453362737,
    -0.793353340291235, -0.8128466845916151, -0.831469612302545, -0.8492021815265788,
    -0.8660254037844387, -0.8819212643483549, -0.8968727415326881, -0.9108638249211759,
    -0.9238795325112867, -0.9359059267573258, -0.9469301294951056, -0.9569403357322087,
    -0.9659258262890682, -0.9738769792773336, -0.9807852804032304, -0.986643332084879,
    -0.9914448613738104, -0.9951847266721968, -0.9978589232386035, -0.9994645874763657,
    -1.0, -0.9994645874763657, -0.9978589232386035, -0.9951847266721969,
    -0.9914448613738104, -0.986643332084879, -0.9807852804032305, -0.9738769792773336,
    -0.9659258262890683, -0.9569403357322088, -0.9469301294951057, -0.9359059267573259,
    -0.9238795325112868, -0.910863824921176, -0.8968727415326883, -0.881921264348355,
    -0.8660254037844388, -0.8492021815265789, -0.8314696123025455, -0.812846684591615,
    -0.7933533402912352, -0.7730104533627371, -0.7518398074789775, -0.7298640726978359,
    -0.7071067811865479, -0.6835923020228712, -0.6593458151000691, -0.6343932841636459,
    -0.6087614290087209, -0.5824776968678023, -0.5555702330196022, -0.5280678506503678,
    -0.5000000000000004, -0.47139673682599786, -0.44228869021900136, -0.41270702980439467,
    -0.3826834323650895, -0.35225004792123393, -0.3214394653031618, -0.29028467725446244,
    -0.25881904510252063, -0.22707626303437292, -0.19509032201612866, -0.16289547339458896,
    -0.13052619222005163, -0.09801714032956134, -0.06540312923014273, -0.03271908282177651,
    0.0, 0.032719082821776144, 0.06540312923014237, 0.09801714032956096,
    0.13052619222005127, 0.1628954733945886, 0.1950903220161283, 0.22707626303437256,
    0.2588190451025203, 0.29028467725446205, 0.3214394653031615, 0.35225004792123354,
    0.38268343236508917, 0.41270702980439433, 0.442288690219001, 0.4713967368259976,
    0.5000000000000001, 0.5280678506503674, 0.5555702330196018, 0.5824776968678019,
    0.6087614290087199, 0.6343932841636449, 0.6593458151000691, 0.6835923020228717,
    0.7071067811865474, 0.7298640726978356, 0.7518398074789775, 0.7730104533627367,
    0.7933533402912349, 0.8128466845916151, 0.8314696123025448, 0.8492021815265786,
    0.8660254037844384, 0.8819212643483553, 0.8968727415326883, 0.9108638249211758,
    0.9238795325112868, 0.9359059267573255, 0.9469301294951056, 0.9569403357322088,
    0.9659258262890681, 0.9738769792773335, 0.9807852804032303, 0.9866433320848791,
    0.9914448613738104, 0.9951847266721969, 0.9978589232386035, 0.9994645874763657};

// v * exp(S 2 pi i e / L) for compile-time L | 192 and e (after unrolling).
template <int S, typename T>
__device__ __forceinline__ cplx<T> twiddle_ct(cplx<T> v, int L, int e) {
    const int k = ((e % L) + L) % L * (192 / L);
    if (k == 0) return v;
    if (k == 48) return mul_si<S>(v);
    if (k == 96) return {-v.re, -v.im};
    if (k == 144) return mul_si<-S>(v);
    const T c = (T)kCos192[k];
    const T s = (T)(S * kCos192[(k + 144) % 192]);
    return cmul(v, cplx<T>{c, s});
}

template <int S, typename T>
__device__ __forceinline__ void dft2(cplx<T>* v) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <int S, typename T>
__device__ __forceinline__ void dft4(cplx<T>* v) {
    const cplx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cplx<T> s13 = cadd(v[1], v[3]), d13 = mul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

// y1 = a + w b + w^2 c with w = exp(S 2 pi i / 3) = -1/2 + S i sqrt(3)/2.
template <int S, typename T>
__device__ __forceinline__ void dft3(cplx<T>* v) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    const cplx<T> s = cadd(v[1], v[2]);
    const cplx<T> d = csub(v[1], v[2]);
    const cplx<T> m = {v[0].re - (T)0.5 * s.re, v[0].im - (T)0.5 * s.im};
    const cplx<T> r = mul_si<S>(cplx<T>{h * d.re, h * d.im});
    v[0] = cadd(v[0], s);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

template <int R, int S, typename T>
__device__ __forceinline__ void dft_base(cplx<T>* v) {
    if constexpr (R == 2)
        dft2<S>(v);
    else if constexpr (R == 3)
        dft3<S>(v);
    else if constexpr (R == 4)
        dft4<S>(v);
}

// One in-register Stockham stage of an R-point DFT with radix r (2, 3 or 4).
template <int R, int r, int Ns, int S, typename T>
__device__ __forceinline__ void reg_stage(cplx<T>* x) {
    cplx<T> y[R];
#pragma unroll
    for (int j = 0; j < R / r; ++j) {
        const int k = j % Ns;
        cplx<T> v[r];
#pragma unroll
        for (int q = 0; q < r; ++q) v[q] = x[j + q * (R / r)];
#pragma unroll
        for (int q = 1; q < r; ++q) v[q] = twiddle_ct<S>(v[q], Ns * r, q * k);
        dft_base<r, S>(v);
#pragma unroll
        for (int q = 0; q < r; ++q) y[(j / Ns) * Ns * r + k + q * Ns] = v[q];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = y[i];
}

template <int R, int Ns, int S, typename T>
__device__ __forceinline__ void reg_stages(cplx<T>* v) {
    if constexpr (Ns < R) {
        constexpr int rem = R / Ns;
        constexpr int r = (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : 3;
        reg_stage<R, r, Ns, S>(v);
        reg_stages<R, Ns * r, S>(v);
    }
}

// R-point DFT in registers, natural order in and out.
template <int R, int S, typename T>
__device__ __forceinline__ void dft_reg(cplx<T>* v) {
    if constexpr (R == 2 || R == 3 || R == 4)
        dft_base<R, S>(v);
    else
        reg_stages<R, 1, S>(v);
}

template <int... R>
struct RList {};

template <int A, int... Rest>
struct First {
    static constexpr int value = A;
};
template <int... R>
struct LastOf;
template <int A>
struct LastOf<A> {
    static constexpr int value = A;
};
template <int A, int B, int... Rest>
struct LastOf<A, B, Rest...> {
    static constexpr int value = LastOf<B, Rest...>::value;
};

// Line-DFT decomposition per size: TPL threads per line, radix list with equal
// first and last radix (single-stage sizes trivially).
template <int N>
struct LinePlan;
template <>
struct LinePlan<2> {
    static constexpr int TPL = 1;
    using L = RList<2>;
};
template <>
struct LinePlan<4> {
    static constexpr int TPL = 1;
    using L = RList<4>;
};
template <>
struct LinePlan<8> {
    static constexpr int TPL = 1;
    using L = RList<8>;
};
template <>
struct LinePlan<16> {
    static constexpr int TPL = 4;
    using L = RList<4, 4>;
};
template <>
struct LinePlan<32> {
    static constexpr int TPL = 8;
    using L = RList<4, 2, 4>;
};
template <>
struct LinePlan<64> {
    static constexpr int TPL = 8;
    using L = RList<8, 8>;
};
template <>
struct LinePlan<128> {
    static constexpr int TPL = 16;
    using L = RList<4, 8, 4>;
};
template <>
struct LinePlan<256> {
    static constexpr int TPL = 16;
    using L = RList<16, 16>;
};
template <>
struct LinePlan<512> {
    static constexpr int TPL = 64;
    using L = RList<8, 8, 8>;
};
template <>
struct LinePlan<1024> {
    static constexpr int TPL = 64;
    using L = RList<16, 4, 16>;
};
template <>
struct LinePlan<2048> {
    static constexpr int TPL = 128;
    using L = RList<16, 8, 16>;
};
template <>
struct LinePlan<4096> {
    static constexpr int TPL = 256;
    using L = RList<16, 16, 16>;
};

template <>
struct LinePlan<6> {
    static constexpr int TPL = 1;
    using L = RList<6>;
};
template <>
struct LinePlan<12> {
    static constexpr int TPL = 1;
    using L = RList<12>;
};
template <>
struct LinePlan<24> {
    static constexpr int TPL = 1;
    using L = RList<24>;
};
template <>
struct LinePlan<48> {
    static constexpr int TPL = 4;
    using L = RList<4, 3, 4>;
};
template <>
struct LinePlan<96> {
    static constexpr int TPL = 8;
    using L = RList<4, 6, 4>;
};
template <>
struct LinePlan<192> {
    static constexpr int TPL = 8;
    using L = RList<8, 3, 8>;
};
template <>
struct LinePlan<384> {
    static constexpr int TPL = 16;
    using L = RList<8, 6, 8>;
};
template <>
struct LinePlan<768> {
    static constexpr int TPL = 32;
    using L = RList<8, 12, 8>;
};

// Alternative line plans (V = 1) that the ragged batch's schedule tuner
// times against LinePlan<N> (V = 0) and that the single-image passes take
// where they measured faster: another split of the line over threads and
// radices, the first and last radix equal and every radix dividing the
// per-thread sample count (lines inside one wavefront up to 1024).
template <int N, int V>
struct PlanVariant : LinePlan<N> {
    static constexpr bool exists = V == 0;
};
#define NSLCT_PLAN_VARIANT(n, tpl, ...)           \
    template <>                                   \
    struct PlanVariant<n, 1> {                    \
        static constexpr bool exists = true;      \
        static constexpr int TPL = tpl;           \
        using L = RList<__VA_ARGS__>;             \
    };
NSLCT_PLAN_VARIANT(64, 16, 4, 4, 4)
NSLCT_PLAN_VARIANT(128, 8, 8, 2, 8)
NSLCT_PLAN_VARIANT(192, 16, 4, 12, 4)
NSLCT_PLAN_VARIANT(256, 32, 8, 4, 8)
NSLCT_PLAN_VARIANT(384, 32, 4, 6, 4, 4)
NSLCT_PLAN_VARIANT(512, 32, 16, 2, 16)
NSLCT_PLAN_VARIANT(768, 64, 4, 12, 4, 4)
NSLCT_PLAN_VARIANT(1024, 32, 16, 4, 16)
NSLCT_PLAN_VARIANT(4096, 128, 16, 16, 16)
#undef NSLCT_PLAN_VARIANT

// LDS index of line position p (one padding element every 16).
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }
template <int N>
constexpr int lds_line_elems() {
    return N + (N >> 4) + 1;
}

// Twiddle tables W_NT^k = exp(-2 pi i k / NT), filled once per device;
// NT = 3 * 4096 serves every supported N (N divides NT).
constexpr int kTwiddleN = 12288;

// Orders this wavefront's LDS writes before its later LDS reads (a line
// that lives inside one wavefront needs no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int N, int TPL, typename PL = typename LinePlan<N>::L>
struct LineFFT {
    static constexpr int E = N / TPL;
    // A line owned by at most one wavefront synchronises at wavefront scope.
    static constexpr bool kWave = TPL <= 64;

    __device__ __forceinline__ static void sync() {
        if constexpr (kWave)
            wave_lds_sync();
        else
            __syncthreads();
    }

    // Stages whose twiddle exponent k = j mod Ns is the same for all of a
    // thread's butterflies (TPL a multiple of Ns) keep their R-1 twiddles in
    // registers, loaded once per kernel; the others read the table.
    template <int Ns, int R>
    static constexpr bool preloaded() {
        return Ns > 1 && TPL % Ns == 0;
    }
    template <int Ns, int R, int... Rest>
    static constexpr int tw_count() {
        constexpr int here = preloaded<Ns, R>() ? R - 1 : 0;
        if constexpr (sizeof...(Rest) > 0)
            return here + tw_count<Ns * R, Rest...>();
        else
            return here;
    }
    template <int... R>
    static constexpr int tw_total(RList<R...>) {
        return tw_count<1, R...>();
    }
    static constexpr int TW = tw_total(PL{}) > 0 ? tw_total(PL{}) : 1;

    template <int Ns, int R, int... Rest>
    __device__ __forceinline__ static void preload_from(cplx<T>* w, int off, int t, const cplx<T>* __restrict__ tab) {
        if constexpr (preloaded<Ns, R>()) {
            const int k = t % Ns;
            constexpr int step = kTwiddleN / (Ns * R);
#pragma unroll
            for (int q = 1; q < R; ++q) w[off + q - 1] = tab[((q * k) % (Ns * R)) * step];
        }
        if constexpr (sizeof...(Rest) > 0)
            preload_from<Ns * R, Rest...>(w, off + (preloaded<Ns, R>() ? R - 1 : 0), t, tab);
    }
    template <int... R>
    __device__ __forceinline__ static void preload_list(RList<R...>, cplx<T>* w, int t,
                                                        const cplx<T>* __restrict__ tab) {
        preload_from<1, R...>(w, 0, t, tab);
    }
    // Loads this thread's register twiddles (forward sign) for all stages.
    __device__ __forceinline__ static void preload(cplx<T>* w, int t, const cplx<T>* __restrict__ tab) {
        preload_list(PL{}, w, t, tab);
    }

    // One Stockham stage (twiddles + radix-R butterflies) on the registers.
    template <int S, int Ns, int R, int OFF>
    __device__ __forceinline__ static void stage(cplx<T>* v, int t, const cplx<T>* w,
                                                 const cplx<T>* __restrict__ tab) {
        static_assert(E % R == 0, "radix must divide the per-thread sample count");
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            if constexpr (Ns > 1) {
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    cplx<T> tw;
                    if constexpr (preloaded<Ns, R>()) {
                        tw = w[OFF + q - 1];
                    } else {
                        const int j = t + TPL * i;
                        const int k = j % Ns;
                        constexpr int step = kTwiddleN / (Ns * R);
                        tw = tab[((q * k) % (Ns * R)) * step];
                    }
                    if constexpr (S > 0) tw.im = -tw.im;
                    v[i * R + q] = cmul(v[i * R + q], tw);
                }
            }
            dft_reg<R, S>(&v[i * R]);
        }
    }

    // Stage-s outputs to LDS, then stage-(s+1) inputs back to registers.
    // lds_pad(p + m) = lds_pad(p) + m + m / 16 for m a multiple of 16 (p >= 0),
    // so where the index steps are multiples of 16 every access of a loop is
    // an immediate offset from one padded base; otherwise each is padded.
    template <int Ns, int R, int Rn>
    __device__ __forceinline__ static void exchange(cplx<T>* v, cplx<T>* lds, int t) {
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            const int j = t + TPL * i;
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
            if constexpr (Ns % 16 == 0) {
                const int pb = lds_pad(base);
#pragma unroll
                for (int q = 0; q < R; ++q) lds[pb + q * (Ns + Ns / 16)] = v[i * R + q];
            } else if constexpr (Ns == 1 && 16 % R == 0) {
                // base = R j with R | 16: the R outputs share one padding group.
                const int pb = lds_pad(base);
#pragma unroll
                for (int q = 0; q < R; ++q) lds[pb + q] = v[i * R + q];
            } else if constexpr (16 % Ns == 0 && R > 16 / Ns) {
                // Offsets q Ns repeat modulo 16 with period P = 16 / Ns: one
                // padded base per residue q0 < P, then steps of 16.
                constexpr int P = 16 / Ns;
                int pb[P];
#pragma unroll
                for (int q0 = 0; q0 < P; ++q0) pb[q0] = lds_pad(base + q0 * Ns);
#pragma unroll
                for (int q = 0; q < R; ++q) lds[pb[q % P] + (q / P) * 17] = v[i * R + q];
            } else {
#pragma unroll
                for (int q = 0; q < R; ++q) lds[lds_pad(base + q * Ns)] = v[i * R + q];
            }
        }
        sync();
        constexpr int st = N / Rn;
        const int pt = lds_pad(t);
#pragma unroll
        for (int i = 0; i < E / Rn; ++i) {
            const int j = t + TPL * i;
            if constexpr (st % 16 == 0 && TPL % 16 == 0) {
                const int pj = pt + i * (TPL + TPL / 16);
#pragma unroll
                for (int q = 0; q < Rn; ++q) v[i * Rn + q] = lds[pj + q * (st + st / 16)];
            } else {
#pragma unroll
                for (int q = 0; q < Rn; ++q) v[i * Rn + q] = lds[lds_pad(j + q * st)];
            }
        }
        sync();
    }

    template <int S, int Ns, int OFF, int R, int... Rest>
    __device__ __forceinline__ static void run_stages(cplx<T>* v, cplx<T>* lds, int t, const cplx<T>* w,
                                                      const cplx<T>* __restrict__ tab) {
        stage<S, Ns, R, OFF>(v, t, w, tab);
        if constexpr (sizeof...(Rest) > 0) {
            constexpr int Rn = First<Rest...>::value;
            exchange<Ns, R, Rn>(v, lds, t);
            run_stages<S, Ns * R, OFF + (preloaded<Ns, R>() ? R - 1 : 0), Rest...>(v, lds, t, w, tab);
        }
    }

    template <int S, int... R>
    __device__ __forceinline__ static void run(RList<R...>, cplx<T>* v, cplx<T>* lds, int t, const cplx<T>* w,
                                               const cplx<T>* __restrict__ tab) {
        run_stages<S, 1, 0, R...>(v, lds, t, w, tab);
    }

    // Full line DFT with exponent sign S: registers hold positions
    // t + TPL*i + q*(N/R0) before and after (R0 = first = last radix).
    template <int S>
    __device__ __forceinline__ static void dft(cplx<T>* v, cplx<T>* lds, int t, const cplx<T>* w,
                                               const cplx<T>* __restrict__ tab) {
        run<S>(PL{}, v, lds, t, w, tab);
    }

    template <int... R>
    static constexpr int first_radix(RList<R...>) {
        return First<R...>::value;
    }
    template <int... R>
    static constexpr int last_radix(RList<R...>) {
        return LastOf<R...>::value;
    }
    static constexpr int R0 = first_radix(PL{});
    static_assert(R0 == last_radix(PL{}), "first and last radix must match");
    static_assert(E % R0 == 0, "bad line plan");
    static_assert(R0 % 2 == 0, "the chirp index split assumes an even first radix");
};

}  // namespace nslct
