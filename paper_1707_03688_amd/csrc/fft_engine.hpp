// Device-side building blocks of the fused NsDLCT passes (gfx950).
//
//  * cplx<T>            interleaved complex value in registers
//  * dft_reg<R, S>      R-point DFT (R = 2..64) fully in registers, exponent
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

// cos(2 pi k / 64), k = 0..63 (sin(2 pi k/64) = entry (k + 48) mod 64).
constexpr double kCos64[64] = {
    1.0, 0.9951847266721969, 0.9807852804032304, 0.9569403357322088,
    0.9238795325112867, 0.881921264348355, 0.8314696123025452, 0.773010453362737,
    0.7071067811865476, 0.6343932841636455, 0.5555702330196023, 0.4713967368259978,
    0.38268343236508984, 0.29028467725446233, 0.19509032201612833, 0.09801714032956077,
    0.0, -0.09801714032956065, -0.1950903220161282, -0.29028467725446216,
    -0.3826834323650897, -0.4713967368259977, -0.555570233019602, -0.6343932841636454,
    -0.7071067811865475, -0.773010453362737, -0.8314696123025453, -0.8819212643483549,
    -0.9238795325112867, -0.9569403357322088, -0.9807852804032304, -0.9951847266721968,
    -1.0, -0.9951847266721969, -0.9807852804032304, -0.9569403357322089,
    -0.9238795325112868, -0.881921264348355, -0.8314696123025455, -0.7730104533627371,
    -0.7071067811865477, -0.6343932841636459, -0.5555702330196022, -0.47139673682599786,
    -0.38268343236509034, -0.29028467725446244, -0.19509032201612866, -0.09801714032956045,
    0.0, 0.09801714032956009, 0.1950903220161283, 0.29028467725446205,
    0.38268343236509, 0.4713967368259976, 0.5555702330196018, 0.6343932841636456,
    0.7071067811865474, 0.7730104533627367, 0.8314696123025452, 0.8819212643483548,
    0.9238795325112865, 0.9569403357322088, 0.9807852804032303, 0.9951847266721969};

// v * exp(S 2 pi i e / L) for compile-time L | 64 and e (after unrolling).
template <int S, typename T>
__device__ __forceinline__ cplx<T> twiddle_ct(cplx<T> v, int L, int e) {
    const int k = ((e % L) + L) % L * (64 / L);
    if (k == 0) return v;
    if (k == 16) return mul_si<S>(v);
    if (k == 32) return {-v.re, -v.im};
    if (k == 48) return mul_si<-S>(v);
    const T c = (T)kCos64[k];
    const T s = (T)(S * kCos64[(k + 48) & 63]);
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

template <int R, int S, typename T>
__device__ __forceinline__ void dft_base(cplx<T>* v) {
    if constexpr (R == 2)
        dft2<S>(v);
    else if constexpr (R == 4)
        dft4<S>(v);
}

// One in-register Stockham stage of an R-point DFT with radix r (r = 2 or 4).
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
        constexpr int r = (rem % 4 == 0) ? 4 : 2;
        reg_stage<R, r, Ns, S>(v);
        reg_stages<R, Ns * r, S>(v);
    }
}

// R-point DFT in registers, natural order in and out.
template <int R, int S, typename T>
__device__ __forceinline__ void dft_reg(cplx<T>* v) {
    if constexpr (R == 2 || R == 4)
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
template <int A>
struct Last1 {
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

// LDS index of line position p (one padding element every 16).
__device__ __forceinline__ int lds_pad(int p) { return p + (p >> 4); }
template <int N>
constexpr int lds_line_elems() {
    return N + (N >> 4) + 1;
}

// Twiddle tables W_NT^k = exp(-2 pi i k / NT), filled once per device.
constexpr int kTwiddleN = 4096;

template <typename T, int N, int TPL>
struct LineFFT {
    static constexpr int E = N / TPL;

    // One Stockham stage (twiddles + radix-R butterflies) on the registers.
    template <int S, int Ns, int R>
    __device__ __forceinline__ static void stage(cplx<T>* v, int t, const cplx<T>* __restrict__ tw) {
        static_assert(E % R == 0, "radix must divide the per-thread sample count");
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            if constexpr (Ns > 1) {
                const int j = t + TPL * i;
                const int k = j % Ns;
                constexpr int step = kTwiddleN / (Ns * R);
#pragma unroll
                for (int q = 1; q < R; ++q) {
                    const int e = (q * k) % (Ns * R);
                    cplx<T> w = tw[e * step];
                    if constexpr (S > 0) w.im = -w.im;
                    v[i * R + q] = cmul(v[i * R + q], w);
                }
            }
            dft_reg<R, S>(&v[i * R]);
        }
    }

    // Stage-s outputs to LDS, then stage-(s+1) inputs back to registers.
    template <int Ns, int R, int Rn>
    __device__ __forceinline__ static void exchange(cplx<T>* v, cplx<T>* lds, int t) {
#pragma unroll
        for (int i = 0; i < E / R; ++i) {
            const int j = t + TPL * i;
            const int k = j % Ns;
            const int base = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) lds[lds_pad(base + q * Ns)] = v[i * R + q];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E / Rn; ++i) {
            const int j = t + TPL * i;
#pragma unroll
            for (int q = 0; q < Rn; ++q) v[i * Rn + q] = lds[lds_pad(j + q * (N / Rn))];
        }
        __syncthreads();
    }

    template <int S, int Ns, int R, int... Rest>
    __device__ __forceinline__ static void run_stages(cplx<T>* v, cplx<T>* lds, int t,
                                                      const cplx<T>* __restrict__ tw) {
        stage<S, Ns, R>(v, t, tw);
        if constexpr (sizeof...(Rest) > 0) {
            constexpr int Rn = First<Rest...>::value;
            exchange<Ns, R, Rn>(v, lds, t);
            run_stages<S, Ns * R, Rest...>(v, lds, t, tw);
        }
    }

    template <int S, int... R>
    __device__ __forceinline__ static void run(RList<R...>, cplx<T>* v, cplx<T>* lds, int t,
                                               const cplx<T>* __restrict__ tw) {
        run_stages<S, 1, R...>(v, lds, t, tw);
    }

    // Full line DFT with exponent sign S: registers hold positions
    // t + TPL*i + q*(N/R0) before and after (R0 = first = last radix).
    template <int S>
    __device__ __forceinline__ static void dft(cplx<T>* v, cplx<T>* lds, int t,
                                               const cplx<T>* __restrict__ tw) {
        run<S>(typename LinePlan<N>::L{}, v, lds, t, tw);
    }

    template <int... R>
    static constexpr int first_radix(RList<R...>) {
        return First<R...>::value;
    }
    template <int... R>
    static constexpr int last_radix(RList<R...>) {
        return LastOf<R...>::value;
    }
    static constexpr int R0 = first_radix(typename LinePlan<N>::L{});
    static_assert(R0 == last_radix(typename LinePlan<N>::L{}), "first and last radix must match");
    static_assert(E % R0 == 0, "bad line plan");
};

}  // namespace nslct
