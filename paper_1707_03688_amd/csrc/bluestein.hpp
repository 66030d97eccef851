// Bluestein line DFTs for line lengths without a native plan (device code
// shared by the single-image and the batched passes).
//
// Any N <= 2048 that is not 2^k or 3 * 2^k: each N-point line DFT is
// Bluestein's chirp-z form on an M-point line, M the smallest power of two
// >= 2N - 1.  With kn = (k^2 + n^2 - (k - n)^2) / 2, a DFT of exponent sign S
// is X_k = c_k sum_n (x_n c_n) b_(k-n), c_n = exp(S j pi n^2 / N),
// b_m = exp(-S j pi m^2 / N): a linear convolution evaluated as FFT_M ->
// multiply by FFT_M(b) / M -> inverse FFT_M.  The chirp phases come from the
// exact integer n^2 mod 2N; FFT_M(b) / M for both signs is a table
// computed once per (device, N, precision) in FP64 on the host.
#pragma once

#include "pass_kernels.hpp"

namespace nslct {
namespace {

template <typename T>
struct BsArgs {
    int N;               // line length
    const cplx<T>* tab;  // [0, M): S = -1, [M, 2M): S = +1
};

// exp(S j 2 pi r / (2N)) * scale, r = n^2 mod 2N (exact), in the working precision.
__device__ __forceinline__ cplx<float> bs_chirp(int r, int twoN, int S, float scale) {
    float t = (float)r / (float)twoN;
    if (t >= 0.5f) t -= 1.f;
    return {__builtin_amdgcn_cosf(t) * scale, (float)S * __builtin_amdgcn_sinf(t) * scale};
}
__device__ __forceinline__ cplx<double> bs_chirp(int r, int twoN, int S, double scale) {
    double sn, cs;
    sincospi(2.0 * (double)r / (double)twoN, &sn, &cs);
    return {cs * scale, (double)S * sn * scale};
}

// One pass on lines of length N through M-point Bluestein line DFTs, for
// the line tile `tile` of the image at sample offset img_off; the pass
// structure ([pre] DFT [mid] [DFT], remaps, centring) is that of pass_body,
// with every sample access restricted to positions < N.
template <typename T, int M, bool COL, int LINES>
__device__ __forceinline__ void bs_body(const PassArgs<T>& a, const BsArgs<T>& bs, int tile, size_t img_off,
                                        cplx<T>* lds_all) {
    constexpr int TPL = LinePlan<M>::TPL;
    using F = LineFFT<T, M, TPL>;
    constexpr int E = F::E;
    constexpr int R0 = F::R0;
    constexpr int LL = lds_line_elems<M>();

    const int N = bs.N, twoN = 2 * N;
    const int tid = threadIdx.x;
    const int slot = tid / TPL;
    const int t = tid % TPL;
    const int line = tile * LINES + slot;
    const int nl = a.nlines;
    const bool active = line < nl;
    cplx<T>* lds = lds_all + slot * LL;
    const cplx<T>* __restrict__ tab = twiddles<T>();
    const cplx<T>* __restrict__ in = a.in + img_off;
    cplx<T>* __restrict__ out = a.out + img_off;

    cplx<T> w[F::TW];
    F::preload(w, t, tab);
    auto pos = [&](int r) { return t + TPL * (r / R0) + (r % R0) * (M / R0); };
    auto to_store = [&](int p) { const int q = p + N / 2; return q >= N ? q - N : q; };
    auto addr = [&](int p) { return COL ? (size_t)p * nl + line : (size_t)line * N + p; };

    cplx<T> v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int p = pos(r);
        v[r] = (active && p < N) ? in[addr(a.load_remap ? to_store(p) : p)] : cplx<T>{0, 0};
    }

    const int lc = a.line_centered ? line - nl / 2 : (line >= (nl + 1) / 2 ? line - nl : line);
    const uint64_t l64 = (uint64_t)(int64_t)lc;
    auto chirp = [&](const ChirpArg& c, T scale) {
        const uint64_t A = (COL ? c.c22 : c.c11) * (l64 * l64) + c.c00;
        const uint64_t Bc = c.c12 * l64;
        const uint64_t Q = COL ? c.c11 : c.c22;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int64_t ks = p < (N + 1) / 2 ? p : p - N;
            const uint64_t k64 = (uint64_t)ks;
            const uint64_t ph = A + Bc * k64 + Q * (k64 * k64);
            if (p < N) v[r] = cmul(v[r], turns_cs(ph, scale));
        }
    };
    // N-point DFT of exponent sign S of the positions < N (natural order in
    // and out, zero beyond N).
    auto bdft = [&](int S) {
        const cplx<T>* __restrict__ bt = bs.tab + (S < 0 ? 0 : M);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int rr = (int)(((long long)p * p) % twoN);
            v[r] = p < N ? cmul(v[r], bs_chirp(rr, twoN, S, (T)1)) : cplx<T>{0, 0};
        }
        F::template dft<-1>(v, lds, t, w, tab);
#pragma unroll
        for (int r = 0; r < E; ++r) v[r] = cmul(v[r], bt[pos(r)]);
        F::template dft<+1>(v, lds, t, w, tab);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int rr = (int)(((long long)p * p) % twoN);
            v[r] = p < N ? cmul(v[r], bs_chirp(rr, twoN, S, (T)1)) : cplx<T>{0, 0};
        }
    };

    if (a.pre.on) chirp(a.pre, (T)1);
    const int ndft = a.has_t2 ? 2 : 1;
#pragma nounroll
    for (int k = 0; k < ndft; ++k) {
        bdft(k == 0 ? a.sign1 : a.sign2);
        if (k == 0 && a.mid_on) {
            if (a.mid.on) {
                chirp(a.mid, a.scale);
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) v[r] = {v[r].re * a.scale, v[r].im * a.scale};
            }
        }
    }

    if (active) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            if (p < N) out[addr(a.store_remap ? to_store(p) : p)] = v[r];
        }
    }
}


}  // namespace
}  // namespace nslct
