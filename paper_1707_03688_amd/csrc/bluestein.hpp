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

// Line plan of the M-point lines: the alternative split of a 256-point line
// (8 samples on each of 32 threads instead of 16 on 16) is faster at every
// size measured on gfx950 (one 100^2 complex64 image 65.4 -> 40.1 us,
// complex128 105.9 -> 61.0; 75^2 59.1 -> 37.2), the other lengths' are
// slower (128: 46.9 -> 69.4 us at 40^2; 512, 1024: about 2x).
template <int M>
using BsPlan = PlanVariant<M, (M == 256 ? 1 : 0)>;

// Lines per tile of a Bluestein pass: row tiles of 256 threads, column
// tiles with the thread count of the single-image column tile.
template <typename T, int M, bool COL>
constexpr int bs_tile_lines() {
    constexpr int TPL = BsPlan<M>::TPL;
    return COL ? (col_lines<T, M>() * LinePlan<M>::TPL + TPL - 1) / TPL : row_lines_of<BsPlan<M>>();
}

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
// with every sample access restricted to positions < N.  NS = 2: the
// backward sweep's two signals (a.in / a.out and a.in2 / a.out2) through the
// same steps, with the gradient sums of pass_body at the chirp point.
template <typename T, int M, bool COL, int LINES, int NS = 1>
__device__ __forceinline__ void bs_body(const PassArgs<T>& a, const BsArgs<T>& bs, int tile, size_t img_off,
                                        cplx<T>* lds_all) {
    constexpr int TPL = BsPlan<M>::TPL;
    using F = LineFFT<T, M, TPL, typename BsPlan<M>::L>;
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
    const cplx<T>* ins[2] = {a.in + img_off, NS > 1 ? a.in2 + img_off : nullptr};
    cplx<T>* outs[2] = {a.out + img_off, NS > 1 ? a.out2 + img_off : nullptr};

    cplx<T> w[F::TW];
    F::preload(w, t, tab);
    auto pos = [&](int r) { return t + TPL * (r / R0) + (r % R0) * (M / R0); };
    auto to_store = [&](int p) { const int q = p + N / 2; return q >= N ? q - N : q; };
    auto addr = [&](int p) { return COL ? (size_t)p * nl + line : (size_t)line * N + p; };
    // Signed index along the line of FFT-order position p (as the chirps use it).
    auto signed_k = [&](int p) { return p < (N + 1) / 2 ? p : p - N; };

    cplx<T> v[NS][E];
#pragma unroll
    for (int sg = 0; sg < NS; ++sg)
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            v[sg][r] = (active && p < N) ? ins[sg][addr(a.load_remap ? to_store(p) : p)] : cplx<T>{0, 0};
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
            const uint64_t k64 = (uint64_t)(int64_t)signed_k(p);
            const uint64_t ph = A + Bc * k64 + Q * (k64 * k64);
            const cplx<T> f = turns_cs(ph, scale);
#pragma unroll
            for (int sg = 0; sg < NS; ++sg)
                if (p < N) v[sg][r] = cmul(v[sg][r], f);
        }
    };
    auto scale_all = [&](T sc) {
#pragma unroll
        for (int sg = 0; sg < NS; ++sg)
#pragma unroll
            for (int r = 0; r < E; ++r) v[sg][r] = {v[sg][r].re * sc, v[sg][r].im * sc};
    };
    // N-point DFT of exponent sign S of the positions < N (natural order in
    // and out, zero beyond N), of signal sg.
    auto bdft = [&](int S, int sg) {
        const cplx<T>* __restrict__ bt = bs.tab + (S < 0 ? 0 : M);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int rr = (int)(((long long)p * p) % twoN);
            v[sg][r] = p < N ? cmul(v[sg][r], bs_chirp(rr, twoN, S, (T)1)) : cplx<T>{0, 0};
        }
        F::template dft<-1>(v[sg], lds, t, w, tab);
#pragma unroll
        for (int r = 0; r < E; ++r) v[sg][r] = cmul(v[sg][r], bt[pos(r)]);
        F::template dft<+1>(v[sg], lds, t, w, tab);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int rr = (int)(((long long)p * p) % twoN);
            v[sg][r] = p < N ? cmul(v[sg][r], bs_chirp(rr, twoN, S, (T)1)) : cplx<T>{0, 0};
        }
    };
    // Backward sweep: at the chirp point, sum Im(conj(adjoint) * signal)
    // weighted by x^2, x y, y^2 (signed sample indices) into a.acc[0..2].
    auto gradient_sums = [&]() {
        if constexpr (NS == 2) {
            double sxx = 0, sxy = 0, syy = 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int p = pos(r);
                if (p >= N) continue;
                const double e = (double)signed_k(p);
                const double xi = COL ? e : (double)lc;
                const double yi = COL ? (double)lc : e;
                const double im = (double)v[1][r].re * (double)v[0][r].im - (double)v[1][r].im * (double)v[0][r].re;
                sxx += xi * xi * im;
                sxy += xi * yi * im;
                syy += yi * yi * im;
            }
            block_sum3(sxx, sxy, syy, a.acc);
        }
    };

    if constexpr (NS == 1) {
        if (a.pre.on) chirp(a.pre, (T)1);
        const int ndft = a.has_t2 ? 2 : 1;
#pragma nounroll
        for (int k = 0; k < ndft; ++k) {
            bdft(k == 0 ? a.sign1 : a.sign2, 0);
            if (k == 0 && a.mid_on) {
                if (a.mid.on)
                    chirp(a.mid, a.scale);
                else
                    scale_all(a.scale);
            }
        }
    } else {
        if (!a.mid_on) gradient_sums();
        if (a.pre.on) chirp(a.pre, (T)1);
#pragma unroll
        for (int sg = 0; sg < NS; ++sg) bdft(a.sign1, sg);
        if (a.mid_on) {
            gradient_sums();
            if (a.mid.on)
                chirp(a.mid, a.scale);
            else
                scale_all(a.scale);
        }
        if (a.has_t2) {
#pragma unroll
            for (int sg = 0; sg < NS; ++sg) bdft(a.sign2, sg);
        }
    }

    if (active) {
#pragma unroll
        for (int sg = 0; sg < NS; ++sg)
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int p = pos(r);
                if (p < N) outs[sg][addr(a.store_remap ? to_store(p) : p)] = v[sg][r];
            }
    }
}


}  // namespace
}  // namespace nslct
