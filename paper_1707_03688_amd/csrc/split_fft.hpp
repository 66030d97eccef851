// Split-precision line DFTs on the matrix cores (gfx950).
//
// A radix-16 Stockham stage is the product Y = W16 X of the 16-point DFT
// matrix with the 16 x (N/16) matrix of (twiddled) butterfly inputs.  In real
// form, [Re Y; Im Y] = [[C, -S sin]; [S sin, C]] [Re X; Im X] is a 32 x 32 by
// 32 x M product, which v_mfma_f32_16x16x32_{f16,bf16} computes in two 16-row
// halves for 16 butterflies at a time.  Operands are split into a high and a
// low half-precision part, x = hi + lo with hi = rn(x) and lo = rn(x - hi),
// and the product is accumulated in FP32 as W_hi X_hi + W_hi X_lo + W_lo X_hi
// (the lo * lo term is below the half-precision rounding of the others).
//
// FP16 has a narrow exponent range (largest finite 65504): an unnormalised
// line DFT grows its values by up to 16 per radix-16 stage, and a 4096-long
// column pass starts from row DFT outputs that are up to 4096 times the
// image's mean.  Each butterfly's inputs are therefore scaled by a power of
// two 2^k (exact) so that their largest magnitude lies in [2^13, 2^14) before
// the split, and the FP32 products are scaled back by 2^-k.  The four lanes
// that supply one butterfly (one column of the B operand) share k.  BF16
// parts keep the FP32 exponent range and are not scaled.
//
// Operand layout of the 16x16x32 instruction (checked on the device): lane l
// holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7, and
// receives D[4 (l / 16) + e][l % 16], e = 0..3.  The K index is ordered
// (Re x_q, Im x_q) for q = 0..15, so lane (n = l % 16, g = l / 16) supplies the
// four inputs q = 4g..4g+3 of butterfly n, and the output rows of half h are
// ordered (Re y_r, Im y_r) for r = 8h..8h+7: lane (n, g) receives
// y_{8h+2g} and y_{8h+2g+1}.
#pragma once

#include "fft_engine.hpp"

namespace nslct {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int KIND>
struct SplitKind;
template <>
struct SplitKind<0> {  // FP16 parts
    using E = _Float16;
    using V = f16x8;
    __device__ __forceinline__ static f32x4 mma(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <>
struct SplitKind<1> {  // BF16 parts
    using E = __bf16;
    using V = bf16x8;
    __device__ __forceinline__ static f32x4 mma(V a, V b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// The two constant A operands (hi, lo) of one output half h and sign S.
template <int KIND>
struct SplitW {
    typename SplitKind<KIND>::V hi[2][2], lo[2][2];  // [sign index (0: -1, 1: +1)][half]

    __device__ __forceinline__ void init(int lane) {
        using Ek = typename SplitKind<KIND>::E;
        const int m = lane % 16;
        const int kb = 8 * (lane / 16);
#pragma unroll
        for (int si = 0; si < 2; ++si) {
            const float S = si == 0 ? -1.f : 1.f;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int r = 8 * h + m / 2;  // output index of this row
                const int cr = m % 2;         // 0: real part, 1: imaginary part
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = kb + e;
                    const int q = k / 2, ci = k % 2;
                    const int idx = ((r * q) % 16) * 12;  // 2 pi r q / 16 in 1/192 turns
                    const float c = (float)kCos192[idx];
                    const float s = (float)kCos192[(idx + 144) % 192];
                    float a;
                    if (cr == ci)
                        a = c;
                    else if (cr == 0)
                        a = -S * s;  // Re y <- Im x
                    else
                        a = S * s;   // Im y <- Re x
                    const Ek ah = (Ek)a;
                    hi[si][h][e] = ah;
                    lo[si][h][e] = (Ek)(a - (float)ah);
                }
            }
        }
    }
};

// One radix-16 stage on LDS-resident lines of length N: reads the stage's
// inputs (Stockham positions), twiddles them in FP32, multiplies on the
// matrix cores, writes the outputs.  `threads` = LINES * N / 16; every wave
// handles four groups of 16 butterflies.
template <int KIND, int S, int N, int LINES>
__device__ __forceinline__ void split_stage(cplx<float>* lds, int Ns, const SplitW<KIND>& W,
                                            const cplx<float>* __restrict__ tab) {
    using K = SplitKind<KIND>;
    using Ek = typename K::E;
    constexpr int LL = lds_line_elems<N>();
    constexpr int BPL = N / 16;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int n = lane % 16, g = lane / 16;
    const int si = S < 0 ? 0 : 1;
    cplx<float> y[4][4];
    int line_of[4], base_of[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int beta = 16 * (4 * wave + b) + n;  // butterfly index within the workgroup
        const int line = beta / BPL, j = beta % BPL;
        const int k = j % Ns;
        line_of[b] = line;
        base_of[b] = (j / Ns) * Ns * 16 + k;
        typename K::V bh, bl;
        cplx<float> xs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = 4 * g + e;
            cplx<float> x = lds[line * LL + lds_pad(j + q * (N / 16))];
            if (Ns > 1) {
                const int step = kTwiddleN / (16 * Ns);
                cplx<float> w = tab[((q * k) % (16 * Ns)) * step];
                if (S > 0) w.im = -w.im;
                x = cmul(x, w);
            }
            xs[e] = x;
        }
        int kexp = 0;
        if constexpr (KIND == 0) {
            float m = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e) m = fmaxf(m, fmaxf(fabsf(xs[e].re), fabsf(xs[e].im)));
            m = fmaxf(m, __shfl_xor(m, 16));
            m = fmaxf(m, __shfl_xor(m, 32));
            int ex;
            (void)frexpf(m, &ex);  // m in [2^(ex-1), 2^ex); ex = 0 for m = 0
            kexp = 14 - ex;
#pragma unroll
            for (int e = 0; e < 4; ++e) xs[e] = {ldexpf(xs[e].re, kexp), ldexpf(xs[e].im, kexp)};
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const Ek hr = (Ek)xs[e].re, hi_ = (Ek)xs[e].im;
            bh[2 * e] = hr;
            bh[2 * e + 1] = hi_;
            bl[2 * e] = (Ek)(xs[e].re - (float)hr);
            bl[2 * e + 1] = (Ek)(xs[e].im - (float)hi_);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            d = K::mma(W.hi[si][h], bh, d);
            d = K::mma(W.hi[si][h], bl, d);
            d = K::mma(W.lo[si][h], bh, d);
            if constexpr (KIND == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) d[c] = ldexpf(d[c], -kexp);
            }
            y[b][2 * h] = {d[0], d[1]};      // y_{8h+2g}
            y[b][2 * h + 1] = {d[2], d[3]};  // y_{8h+2g+1}
        }
    }
    __syncthreads();  // every input read before any output lands
#pragma unroll
    for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int o = 0; o < 2; ++o) {
                const int r = 8 * h + 2 * g + o;
                lds[line_of[b] * LL + lds_pad(base_of[b] + r * Ns)] = y[b][2 * h + o];
            }
    }
    __syncthreads();
}

// Full line DFT (N = 16^P) of every line in LDS, natural order in and out.
template <int KIND, int S, int N, int LINES>
__device__ __forceinline__ void split_dft(cplx<float>* lds, const SplitW<KIND>& W, const cplx<float>* __restrict__ tab) {
    static_assert(N == 256 || N == 4096, "split-precision lines are 16^2 or 16^3 long");
#pragma unroll
    for (int Ns = 1; Ns < N; Ns *= 16) split_stage<KIND, S, N, LINES>(lds, Ns, W, tab);
}

}  // namespace nslct
