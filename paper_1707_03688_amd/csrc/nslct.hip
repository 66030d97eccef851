// Fused HIP passes of the 2D HA-NsDLCT for gfx950, and the C ABI.
//
// The chain (Pei & Huang, Sec. 4.2.1 eq. HA28 / Sec. 4.3 eq. CCCMCCCM40) is
// run in the five-slot form
//   G = CM(S4) U^H CM_w(C3) U CM(S2) U^H CM_w(C1) U CM(S0) g
// where U = Ux Uy is the unitary centred 2D DFT, CM the discrete chirp
// multiplication (eq. BasicCM12) on the space grid and CM_w the same on the
// frequency grid (the transfer function of the CC, eq. BasicCC20).  The
// paper's DFT constants dx dy/(j 2 pi) make each CC equal to -U^H CM_w U, so
// the two CCs of a chain multiply to +1 and the unitary form is exact.
// Since Ux and Uy commute, the chain splits into five axis-homogeneous passes,
// each one HBM read and one HBM write of the image:
//   pass 0 rows (y): [CM(S0)] -> FFT_y
//   pass 1 cols (x): FFT_x -> CM_w(C1) / Nx -> IFFT_x
//   pass 2 rows (y): IFFT_y -> CM(S2) / Ny -> FFT_y
//   pass 3 cols (x): FFT_x -> CM_w(C3) / Nx -> IFFT_x
//   pass 4 rows (y): IFFT_y -> CM(S4) / Ny
// Rows are contiguous lines; columns are read as tiles of adjacent columns so
// each row segment is a coalesced burst.  Centred <-> FFT index order is folded
// into load/store addressing: the y axis is centred at pass-0 load and pass-4
// store, the x axis at pass-1 load and pass-3 store; in between the axes stay
// in FFT order.  Chirp phases are exact: 64-bit fixed-point turns times exact
// integer sample indices, wrapping modulo one turn, then sin/cos of the
// reduced angle in the working precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <mutex>
#include <vector>
#include <new>
#include <string>

#include "fft_engine.hpp"
#include "nslct.h"
#include "planner.hpp"
#include "split_fft.hpp"

using namespace nslct;

struct nslct_plan_s {
    PlanData d;
};

struct nslct_batch_s;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// ---------------------------------------------------------------- device data
__device__ cplx<float> g_twf[kTwiddleN];
__device__ cplx<double> g_twd[kTwiddleN];

template <typename T>
__device__ __forceinline__ const cplx<T>* twiddles();
template <>
__device__ __forceinline__ const cplx<float>* twiddles<float>() {
    return g_twf;
}
template <>
__device__ __forceinline__ const cplx<double>* twiddles<double>() {
    return g_twd;
}

__global__ void init_twiddles_kernel() {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < kTwiddleN) {
        double s, c;
        sincospi(2.0 * k / kTwiddleN, &s, &c);  // 2k/NT is exact in FP64
        g_twd[k] = {c, -s};
        g_twf[k] = {(float)c, (float)-s};
    }
}

struct ChirpArg {
    uint64_t c11, c12, c22;
    int on;
};

template <typename T>
struct PassArgs {
    const cplx<T>* in;
    cplx<T>* out;
    long long img_stride;  // samples between consecutive images
    int nlines;            // lines in this pass = length of the other axis
    int load_remap;        // centred -> FFT order along the line at load
    int store_remap;       // FFT -> centred order along the line at store
    int line_centered;     // line index is in centred (1) or FFT (0) order
    int sign1;             // exponent sign of the first line DFT
    int has_t2;            // a second line DFT follows the pointwise product
    int sign2;
    int mid_on;            // pointwise product after the first DFT
    ChirpArg pre, mid;
    T scale;               // folded into the pointwise product
    int post_on;           // reduced schedules (X3 kernels): pointwise product
    int sign3;             // after the second DFT, then a third DFT
    ChirpArg post;
    T scale2;
    const cplx<T>* in2;    // backward sweep: second signal (adjoint) ...
    cplx<T>* out2;
    double* acc;           // ... and the three gradient sums of this pass
};

// Sum of three doubles over the workgroup, added atomically to acc[0..2].
__device__ __forceinline__ void block_sum3(double a0, double a1, double a2, double* acc) {
    __shared__ double red[3][16];
    for (int off = 32; off > 0; off >>= 1) {
        a0 += __shfl_xor(a0, off);
        a1 += __shfl_xor(a1, off);
        a2 += __shfl_xor(a2, off);
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int nw = (blockDim.x + 63) / 64;
    __syncthreads();
    if (lane == 0) {
        red[0][wave] = a0;
        red[1][wave] = a1;
        red[2][wave] = a2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0;
        for (int k = 0; k < nw; ++k) s += red[threadIdx.x][k];
        atomicAdd(acc + threadIdx.x, s);
    }
    __syncthreads();
}

// sin/cos of 2 pi * phase, phase in 64-bit fixed-point turns, times scale.
// FP32: the top 32 bits as a float in [-1/2, 1/2) turns and the hardware
// sine / cosine, which take their argument in turns (measured on gfx950:
// max abs error 1.3e-7 over the whole range).  FP64: all 64 bits and sincospi.
__device__ __forceinline__ cplx<float> turns_cs(uint64_t ph, float scale) {
    const float t = (float)(int32_t)(ph >> 32) * 0x1p-32f;
    return {__builtin_amdgcn_cosf(t) * scale, __builtin_amdgcn_sinf(t) * scale};
}
__device__ __forceinline__ cplx<double> turns_cs(uint64_t ph, double scale) {
    const double t = (double)(int64_t)ph * 0x1p-64;
    double s, c;
    sincospi(2.0 * t, &s, &c);
    return {c * scale, s * scale};
}

// Workgroups are dispatched round-robin over the 8 XCDs; give consecutive
// column tiles (which share cache lines) to workgroups of the same XCD.
__device__ __forceinline__ int xcd_tile(int b, int G) {
    if ((G & 7) != 0) return b;
    return (b & 7) * (G >> 3) + (b >> 3);
}

// Centred <-> FFT order along an N-point line: FFT index i sits at storage
// position (i + floor(N/2)) mod N.
template <int N>
__device__ __forceinline__ int fft_to_store(int i) {
    const int p = i + N / 2;
    return p >= N ? p - N : p;
}
template <int N>
__device__ __forceinline__ int store_to_fft(int p) {
    const int i = p + (N + 1) / 2;
    return i >= N ? i - N : i;
}

// One fused pass over LINES lines of length N per workgroup.  Row passes
// (COL = false) read and write contiguous lines directly.  Column passes
// cover a tile of LINES adjacent columns; their stores (and, for lines
// longer than a wavefront, their loads) are staged through LDS so that the
// global accesses cover LINES consecutive samples of each row (coalesced),
// while each line's FFT work stays with the TPL threads that own it.
template <typename T, int N, bool COL, int LINES, int NS = 1, bool X3 = false>
__device__ __forceinline__ void pass_body(const PassArgs<T>& a, int tile, size_t img_off, cplx<T>* lds_all) {
    constexpr int TPL = LinePlan<N>::TPL;
    using F = LineFFT<T, N, TPL>;
    constexpr int E = F::E;
    constexpr int R0 = F::R0;
    constexpr int LL = lds_line_elems<N>();

    const int tid = threadIdx.x;
    const int slot = tid / TPL;
    const int t = tid % TPL;
    const int line0 = tile * LINES;
    const int line = line0 + slot;
    const int nl = a.nlines;
    const bool active = line < nl;
    cplx<T>* lds = lds_all + slot * LL;
    const cplx<T>* __restrict__ tab = twiddles<T>();
    const cplx<T>* ins[2] = {a.in + img_off, NS > 1 ? a.in2 + img_off : nullptr};
    cplx<T>* outs[2] = {a.out + img_off, NS > 1 ? a.out2 + img_off : nullptr};

    cplx<T> w[F::TW];
    F::preload(w, t, tab);

    auto pos = [&](int r) { return t + TPL * (r / R0) + (r % R0) * (N / R0); };

    // NS signals go through identical arithmetic (NS = 2: the forward output
    // and the adjoint of a backward sweep).
    cplx<T> v[NS][E];
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
        const cplx<T>* __restrict__ in = ins[sg];
        if constexpr (COL && F::kWave) {
            // Lines owned by one wavefront: each lane loads its own column
            // samples directly.  The tile's other columns are read by the
            // neighbouring wavefronts of the workgroup at the same time, so
            // the 32-byte row segments are still served by one cache line,
            // and no workgroup barrier couples the wavefronts before their
            // FFTs (measured faster than staging through LDS at N <= 1024).
            if (active) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int p = pos(r);
                    const int src = a.load_remap ? fft_to_store<N>(p) : p;
                    v[sg][r] = in[(size_t)src * nl + line];
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) v[sg][r] = {0, 0};
            }
        } else if constexpr (COL) {
            // Coalesced tile load: lane -> (column c, row group u).
            const int c = tid % LINES;
            const int u = tid / LINES;
            const bool cok = line0 + c < nl;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int p = u + TPL * k;
                const int i = a.load_remap ? store_to_fft<N>(p) : p;
                lds_all[c * LL + lds_pad(i)] = cok ? in[(size_t)p * nl + line0 + c] : cplx<T>{0, 0};
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < E; ++r) v[sg][r] = lds[lds_pad(pos(r))];
            __syncthreads();
        } else {
            if (active) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int p = pos(r);
                    const int src = a.load_remap ? fft_to_store<N>(p) : p;
                    v[sg][r] = in[(size_t)line * N + src];
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) v[sg][r] = {0, 0};
            }
        }
    }

    const int lc = a.line_centered ? line - nl / 2 : (line >= (nl + 1) / 2 ? line - nl : line);
    // Signed index along the line of register r: t + d(r) with d(r) known at
    // compile time (the wrap to negative indices happens exactly for the
    // upper half of the first-stage radix).
    auto offs = [&](int r) {
        const int q = r % R0;
        return TPL * (r / R0) + (N / R0) * (q < R0 / 2 ? q : q - R0);
    };
    // Chirp exp(j 2 pi phi) with phi = c11 m^2 + c12 m n + c22 n^2 (turns),
    // all in exact 64-bit turns: phi = phi_t + d alpha_t + d^2 Q for the
    // register at signed offset d from t.  The registers i R0 .. i R0 + R0 - 1
    // sit at d = TPL i + M s, s = -R0/2 .. R0/2 - 1 (M = N / R0), so along s
    // phi is advanced by exact second-order differences (two 64-bit adds per
    // sample).
    auto chirp = [&](const ChirpArg& c, T scale) {
        const uint64_t l64 = (uint64_t)(int64_t)lc;
        const uint64_t A = (COL ? c.c22 : c.c11) * (l64 * l64);
        const uint64_t Bc = c.c12 * l64;
        const uint64_t Q = COL ? c.c11 : c.c22;
        const uint64_t t64 = (uint64_t)t;
        const uint64_t phi_t = A + Bc * t64 + Q * (t64 * t64);
        const uint64_t alpha = Bc + 2 * Q * t64;
        constexpr int M = N / R0;
        const uint64_t dd = Q * (uint64_t)(2 * M * M);
#pragma unroll
        for (int i = 0; i < E / R0; ++i) {
            constexpr int h = R0 / 2;
            const int64_t d0 = (int64_t)TPL * i - (int64_t)M * h;
            uint64_t ph = phi_t + alpha * (uint64_t)d0 + Q * (uint64_t)(d0 * d0);
            uint64_t df = alpha * (uint64_t)M + Q * (uint64_t)(2 * d0 * M + (int64_t)M * M);
#pragma unroll
            for (int sidx = 0; sidx < R0; ++sidx) {
                const int q = sidx < h ? sidx + h : sidx - h;  // register of s = sidx - h
                const cplx<T> f = turns_cs(ph, scale);
#pragma unroll
                for (int sg = 0; sg < NS; ++sg) v[sg][i * R0 + q] = cmul(v[sg][i * R0 + q], f);
                ph += df;
                df += dd;
            }
        }
    };
    // Backward sweep: at the chirp point, sum Im(conj(adjoint) * signal)
    // weighted by x^2, x y, y^2 (signed sample indices) into a.acc[0..2].
    auto gradient_sums = [&]() {
        if constexpr (NS == 2) {
            double sxx = 0, sxy = 0, syy = 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const double e = (double)(t + offs(r));
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
        // The pass as a sequence of steps, each a pointwise product (pre
        // chirp; mid chirp or scale; post chirp or scale) followed by a line
        // DFT (the middle step's DFT only when has_t2).  The step loop stays
        // rolled and every DFT runs through one copy of the sign +1 code (a
        // sign -1 DFT is the conjugate of the sign +1 DFT of the conjugate),
        // so a pass executes one copy of the DFT and chirp code however many
        // steps it has: each launch fetches its instructions from L2 again,
        // and this measured 1.2 us faster per 1024-long column pass.
        const int nsteps = X3 ? 3 : 2;
#pragma nounroll
        for (int k = 0; k < nsteps; ++k) {
            const bool step_on = k == 0 ? a.pre.on : (k == 1 ? a.mid_on : a.post_on);
            if (step_on) {
                const ChirpArg c = k == 0 ? a.pre : (k == 1 ? a.mid : a.post);
                const T sc = k == 0 ? (T)1 : (k == 1 ? a.scale : a.scale2);
                if (c.on) {
                    chirp(c, sc);
                } else {
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                        for (int r = 0; r < E; ++r) v[sg][r] = {v[sg][r].re * sc, v[sg][r].im * sc};
                }
            }
            const bool dft_on = k != 1 || a.has_t2;
            if (dft_on) {
                const bool neg = (k == 0 ? a.sign1 : (k == 1 ? a.sign2 : a.sign3)) < 0;
#pragma unroll
                for (int sg = 0; sg < NS; ++sg) {
                    if (neg) {
#pragma unroll
                        for (int r = 0; r < E; ++r) v[sg][r].im = -v[sg][r].im;
                    }
                    F::template dft<+1>(v[sg], lds, t, w, tab);
                    if (neg) {
#pragma unroll
                        for (int r = 0; r < E; ++r) v[sg][r].im = -v[sg][r].im;
                    }
                }
            }
        }
    } else {
        // Two signals (backward sweep): the same steps written out, both DFT
        // signs compiled (a rolled loop needs more registers here).
        if (NS == 2 && !a.mid_on) gradient_sums();
        if (a.pre.on) chirp(a.pre, (T)1);
#pragma unroll
        for (int sg = 0; sg < NS; ++sg) {
            if (a.sign1 < 0)
                F::template dft<-1>(v[sg], lds, t, w, tab);
            else
                F::template dft<+1>(v[sg], lds, t, w, tab);
        }
        if (a.mid_on) {
            if (NS == 2) gradient_sums();
            if (a.mid.on) {
                chirp(a.mid, a.scale);
            } else {
#pragma unroll
                for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                    for (int r = 0; r < E; ++r) v[sg][r] = {v[sg][r].re * a.scale, v[sg][r].im * a.scale};
            }
        }
        if (a.has_t2) {
#pragma unroll
            for (int sg = 0; sg < NS; ++sg) {
                if (a.sign2 < 0)
                    F::template dft<-1>(v[sg], lds, t, w, tab);
                else
                    F::template dft<+1>(v[sg], lds, t, w, tab);
            }
        }
        if constexpr (X3) {
            // Reduced schedules: a second pointwise product and a third DFT.
            if (a.post_on) {
                if (a.post.on) {
                    chirp(a.post, a.scale2);
                } else {
#pragma unroll
                    for (int sg = 0; sg < NS; ++sg)
#pragma unroll
                        for (int r = 0; r < E; ++r) v[sg][r] = {v[sg][r].re * a.scale2, v[sg][r].im * a.scale2};
                }
            }
#pragma unroll
            for (int sg = 0; sg < NS; ++sg) {
                if (a.sign3 < 0)
                    F::template dft<-1>(v[sg], lds, t, w, tab);
                else
                    F::template dft<+1>(v[sg], lds, t, w, tab);
            }
        }
    }

#pragma unroll
    for (int sg = 0; sg < NS; ++sg) {
        cplx<T>* __restrict__ out = outs[sg];
        if constexpr (COL) {
            // Before the first signal's staging each line's LDS region has
            // only been used by that line's own threads, whose last DFT
            // exchange ended with their sync; a second signal reuses regions
            // the whole tile has just read.
            if (sg > 0) __syncthreads();
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int p = pos(r);
                lds[lds_pad(a.store_remap ? fft_to_store<N>(p) : p)] = v[sg][r];
            }
            __syncthreads();
            const int c = tid % LINES;
            const int u = tid / LINES;
            if (line0 + c < nl) {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int p = u + TPL * k;
                    out[(size_t)p * nl + line0 + c] = lds_all[c * LL + lds_pad(p)];
                }
            }
        } else if (active) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int p = pos(r);
                const int dst = a.store_remap ? fft_to_store<N>(p) : p;
                out[(size_t)line * N + dst] = v[sg][r];
            }
        }
    }
}


// Single-plan pass: blockIdx.x = line tile, blockIdx.y = image.
template <typename T, int N, bool COL, int LINES, bool X3 = false>
__global__ void __launch_bounds__(LinePlan<N>::TPL* LINES) nslct_pass(PassArgs<T> a) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<N>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    pass_body<T, N, COL, LINES, 1, X3>(a, tile, (size_t)blockIdx.y * a.img_stride, lds_all);
}

template <typename T, int N>
constexpr int row_lines() {
    return LinePlan<N>::TPL >= 256 ? 1 : 256 / LinePlan<N>::TPL;
}
// Columns per tile: 4 (complex64) or 2 (complex128) adjacent columns, so a
// row segment is 32 bytes, but no more than 512 threads per workgroup: a
// 4096-long complex64 tile of 4 columns (1024 threads, 139 KB of LDS, one
// workgroup per CU in lock step) measured 1.6x slower than 2 columns.  (The
// chain's 4096-long column passes run in three steps instead; these tiles
// serve the reduced schedules and the other lengths.)
template <typename T, int N>
constexpr int col_lines() {
    constexpr int TPL = LinePlan<N>::TPL;
    constexpr int cmin = sizeof(T) == 4 ? 4 : 2;
    constexpr int cap = 512 / TPL;
    constexpr int c = cmin < cap ? cmin : cap;
    return 256 / TPL > c ? 256 / TPL : c;
}

template <typename T, int N, bool COL, bool X3 = false>
hipError_t launch_t(const PassArgs<T>& a, int count, hipStream_t s) {
    constexpr int L = COL ? col_lines<T, N>() : row_lines<T, N>();
    static_assert(L * lds_line_elems<N>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    dim3 grid((a.nlines + L - 1) / L, count);
    dim3 block(LinePlan<N>::TPL * L);
    hipLaunchKernelGGL((nslct_pass<T, N, COL, L, X3>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T, bool COL, bool X3 = false>
hipError_t launch_n(int N, const PassArgs<T>& a, int count, hipStream_t s) {
    switch (N) {
        case 2: return launch_t<T, 2, COL, X3>(a, count, s);
        case 6: return launch_t<T, 6, COL, X3>(a, count, s);
        case 12: return launch_t<T, 12, COL, X3>(a, count, s);
        case 24: return launch_t<T, 24, COL, X3>(a, count, s);
        case 48: return launch_t<T, 48, COL, X3>(a, count, s);
        case 96: return launch_t<T, 96, COL, X3>(a, count, s);
        case 192: return launch_t<T, 192, COL, X3>(a, count, s);
        case 384: return launch_t<T, 384, COL, X3>(a, count, s);
        case 768: return launch_t<T, 768, COL, X3>(a, count, s);
        case 4: return launch_t<T, 4, COL, X3>(a, count, s);
        case 8: return launch_t<T, 8, COL, X3>(a, count, s);
        case 16: return launch_t<T, 16, COL, X3>(a, count, s);
        case 32: return launch_t<T, 32, COL, X3>(a, count, s);
        case 64: return launch_t<T, 64, COL, X3>(a, count, s);
        case 128: return launch_t<T, 128, COL, X3>(a, count, s);
        case 256: return launch_t<T, 256, COL, X3>(a, count, s);
        case 512: return launch_t<T, 512, COL, X3>(a, count, s);
        case 1024: return launch_t<T, 1024, COL, X3>(a, count, s);
        case 2048: return launch_t<T, 2048, COL, X3>(a, count, s);
        case 4096: return launch_t<T, 4096, COL, X3>(a, count, s);
        default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------- 4096-long columns, in three steps
// A column pass over 4096-long columns (FFT -> pointwise product -> inverse
// FFT) as three launches over 64 x 64 blocks of each column, so that every
// global access covers whole 128-byte row segments instead of the 16-byte
// segments of a 2-column whole-column tile, which waste most of every L2
// request.  With n = n1 + 64 n2,
// k = k2 + 64 k1, m = m1 + 64 m2 (all in [0, 64)) and W = exp(S 2 pi j / 4096):
//   A: for each n1, Y[k2] = W^(n1 k2) sum_n2 x[n1 + 64 n2] w64^(n2 k2),
//      stored at row n1 + 64 k2 (rows = n1 mod 64, a strided gather);
//   B: for each k2 (64 contiguous rows): X[k2 + 64 k1] = sum_n1 Y w64^(n1 k1)
//      is the first line DFT; the pointwise product at k; then
//      U[m1] = W'^(k2 m1) sum_k1 X[k2 + 64 k1] w64'^(k1 m1) (second sign),
//      stored at row m1 + 64 k2;
//   C: for each m1, Z[m1 + 64 m2] = sum_k2 U w64'^(k2 m2), the second line
//      DFT, stored at row m (with the FFT -> centred remap if asked).
// Each step is in place over a disjoint set of rows and columns per
// workgroup.  A workgroup covers 128 bytes of every row it touches (16
// complex64 or 8 complex128 columns) so that no cache line is split between
// workgroups (consecutive workgroups run on different XCDs); each wavefront
// holds 8 columns x 8 threads, each thread 8 of a column's 64 samples.
template <typename T>
constexpr int fs_cols() {
    return 128 / (int)sizeof(cplx<T>);
}

// x * exp(S 2 pi j e / 4096) from the forward-sign table (W_12288).
template <typename T>
__device__ __forceinline__ cplx<T> fs_twiddle(cplx<T> x, int e, int S, const cplx<T>* __restrict__ tab) {
    cplx<T> w = tab[(e & 4095) * (kTwiddleN / 4096)];
    if (S > 0) w.im = -w.im;
    return cmul(x, w);
}

// 64-point line DFT of sign S over the registers (positions t + 8 i), the
// sign -1 case as the conjugate of the sign +1 DFT of the conjugate.
template <typename T>
__device__ __forceinline__ void fs_dft64(cplx<T>* v, cplx<T>* lds, int t, const cplx<T>* w,
                                         const cplx<T>* __restrict__ tab, int S) {
    using F = LineFFT<T, 64, 8>;
    if (S < 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r].im = -v[r].im;
    }
    F::template dft<+1>(v, lds, t, w, tab);
    if (S < 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r].im = -v[r].im;
    }
}

// STEP 0 = A, 1 = B, 2 = C.  blockIdx.x = column block + ncb * (block row
// index n1 / k2 / m1), blockIdx.y = image.
template <typename T, int STEP>
__global__ void __launch_bounds__(8 * fs_cols<T>()) nslct_col4096_step(PassArgs<T> a, int ncb) {
    using F = LineFFT<T, 64, 8>;
    static_assert(F::E == 8 && F::R0 == 8, "64-point plan: 8 threads x 8 samples");
    constexpr int N = 4096;
    constexpr int CB = fs_cols<T>();
    __shared__ cplx<T> lds_all[CB * lds_line_elems<64>()];
    const int tid = threadIdx.x;
    const int cl = 8 * (tid / 64) + tid % 8;  // column within the block
    const int t = (tid % 64) / 8;             // thread within the column's 64-point line
    const int cb = blockIdx.x % ncb;
    const int j = blockIdx.x / ncb;  // n1 (A), k2 (B) or m1 (C)
    const int nl = a.nlines;
    const int c = cb * CB + cl;
    const bool active = c < nl;
    const size_t img = (size_t)blockIdx.y * a.img_stride;
    const cplx<T>* __restrict__ in = (STEP == 0 ? a.in : a.out) + img;
    cplx<T>* __restrict__ out = a.out + img;
    cplx<T>* lds = lds_all + cl * lds_line_elems<64>();
    const cplx<T>* __restrict__ tab = twiddles<T>();
    cplx<T> w[F::TW];
    F::preload(w, t, tab);

    // Register i holds block position t + 8 i; its image row:
    auto row = [&](int i) {
        const int b = t + 8 * i;
        if constexpr (STEP == 0) {
            const int n = j + 64 * b;
            return a.load_remap ? fft_to_store<N>(n) : n;
        } else if constexpr (STEP == 1) {
            return 64 * j + b;
        } else {
            return j + 64 * b;
        }
    };
    cplx<T> v[8];
    if (active) {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = in[(size_t)row(i) * nl + c];
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = {0, 0};
    }

    if constexpr (STEP == 0) {
        fs_dft64(v, lds, t, w, tab, a.sign1);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = fs_twiddle(v[i], j * (t + 8 * i), a.sign1, tab);
    } else if constexpr (STEP == 1) {
        fs_dft64(v, lds, t, w, tab, a.sign1);
        // Register i now holds k1 = t + 8 i, i.e. FFT index k = j + 64 k1.
        const int lc = a.line_centered ? c - nl / 2 : (c >= (nl + 1) / 2 ? c - nl : c);
        const uint64_t l64 = (uint64_t)(int64_t)lc;
        const uint64_t A0 = a.mid.c22 * (l64 * l64);
        const uint64_t Bc = a.mid.c12 * l64;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (a.mid.on) {
                const int k = j + 64 * (t + 8 * i);
                const int64_t e = k < N / 2 ? k : k - N;
                const uint64_t e64 = (uint64_t)e;
                const uint64_t ph = A0 + Bc * e64 + a.mid.c11 * (e64 * e64);
                v[i] = cmul(v[i], turns_cs(ph, a.scale));
            } else {
                v[i] = {v[i].re * a.scale, v[i].im * a.scale};
            }
        }
        fs_dft64(v, lds, t, w, tab, a.sign2);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = fs_twiddle(v[i], j * (t + 8 * i), a.sign2, tab);
    } else {
        fs_dft64(v, lds, t, w, tab, a.sign2);
    }

    if (active) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int b = t + 8 * i;
            int r;
            if constexpr (STEP == 0) {
                r = j + 64 * b;
            } else if constexpr (STEP == 1) {
                r = 64 * j + b;
            } else {
                const int m = j + 64 * b;
                r = a.store_remap ? fft_to_store<N>(m) : m;
            }
            out[(size_t)r * nl + c] = v[i];
        }
    }
}

// The column pass of the five-slot chain (first DFT, pointwise product,
// second DFT; no product before the first DFT) on 4096-long columns.
template <typename T>
bool col4096_applies(const PassArgs<T>& a, int N) {
    return N == 4096 && a.has_t2 && a.mid_on && !a.pre.on;
}

template <typename T>
hipError_t launch_col4096(const PassArgs<T>& a, int count, hipStream_t s) {
    constexpr int CB = fs_cols<T>();
    const int ncb = (a.nlines + CB - 1) / CB;
    const dim3 grid(ncb * 64, count), block(8 * CB);
    hipLaunchKernelGGL((nslct_col4096_step<T, 0>), grid, block, 0, s, a, ncb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((nslct_col4096_step<T, 1>), grid, block, 0, s, a, ncb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((nslct_col4096_step<T, 2>), grid, block, 0, s, a, ncb);
    return hipGetLastError();
}

// Per-device one-time setup (twiddle tables).
std::mutex g_init_mu;
bool g_inited[64] = {};

int ensure_device_ready() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(NSLCT_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_inited[dev]) return NSLCT_OK;
    hipLaunchKernelGGL(init_twiddles_kernel, dim3((kTwiddleN + 255) / 256), dim3(256), 0, 0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("twiddle init: ") + hipGetErrorString(e));
    g_inited[dev] = true;
    return NSLCT_OK;
}

ChirpArg to_arg(const ChirpTurns& c) { return {c.c11, c.c12, c.c22, c.nonzero}; }

// Arguments of pass `pass` (0..4) of the five-slot chain whose chirps are
// `turns[0..4]`, for an Nx x Ny image (host and device).
template <typename T>
__host__ __device__ inline PassArgs<T> make_pass_args(int Nx, int Ny, const ChirpArg* turns, int pass,
                                                     const void* in, void* out) {
    PassArgs<T> a{};
    a.in = (const cplx<T>*)in;
    a.out = (cplx<T>*)out;
    a.img_stride = (long long)Nx * Ny;
    const bool col = (pass == 1 || pass == 3);
    a.nlines = col ? Ny : Nx;
    a.pre.on = 0;
    a.mid.on = 0;
    a.scale = (T)1;
    switch (pass) {
        case 0:
            a.load_remap = 1;
            a.line_centered = 1;
            a.pre = turns[0];
            a.sign1 = -1;
            break;
        case 1:
        case 3:
            a.load_remap = pass == 1;
            a.store_remap = pass == 3;
            a.line_centered = 0;
            a.sign1 = -1;
            a.mid_on = 1;
            a.mid = turns[pass];
            a.scale = (T)(1.0 / Nx);
            a.has_t2 = 1;
            a.sign2 = +1;
            break;
        case 2:
            a.sign1 = +1;
            a.mid_on = 1;
            a.mid = turns[2];
            a.scale = (T)(1.0 / Ny);
            a.has_t2 = 1;
            a.sign2 = -1;
            break;
        default:
            a.store_remap = 1;
            a.line_centered = 1;
            a.sign1 = +1;
            a.mid_on = 1;
            a.mid = turns[4];
            a.scale = (T)(1.0 / Ny);
            break;
    }
    return a;
}

void chain_args(const PlanData& d, int dir, ChirpArg out[5]) {
    for (int k = 0; k < 5; ++k) out[k] = to_arg(d.dir[dir].turns[k]);
}

template <typename T>
PassArgs<T> pass_args(const PlanData& d, int dir, int pass, const void* in, void* out) {
    ChirpArg c[5];
    chain_args(d, dir, c);
    return make_pass_args<T>(d.Nx, d.Ny, c, pass, in, out);
}

// ------------------------------------------------------ split precision
// Passes whose line DFTs run on the matrix cores with split half-precision
// operands (FP32 accumulation); storage complex64, chirps as in the FP32
// path.  Lines (16^2 or 16^3 long) live in LDS for the whole pass; every
// element-wise step (chirp, scale) is one sweep over LDS.
template <int N, bool COL>
constexpr int split_lines() {
    return N == 4096 ? (COL ? 2 : 1) : 16;
}

template <int KIND, int N, bool COL>
__global__ void __launch_bounds__((split_lines<N, COL>() * N / 16)) nslct_split_pass(PassArgs<float> a) {
    constexpr int LINES = split_lines<N, COL>();
    constexpr int THREADS = LINES * N / 16;
    constexpr int PER = LINES * N / THREADS;  // = 16 elements per thread per sweep
    constexpr int LL = lds_line_elems<N>();
    __shared__ cplx<float> lds[LINES * LL];
    SplitW<KIND> W;  // this lane's A operands (per-lane values, in registers)
    const int tid = threadIdx.x;
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int line0 = tile * LINES;
    const int nl = a.nlines;
    const cplx<float>* __restrict__ in = a.in + (size_t)blockIdx.y * a.img_stride;
    cplx<float>* __restrict__ out = a.out + (size_t)blockIdx.y * a.img_stride;
    const cplx<float>* __restrict__ tab = twiddles<float>();
    W.init(tid % 64);

    // Load into LDS in FFT order.
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = tid + THREADS * k;
        if constexpr (COL) {
            const int c = idx % LINES, p = idx / LINES;
            const int i = a.load_remap ? store_to_fft<N>(p) : p;
            lds[c * LL + lds_pad(i)] = line0 + c < nl ? in[(size_t)p * nl + line0 + c] : cplx<float>{0, 0};
        } else {
            const int ln = idx / N, p = idx % N;
            const int src = a.load_remap ? fft_to_store<N>(p) : p;
            lds[ln * LL + lds_pad(p)] = line0 + ln < nl ? in[(size_t)(line0 + ln) * N + src] : cplx<float>{0, 0};
        }
    }
    __syncthreads();

    auto chirp = [&](const ChirpArg& c, float scale) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int idx = tid + THREADS * k;
            const int ln = idx / N, p = idx % N;
            const int line = line0 + ln;
            const int lc = a.line_centered ? line - nl / 2 : (line >= (nl + 1) / 2 ? line - nl : line);
            const int e = p >= (N + 1) / 2 ? p - N : p;
            const uint64_t l64 = (uint64_t)(int64_t)lc, e64 = (uint64_t)(int64_t)e;
            const uint64_t ph = (COL ? c.c22 : c.c11) * (l64 * l64) + c.c12 * (l64 * e64) +
                                (COL ? c.c11 : c.c22) * (e64 * e64);
            cplx<float>& v = lds[ln * LL + lds_pad(p)];
            v = cmul(v, turns_cs(ph, scale));
        }
        __syncthreads();
    };

    if (a.pre.on) chirp(a.pre, 1.f);
    if (a.sign1 < 0)
        split_dft<KIND, -1, N, LINES>(lds, W, tab);
    else
        split_dft<KIND, +1, N, LINES>(lds, W, tab);
    if (a.mid_on) chirp(a.mid, a.scale);
    if (a.has_t2) {
        if (a.sign2 < 0)
            split_dft<KIND, -1, N, LINES>(lds, W, tab);
        else
            split_dft<KIND, +1, N, LINES>(lds, W, tab);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = tid + THREADS * k;
        if constexpr (COL) {
            const int c = idx % LINES, p = idx / LINES;
            if (line0 + c < nl)
                out[(size_t)p * nl + line0 + c] = lds[c * LL + lds_pad(a.store_remap ? store_to_fft<N>(p) : p)];
        } else {
            const int ln = idx / N, p = idx % N;
            if (line0 + ln < nl)
                out[(size_t)(line0 + ln) * N + (a.store_remap ? fft_to_store<N>(p) : p)] = lds[ln * LL + lds_pad(p)];
        }
    }
}

bool split_size_ok(int n) { return n == 256 || n == 4096; }

template <int KIND, bool COL>
hipError_t launch_split_n(int N, const PassArgs<float>& a, int count, hipStream_t s) {
    switch (N) {
        case 256: {
            constexpr int L = split_lines<256, COL>();
            hipLaunchKernelGGL((nslct_split_pass<KIND, 256, COL>), dim3((a.nlines + L - 1) / L, count),
                               dim3(L * 256 / 16), 0, s, a);
            return hipGetLastError();
        }
        case 4096: {
            constexpr int L = split_lines<4096, COL>();
            hipLaunchKernelGGL((nslct_split_pass<KIND, 4096, COL>), dim3((a.nlines + L - 1) / L, count),
                               dim3(L * 4096 / 16), 0, s, a);
            return hipGetLastError();
        }
        default:
            return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------- backward
// Backward sweep: the inverse chain applied to the forward output G and to
// the incoming gradient at once, with the gradient sums at every chirp point.
template <typename T, int N, bool COL, int LINES>
__global__ void __launch_bounds__(LinePlan<N>::TPL* LINES) nslct_pair_pass(PassArgs<T> a) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<N>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    pass_body<T, N, COL, LINES, 2>(a, tile, (size_t)blockIdx.y * a.img_stride, lds_all);
}

#define NSLCT_PAIR_SIZES(X) X(8) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool pair_size_ok(int n) {
    switch (n) {
#define NSLCT_PAIR_OK(v) case v:
        NSLCT_PAIR_SIZES(NSLCT_PAIR_OK)
#undef NSLCT_PAIR_OK
        return true;
        default:
            return false;
    }
}

template <typename T, bool COL>
hipError_t launch_pair_n(int N, const PassArgs<T>& a, int count, hipStream_t s) {
    switch (N) {
#define NSLCT_PAIR_LAUNCH(v)                                                                     \
    case v: {                                                                                    \
        constexpr int L = COL ? col_lines<T, v>() : row_lines<T, v>();                           \
        hipLaunchKernelGGL((nslct_pair_pass<T, v, COL, L>), dim3((a.nlines + L - 1) / L, count), \
                           dim3(LinePlan<v>::TPL * L), 0, s, a);                                 \
        return hipGetLastError();                                                                \
    }
        NSLCT_PAIR_SIZES(NSLCT_PAIR_LAUNCH)
#undef NSLCT_PAIR_LAUNCH
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t run_backward_t(const PlanData& d, int count, const void* G, const void* gout, void* work, void* gx,
                          double* sums, hipStream_t s) {
    for (int pass = 0; pass < 5; ++pass) {
        PassArgs<T> a = pass_args<T>(d, 1, pass, pass == 0 ? G : work, work);
        a.in2 = (const cplx<T>*)(pass == 0 ? gout : gx);
        a.out2 = (cplx<T>*)gx;
        a.acc = sums + 3 * pass;
        const bool col = (pass == 1 || pass == 3);
        const hipError_t e = col ? launch_pair_n<T, true>(d.Nx, a, count, s) : launch_pair_n<T, false>(d.Ny, a, count, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ----------------------------------------------------------------- batched
// One pass of one image of a ragged batch, built on the host: the pass
// arguments (input and output pointers are taken from BatchArgs) and the
// image's sample offset in the packed buffer.  Entry (img * 2 + dir) * 5 +
// pass.
template <typename T>
struct BatchPass {
    PassArgs<T> a;
    long long off;
};
struct BatchItem {
    int img;   // -1: padding item
    int tile;  // line tile of that image
};
template <typename T>
struct BatchArgs {
    const cplx<T>* in;
    cplx<T>* out;
    const BatchPass<T>* passes;
    const BatchItem* items;
    int nitems;
    int dir;
    int pass;
};

constexpr int kBatchThreads = 256;
// Line lengths the batched kernel handles (all with TPL <= 64).
#define NSLCT_BATCH_SIZES(X) X(64) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Lines per work item: kBatchThreads threads' worth, doubled for complex64
// column tiles (1024-long columns: 8 columns, 64-byte row segments; measured
// 2.75 -> 2.68 ms on the 256-image ragged batch).
template <int N, bool COL = false, typename T = float>
constexpr int batch_lines() {
    return ((COL && sizeof(T) == 4) ? 2 : 1) * kBatchThreads / LinePlan<N>::TPL;
}
bool batch_size_ok(int n) {
    switch (n) {
#define NSLCT_CASE_OK(v) case v:
        NSLCT_BATCH_SIZES(NSLCT_CASE_OK)
#undef NSLCT_CASE_OK
        return true;
        default:
            return false;
    }
}

int host_batch_lines(int n, bool col, bool dbl) {
    switch (n) {
#define NSLCT_CASE_L(v) \
    case v:           \
        return (col && !dbl) ? batch_lines<v, true, float>() : batch_lines<v>();
        NSLCT_BATCH_SIZES(NSLCT_CASE_L)
#undef NSLCT_CASE_L
        default:
            return 1;
    }
}

// Batched pass over the images of one line length N.  LOOP: a persistent
// grid whose workgroups walk the group's item list with a grid stride (item
// i belongs to XCD i mod 8, which is also the XCD of every workgroup that
// visits it: the grid size is a multiple of 8); otherwise one workgroup per
// item, without the loop, whose loop-invariant values would otherwise stay
// in registers across iterations.
template <typename T, int N, bool COL, bool LOOP>
__global__ void __launch_bounds__((batch_lines<N, COL, T>() * LinePlan<N>::TPL))
    nslct_batched_pass(BatchArgs<T> b, const BatchItem* __restrict__ items, const BatchPass<T>* __restrict__ passes) {
    constexpr int L = batch_lines<N, COL, T>();
    __shared__ cplx<T> lds[L * lds_line_elems<N>()];
    // The work list and the pass table come in as restrict parameters (no
    // store of the kernel can alias them), so their uniform-index loads are
    // scalar and the pass arguments stay in scalar registers.
    auto item = [&](int it) {
        const BatchItem w = items[it];
        if (w.img >= 0) {
            const int k = (w.img * 2 + b.dir) * 5 + b.pass;
            PassArgs<T> a = passes[k].a;
            a.in = b.in;
            a.out = b.out;
            pass_body<T, N, COL, L>(a, w.tile, (size_t)passes[k].off, lds);
        }
    };
    if constexpr (LOOP) {
        for (int it = blockIdx.x; it < b.nitems; it += gridDim.x) {
            item(it);
            __syncthreads();
        }
    } else {
        if ((int)blockIdx.x < b.nitems) item(blockIdx.x);
    }
}

template <typename T, bool COL>
hipError_t launch_batched_group(int N, const BatchArgs<T>& a, int grid, hipStream_t s) {
    switch (N) {
#define NSLCT_CASE_LAUNCH(v)                                                                        \
    case v:                                                                                         \
        if (grid >= a.nitems)                                                                       \
            hipLaunchKernelGGL((nslct_batched_pass<T, v, COL, false>), dim3(a.nitems),               \
                               dim3(batch_lines<v, COL, T>() * LinePlan<v>::TPL), 0, s, a,          \
                               a.items, a.passes);                                                  \
        else                                                                                        \
            hipLaunchKernelGGL((nslct_batched_pass<T, v, COL, true>), dim3(grid),                    \
                               dim3(batch_lines<v, COL, T>() * LinePlan<v>::TPL), 0, s, a,          \
                               a.items, a.passes);                                                  \
        return hipGetLastError();
        NSLCT_BATCH_SIZES(NSLCT_CASE_LAUNCH)
#undef NSLCT_CASE_LAUNCH
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pass_typed(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s);

template <int KIND, bool COL>
hipError_t launch_split_n(int N, const PassArgs<float>& a, int count, hipStream_t s);

// ---------------------------------------------------------------- Bluestein
// Line lengths N without a native plan (any N <= 2048 that is not 2^k or
// 3 * 2^k): each N-point line DFT is Bluestein's chirp-z form on an M-point
// line, M the smallest power of two >= 2N - 1.  With kn = (k^2 + n^2 -
// (k - n)^2) / 2, a DFT of exponent sign S is
//   X_k = c_k sum_n (x_n c_n) b_(k-n),  c_n = exp(S j pi n^2 / N),
//   b_m = exp(-S j pi m^2 / N),
// a linear convolution evaluated as FFT_M -> multiply by FFT_M(b) / M ->
// inverse FFT_M.  The chirp phases come from the exact integer n^2 mod 2N.
// FFT_M(b) / M for S = -1 and S = +1 is tabulated once per (device, N,
// precision) in FP64 on the host.
template <typename T>
struct BsArgs {
    int N;               // line length
    const cplx<T>* tab;  // [0, M): S = -1, [M, 2M): S = +1
};

bool native_line(int n) {
    if (n >= 2 && n <= 4096 && (n & (n - 1)) == 0) return true;
    if (n % 3 == 0 && n >= 6 && n <= 768) {
        const int m = n / 3;
        return (m & (m - 1)) == 0;
    }
    return false;
}

int bluestein_length(int n) {
    int m = 1;
    while (m < 2 * n - 1) m <<= 1;
    return m;
}

std::mutex g_bs_mu;
std::vector<std::pair<std::array<int, 4>, void*>> g_bs;  // (device, N, M, fp64) -> table

int bs_tables(int N, int M, bool dbl, const void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    const std::array<int, 4> key{dev, N, M, dbl ? 1 : 0};
    std::lock_guard<std::mutex> lk(g_bs_mu);
    for (const auto& kv : g_bs)
        if (kv.first == key) {
            *out = kv.second;
            return NSLCT_OK;
        }
    // b_m for S = -1 (exp(+j pi m^2 / N)) at m and M - m; B = FFT_M(b).
    const double pi = 3.14159265358979323846;
    std::vector<double> br(M, 0.0), bi(M, 0.0), cr(M), ci(M);
    for (int m = 0; m < N; ++m) {
        const long long r = ((long long)m * m) % (2LL * N);
        br[m] = std::cos(pi * (double)r / N);
        bi[m] = std::sin(pi * (double)r / N);
        if (m > 0) {
            br[M - m] = br[m];
            bi[M - m] = bi[m];
        }
    }
    for (int k = 0; k < M; ++k) {
        cr[k] = std::cos(2 * pi * k / M);
        ci[k] = -std::sin(2 * pi * k / M);
    }
    std::vector<double> Br(M), Bi(M);
    for (int p = 0; p < M; ++p) {
        double sr = 0, si = 0;
        for (int m = 0; m < M; ++m) {
            if (m >= N && m <= M - N) continue;  // b is zero there
            const int k = (int)(((long long)p * m) % M);
            sr += br[m] * cr[k] - bi[m] * ci[k];
            si += br[m] * ci[k] + bi[m] * cr[k];
        }
        Br[p] = sr / M;
        Bi[p] = si / M;
    }
    const size_t elem = dbl ? sizeof(cplx<double>) : sizeof(cplx<float>);
    std::vector<unsigned char> host(2 * (size_t)M * elem);
    for (int p = 0; p < M; ++p)
        for (int sidx = 0; sidx < 2; ++sidx) {
            const double re = Br[p], im = sidx == 0 ? Bi[p] : -Bi[p];  // S = +1: conjugate (b is even)
            const size_t at = ((size_t)sidx * M + p);
            if (dbl)
                reinterpret_cast<cplx<double>*>(host.data())[at] = {re, im};
            else
                reinterpret_cast<cplx<float>*>(host.data())[at] = {(float)re, (float)im};
        }
    void* dptr = nullptr;
    e = hipMalloc(&dptr, host.size());
    if (e == hipSuccess) e = hipMemcpy(dptr, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (dptr) (void)hipFree(dptr);
        return fail(NSLCT_E_HIP, std::string("Bluestein table: ") + hipGetErrorString(e));
    }
    g_bs.push_back({key, dptr});
    *out = dptr;
    return NSLCT_OK;
}

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

// One pass on lines of length N through M-point Bluestein line DFTs; the
// pass structure ([pre] DFT [mid] [DFT], remaps, centring) is that of
// pass_body, with every sample access restricted to positions < N.
template <typename T, int M, bool COL, int LINES>
__global__ void __launch_bounds__(LinePlan<M>::TPL* LINES) nslct_bs_pass(PassArgs<T> a, BsArgs<T> bs) {
    constexpr int TPL = LinePlan<M>::TPL;
    using F = LineFFT<T, M, TPL>;
    constexpr int E = F::E;
    constexpr int R0 = F::R0;
    constexpr int LL = lds_line_elems<M>();
    __shared__ cplx<T> lds_all[LINES * LL];

    const int N = bs.N, twoN = 2 * N;
    const int tid = threadIdx.x;
    const int slot = tid / TPL;
    const int t = tid % TPL;
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int line = tile * LINES + slot;
    const int nl = a.nlines;
    const bool active = line < nl;
    cplx<T>* lds = lds_all + slot * LL;
    const cplx<T>* __restrict__ tab = twiddles<T>();
    const size_t img_off = (size_t)blockIdx.y * a.img_stride;
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
        const uint64_t A = (COL ? c.c22 : c.c11) * (l64 * l64);
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

template <typename T, int M, bool COL>
hipError_t launch_bs_t(const PassArgs<T>& a, const BsArgs<T>& b, int count, hipStream_t s) {
    constexpr int L = COL ? col_lines<T, M>() : row_lines<T, M>();
    static_assert(L * lds_line_elems<M>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    hipLaunchKernelGGL((nslct_bs_pass<T, M, COL, L>), dim3((a.nlines + L - 1) / L, count),
                       dim3(LinePlan<M>::TPL * L), 0, s, a, b);
    return hipGetLastError();
}

template <typename T, bool COL>
hipError_t launch_bs_n(int M, const PassArgs<T>& a, const BsArgs<T>& b, int count, hipStream_t s) {
    switch (M) {
        case 8: return launch_bs_t<T, 8, COL>(a, b, count, s);
        case 16: return launch_bs_t<T, 16, COL>(a, b, count, s);
        case 32: return launch_bs_t<T, 32, COL>(a, b, count, s);
        case 64: return launch_bs_t<T, 64, COL>(a, b, count, s);
        case 128: return launch_bs_t<T, 128, COL>(a, b, count, s);
        case 256: return launch_bs_t<T, 256, COL>(a, b, count, s);
        case 512: return launch_bs_t<T, 512, COL>(a, b, count, s);
        case 1024: return launch_bs_t<T, 1024, COL>(a, b, count, s);
        case 2048: return launch_bs_t<T, 2048, COL>(a, b, count, s);
        case 4096: return launch_bs_t<T, 4096, COL>(a, b, count, s);
        default: return hipErrorInvalidValue;
    }
}

// Bluestein tables of every non-native axis of a plan on the current device
// (computed and uploaded on first use).
int prepare_plan_tables(const PlanData& d) {
    const bool split = d.precision == NSLCT_C64_SPLIT_F16 || d.precision == NSLCT_C64_SPLIT_BF16;
    if (split) return NSLCT_OK;
    for (int n : {d.Nx, d.Ny}) {
        if (native_line(n)) continue;
        const void* tabp = nullptr;
        const int rc = bs_tables(n, bluestein_length(n), d.precision == NSLCT_C128, &tabp);
        if (rc) return rc;
    }
    return NSLCT_OK;
}

template <typename T>
hipError_t launch_pass_typed(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s) {
    const PassArgs<T> a = pass_args<T>(d, dir, pass, in, out);
    const bool col = (pass == 1 || pass == 3);
    const int N = col ? d.Nx : d.Ny;
    if (!native_line(N)) {
        const void* tabp = nullptr;
        if (bs_tables(N, bluestein_length(N), sizeof(T) == 8, &tabp) != NSLCT_OK) return hipErrorInvalidValue;
        const BsArgs<T> b{N, (const cplx<T>*)tabp};
        const int M = bluestein_length(N);
        return col ? launch_bs_n<T, true>(M, a, b, count, s) : launch_bs_n<T, false>(M, a, b, count, s);
    }
    if (col && col4096_applies(a, N)) return launch_col4096(a, count, s);
    return col ? launch_n<T, true>(d.Nx, a, count, s) : launch_n<T, false>(d.Ny, a, count, s);
}

// Passes of the single-image path: the three-pass schedule of a reduced
// chain (CM-CC-CM, LC) in c64 / c128, else the five-pass chain.
int plan_passes(const PlanData& d) {
    const bool split = d.precision == NSLCT_C64_SPLIT_F16 || d.precision == NSLCT_C64_SPLIT_BF16;
    return (!split && d.prog[0].npass > 0) ? d.prog[0].npass : 5;
}

template <typename T>
PassArgs<T> program_args(const PlanData& d, int dir, int k, const void* in, void* out) {
    const ProgPass& q = d.prog[dir].p[k];
    PassArgs<T> a{};
    a.in = (const cplx<T>*)in;
    a.out = (cplx<T>*)out;
    a.img_stride = (long long)d.Nx * d.Ny;
    a.nlines = q.col ? d.Ny : d.Nx;
    a.load_remap = q.load_remap;
    a.store_remap = q.store_remap;
    a.line_centered = q.line_centered;
    a.sign1 = q.sign[0];
    a.pre = to_arg(q.pre);
    a.pre.on = q.pre_on && q.pre.nonzero;
    a.mid_on = q.mid_on;
    a.mid = to_arg(q.mid);
    a.scale = (T)q.scale_mid;
    a.has_t2 = q.ndft >= 2;
    a.sign2 = q.sign[1];
    a.post_on = q.post_on;
    a.post = to_arg(q.post);
    a.scale2 = (T)q.scale_post;
    a.sign3 = q.sign[2];
    return a;
}

template <typename T>
hipError_t launch_program_pass(const PlanData& d, int dir, int k, int count, const void* in, void* out,
                               hipStream_t s) {
    const ProgPass& q = d.prog[dir].p[k];
    const PassArgs<T> a = program_args<T>(d, dir, k, in, out);
    if (q.ndft == 3)
        return q.col ? launch_n<T, true, true>(d.Nx, a, count, s) : launch_n<T, false, true>(d.Ny, a, count, s);
    return q.col ? launch_n<T, true>(d.Nx, a, count, s) : launch_n<T, false>(d.Ny, a, count, s);
}

hipError_t launch_pass(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                       hipStream_t s) {
    if (plan_passes(d) != 5)
        return d.precision == NSLCT_C128 ? launch_program_pass<double>(d, dir, pass, count, in, out, s)
                                         : launch_program_pass<float>(d, dir, pass, count, in, out, s);
    if (d.precision == NSLCT_C64_SPLIT_F16 || d.precision == NSLCT_C64_SPLIT_BF16) {
        const PassArgs<float> a = pass_args<float>(d, dir, pass, in, out);
        const bool col = (pass == 1 || pass == 3);
        const int N = col ? d.Nx : d.Ny;
        if (d.precision == NSLCT_C64_SPLIT_F16)
            return col ? launch_split_n<0, true>(N, a, count, s) : launch_split_n<0, false>(N, a, count, s);
        return col ? launch_split_n<1, true>(N, a, count, s) : launch_split_n<1, false>(N, a, count, s);
    }
    return d.precision == NSLCT_C128 ? launch_pass_typed<double>(d, dir, pass, count, in, out, s)
                                     : launch_pass_typed<float>(d, dir, pass, count, in, out, s);
}

int check_ptrs(const void* in, const void* out) {
    if (!in || !out) return fail(NSLCT_E_ARG, "null image pointer");
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15))
        return fail(NSLCT_E_ARG, "image pointers must be 16-byte aligned");
    return NSLCT_OK;
}

int run_chain(nslct_plan_t plan, int dir, int count, const void* in, void* out, void* stream) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    if (count < 0 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [0, 65535]");
    int rc = check_ptrs(in, out);
    if (rc) return rc;
    if (count == 0) return NSLCT_OK;
    rc = ensure_device_ready();
    if (!rc) rc = prepare_plan_tables(plan->d);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int np = plan_passes(plan->d);
    for (int pass = 0; pass < np; ++pass) {
        hipError_t e = launch_pass(plan->d, dir, pass, count, pass == 0 ? in : out, out, s);
        if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("pass launch: ") + hipGetErrorString(e));
    }
    return NSLCT_OK;
}

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}


// Launches the five batched passes of direction `dir` on `s`.
template <typename T>
hipError_t run_batched_t(const nslct_batch_s& b, int dir, const void* in, void* out, hipStream_t s);

}  // namespace

struct nslct_batch_s {
    int count = 0;
    int precision = NSLCT_C64;
    int device = 0;
    size_t total = 0;                 // samples in the packed buffer
    std::vector<long long> offsets;
    std::vector<nslct_plan_s> plans;  // copies of the input plans
    void* d_passes = nullptr;  // BatchPass<T>[count * 10], T by precision
    // Work groups: one per (pass kind, line length).  Row passes ([0]) take
    // lines of length Ny, column passes ([1]) lines of length Nx.
    struct Group {
        int N;
        int nitems;
        int grid;
        BatchItem* items;
    };
    std::vector<Group> groups[2];
    int mult = 0;  // autotuned persistent workgroups per CU (0: one per item)
    int cus = 256;  // compute units of the device
    double tuned_us = 0.0;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side;  // fork streams for concurrent groups
    std::vector<hipEvent_t> ev;     // fork / join events
    struct Graph {
        const void* in;
        void* out;
        int dir;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    std::mutex mu;

    ~nslct_batch_s() {
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
        for (auto e : ev) (void)hipEventDestroy(e);
        for (auto st : side) (void)hipStreamDestroy(st);
        if (cap) (void)hipStreamDestroy(cap);
        if (d_passes) (void)hipFree(d_passes);
        for (auto& gs : groups)
            for (auto& g : gs)
                if (g.items) (void)hipFree(g.items);
    }
};

namespace {

template <typename T>
hipError_t run_batched_t(const nslct_batch_s& b, int dir, const void* in, void* out, hipStream_t s) {
    for (int pass = 0; pass < 5; ++pass) {
        const int col = (pass == 1 || pass == 3) ? 1 : 0;
        const auto& gs = b.groups[col];
        // Groups of one pass are independent: with fork streams they run
        // concurrently (joined before the next pass).
        const bool fork = gs.size() > 1 && b.side.size() >= gs.size();
        hipError_t e = hipSuccess;
        if (fork) {
            e = hipEventRecord(b.ev[0], s);
            for (size_t k = 0; k < gs.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(b.side[k], b.ev[0], 0);
        }
        for (size_t k = 0; k < gs.size() && e == hipSuccess; ++k) {
            BatchArgs<T> a;
            a.in = (const cplx<T>*)(pass == 0 ? in : out);
            a.out = (cplx<T>*)out;
            a.passes = (const BatchPass<T>*)b.d_passes;
            a.items = gs[k].items;
            a.nitems = gs[k].nitems;
            a.dir = dir;
            a.pass = pass;
            hipStream_t st = fork ? b.side[k] : s;
            e = col ? launch_batched_group<T, true>(gs[k].N, a, gs[k].grid, st)
                    : launch_batched_group<T, false>(gs[k].N, a, gs[k].grid, st);
            if (e == hipSuccess && fork) e = hipEventRecord(b.ev[1 + k], st);
        }
        if (fork)
            for (size_t k = 0; k < gs.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, b.ev[1 + k], 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_batched(const nslct_batch_s& b, int dir, const void* in, void* out, hipStream_t s) {
    return b.precision == NSLCT_C128 ? run_batched_t<double>(b, dir, in, out, s)
                                     : run_batched_t<float>(b, dir, in, out, s);
}

// Work items of the images whose pass lines have length N, dealt to the 8
// XCDs: whole images go to the least-loaded XCD (largest first), and item i
// of the list belongs to XCD i mod 8, so adjacent line tiles of one image
// share an XCD and its L2.
std::vector<BatchItem> build_items(const nslct_batch_s& b, bool col, int N) {
    std::vector<int> order;
    for (int i = 0; i < b.count; ++i) {
        const PlanData& d = b.plans[i].d;
        if ((col ? d.Nx : d.Ny) == N) order.push_back(i);
    }
    auto cost = [&](int i) {
        const PlanData& d = b.plans[i].d;
        return (double)d.Nx * d.Ny;
    };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<std::vector<BatchItem>> per(8);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int L = host_batch_lines(N, col, b.precision == NSLCT_C128);
    for (int i : order) {
        const PlanData& d = b.plans[i].d;
        const int nl = col ? d.Ny : d.Nx;
        const int tiles = (nl + L - 1) / L;
        int x = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[x]) x = k;
        load[x] += cost(i);
        for (int t = 0; t < tiles; ++t) per[x].push_back({i, t});
    }
    size_t len = 0;
    for (auto& v : per) len = std::max(len, v.size());
    std::vector<BatchItem> items(8 * len, BatchItem{-1, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t k = 0; k < per[x].size(); ++k) items[8 * k + x] = per[x][k];
    return items;
}

void set_grids(nslct_batch_s* b, int mult, int cus) {
    b->mult = mult;
    for (auto& gs : b->groups)
        for (auto& g : gs) {
            const int want = mult == 0 ? g.nitems : ((mult * cus + 7) / 8) * 8;
            g.grid = std::max(8, std::min(want, g.nitems));
        }
}

int batch_fail(nslct_batch_s* b, hipError_t e, const char* what) {
    delete b;
    return fail(NSLCT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Builds and uploads the per-(image, direction, pass) argument table.
template <typename T>
hipError_t upload_batch_passes(nslct_batch_s& b) {
    std::vector<BatchPass<T>> tab((size_t)b.count * 10);
    for (int i = 0; i < b.count; ++i) {
        const PlanData& d = b.plans[i].d;
        for (int dir = 0; dir < 2; ++dir) {
            ChirpArg c[5];
            chain_args(d, dir, c);
            for (int pass = 0; pass < 5; ++pass) {
                BatchPass<T>& e = tab[((size_t)i * 2 + dir) * 5 + pass];
                e.a = make_pass_args<T>(d.Nx, d.Ny, c, pass, nullptr, nullptr);
                e.off = b.offsets[i];
            }
        }
    }
    hipError_t e = hipMalloc(&b.d_passes, sizeof(BatchPass<T>) * tab.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(b.d_passes, tab.data(), sizeof(BatchPass<T>) * tab.size(), hipMemcpyHostToDevice);
}

}  // namespace

extern "C" {

void nslct_opts_default(nslct_opts* o) {
    if (!o) return;
    o->precision = NSLCT_C64;
    o->type_override = 0;
    o->symplectic_tol = 1e-9;
}

int nslct_plan_ex(const double abcd[16], int Nx, int Ny, double dx, double dy, const nslct_opts* opts,
                  nslct_plan_t* out) {
    if (!abcd || !out) return fail(NSLCT_E_ARG, "null argument");
    *out = nullptr;
    nslct_opts o;
    nslct_opts_default(&o);
    if (opts) o = *opts;
    auto* p = new (std::nothrow) nslct_plan_s;
    if (!p) return fail(NSLCT_E_ARG, "out of host memory");
    std::string err;
    const int rc = build_plan(abcd, Nx, Ny, dx, dy, o, &p->d, &err);
    if (rc) {
        delete p;
        return fail(rc, err);
    }
    *out = p;
    return NSLCT_OK;
}

int nslct_plan(const double abcd[16], int Nx, int Ny, double dx, double dy, nslct_plan_t* out) {
    return nslct_plan_ex(abcd, Nx, Ny, dx, dy, nullptr, out);
}

int nslct_plan_from_stages(const nslct_stages* st, int Nx, int Ny, const nslct_opts* opts, nslct_plan_t* out) {
    if (!st || !out) return fail(NSLCT_E_ARG, "null argument");
    *out = nullptr;
    nslct_opts o;
    nslct_opts_default(&o);
    if (opts) o = *opts;
    auto* p = new (std::nothrow) nslct_plan_s;
    if (!p) return fail(NSLCT_E_ARG, "out of host memory");
    std::string err;
    const int rc = build_plan_from_stages(*st, Nx, Ny, o, &p->d, &err);
    if (rc) {
        delete p;
        return fail(rc, err);
    }
    *out = p;
    return NSLCT_OK;
}

int nslct_plan_get_stages(nslct_plan_t plan, nslct_stages* out) {
    if (!plan || !out) return fail(NSLCT_E_ARG, "null argument");
    *out = plan->d.st;
    return NSLCT_OK;
}

int nslct_plan_box_check(nslct_plan_t plan, double frac, int* ok) {
    if (!plan || !ok || !(frac > 0)) return fail(NSLCT_E_ARG, "bad argument");
    *ok = box_check(plan->d, frac) ? 1 : 0;
    return NSLCT_OK;
}

void nslct_plan_destroy(nslct_plan_t plan) { delete plan; }

int nslct_forward(nslct_plan_t plan, const void* in, void* out, void* stream) {
    return run_chain(plan, 0, 1, in, out, stream);
}

int nslct_inverse(nslct_plan_t plan, const void* in, void* out, void* stream) {
    return run_chain(plan, 1, 1, in, out, stream);
}

int nslct_forward_many(nslct_plan_t plan, int count, const void* in, void* out, void* stream) {
    return run_chain(plan, 0, count, in, out, stream);
}

int nslct_inverse_many(nslct_plan_t plan, int count, const void* in, void* out, void* stream) {
    return run_chain(plan, 1, count, in, out, stream);
}

int nslct_launch_pass(nslct_plan_t plan, int direction, int pass, int count, const void* in, void* out,
                      void* stream) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    if (direction != 0 && direction != 1) return fail(NSLCT_E_ARG, "direction must be 0 or 1");
    if (pass < 0 || pass >= plan_passes(plan->d))
        return fail(NSLCT_E_ARG, "pass must be in [0, nslct_plan_passes)");
    if (count < 1 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [1, 65535]");
    int rc = check_ptrs(in, out);
    if (rc) return rc;
    rc = ensure_device_ready();
    if (!rc) rc = prepare_plan_tables(plan->d);
    if (rc) return rc;
    hipError_t e = launch_pass(plan->d, direction, pass, count, in, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("pass launch: ") + hipGetErrorString(e));
    return NSLCT_OK;
}

int nslct_plan_passes(nslct_plan_t plan, int* npasses) {
    if (!plan || !npasses) return fail(NSLCT_E_ARG, "null argument");
    *npasses = plan_passes(plan->d);
    return NSLCT_OK;
}

int nslct_device_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(NSLCT_E_ARG, "copy needs 16-byte aligned pointers and size");
    if (bytes == 0) return NSLCT_OK;
    const size_t n = bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint4*)src, (uint4*)dst, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("copy launch: ") + hipGetErrorString(e));
    return NSLCT_OK;
}

int nslct_batch_create(const nslct_plan_t* plans, int count, nslct_batch_t* out) {
    if (!plans || !out || count < 1) return fail(NSLCT_E_ARG, "need plans, count >= 1 and out");
    *out = nullptr;
    auto* b = new (std::nothrow) nslct_batch_s;
    if (!b) return fail(NSLCT_E_ARG, "out of host memory");
    b->count = count;
    b->precision = plans[0] ? plans[0]->d.precision : NSLCT_C64;
    b->plans.resize(count);
    b->offsets.resize(count);
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) {
            delete b;
            return fail(NSLCT_E_ARG, "null plan in batch");
        }
        const PlanData& d = plans[i]->d;
        if (d.precision != b->precision) {
            delete b;
            return fail(NSLCT_E_ARG, "all plans of a batch must share one precision");
        }
        if (d.precision != NSLCT_C64 && d.precision != NSLCT_C128) {
            delete b;
            return fail(NSLCT_E_UNSUPPORTED, "batches run complex64 or complex128 plans");
        }
        if (!batch_size_ok(d.Nx) || !batch_size_ok(d.Ny)) {
            delete b;
            return fail(NSLCT_E_SIZE, "batched sides must be one of 64, 128, 192, 256, 384, 512, 768, 1024");
        }
        b->plans[i].d = d;
        b->offsets[i] = (long long)b->total;
        b->total += (size_t)d.Nx * d.Ny;
    }
    int rc = ensure_device_ready();
    if (rc) {
        delete b;
        return rc;
    }
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) return batch_fail(b, e, "hipGetDevice");
    e = b->precision == NSLCT_C128 ? upload_batch_passes<double>(*b) : upload_batch_passes<float>(*b);
    if (e != hipSuccess) return batch_fail(b, e, "pass table upload");
    for (int col = 0; col < 2; ++col) {
        std::vector<int> sizes;
        for (int i = 0; i < count; ++i) {
            const int N = col ? b->plans[i].d.Nx : b->plans[i].d.Ny;
            if (std::find(sizes.begin(), sizes.end(), N) == sizes.end()) sizes.push_back(N);
        }
        std::sort(sizes.begin(), sizes.end(), std::greater<int>());
        for (int N : sizes) {
            const std::vector<BatchItem> items = build_items(*b, col == 1, N);
            nslct_batch_s::Group g{N, (int)items.size(), 8, nullptr};
            e = hipMalloc(&g.items, sizeof(BatchItem) * items.size());
            if (e != hipSuccess) return batch_fail(b, e, "hipMalloc");
            b->groups[col].push_back(g);
            e = hipMemcpy(g.items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) return batch_fail(b, e, "hipMemcpy");
        }
    }
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return batch_fail(b, e, "hipStreamCreate");
    const size_t nside = std::max(b->groups[0].size(), b->groups[1].size());
    for (size_t k = 0; k < nside && nside > 1; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return batch_fail(b, e, "hipStreamCreate");
        b->side.push_back(st);
    }
    for (size_t k = 0; k < nside + 1 && nside > 1; ++k) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return batch_fail(b, e, "hipEventCreate");
        b->ev.push_back(ev);
    }

    // Autotune the persistent grid (workgroups per CU) on scratch images.
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) cus = 256;
    b->cus = cus;
    const size_t bytes = b->total * (b->precision == NSLCT_C128 ? 16 : 8);
    void* scratch = nullptr;
    e = hipMalloc(&scratch, bytes);
    if (e != hipSuccess) return batch_fail(b, e, "hipMalloc (autotune scratch)");
    e = hipMemsetAsync(scratch, 0, bytes, b->cap);
    const int mults[] = {0, 1, 2, 4, 8};  // 0: one workgroup per item
    double best = 1e30;
    int best_mult = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int m : mults) {
        if (e != hipSuccess) break;
        set_grids(b, m, cus);
        e = run_batched(*b, 0, scratch, scratch, b->cap);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, b->cap);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run_batched(*b, 0, scratch, scratch, b->cap);
        if (e == hipSuccess) e = hipEventRecord(e1, b->cap);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms / 3 * 1e3 < best) {
            best = ms / 3 * 1e3;
            best_mult = m;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (e != hipSuccess) return batch_fail(b, e, "autotune");
    set_grids(b, best_mult, cus);
    b->tuned_us = best;
    *out = b;
    return NSLCT_OK;
}

int nslct_batch_info(nslct_batch_t batch, size_t* total_samples, int* mult, double* tuned_us) {
    if (!batch) return fail(NSLCT_E_ARG, "null batch");
    if (total_samples) *total_samples = batch->total;
    if (mult) *mult = batch->mult;
    if (tuned_us) *tuned_us = batch->tuned_us;
    return NSLCT_OK;
}

int nslct_batch_set_grid(nslct_batch_t batch, int mult) {
    if (!batch) return fail(NSLCT_E_ARG, "null batch");
    if (mult != 0 && mult != 1 && mult != 2 && mult != 4 && mult != 8)
        return fail(NSLCT_E_ARG, "mult must be 0, 1, 2, 4 or 8");
    std::lock_guard<std::mutex> lk(batch->mu);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && dev != batch->device) e = hipSetDevice(batch->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (dev >= 0 && dev != batch->device) (void)hipSetDevice(dev);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("set grid: ") + hipGetErrorString(e));
    for (auto& g : batch->graphs) (void)hipGraphExecDestroy(g.exec);
    batch->graphs.clear();
    set_grids(batch, mult, batch->cus);
    return NSLCT_OK;
}

int nslct_batch_run(nslct_batch_t batch, int direction, int mode, const void* in, void* out, void* stream) {
    if (!batch) return fail(NSLCT_E_ARG, "null batch");
    if (direction != 0 && direction != 1) return fail(NSLCT_E_ARG, "direction must be 0 or 1");
    if (mode < 0 || mode > 2) return fail(NSLCT_E_ARG, "mode must be 0, 1 or 2");
    int rc = check_ptrs(in, out);
    if (rc) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != batch->device) return fail(NSLCT_E_ARG, "batch used on another device than it was created on");
    hipStream_t s = (hipStream_t)stream;
    if (mode == 2) {  // per-image loop, one chain of launches per image
        const size_t es = batch->precision == NSLCT_C128 ? 16 : 8;
        for (int i = 0; i < batch->count; ++i) {
            const char* pi = (const char*)in + batch->offsets[i] * es;
            char* po = (char*)out + batch->offsets[i] * es;
            rc = run_chain(&batch->plans[i], direction, 1, pi, po, stream);
            if (rc) return rc;
        }
        return NSLCT_OK;
    }
    if (mode == 1) {
        const hipError_t e = run_batched(*batch, direction, in, out, s);
        return e == hipSuccess ? NSLCT_OK : fail(NSLCT_E_HIP, std::string("batched launch: ") + hipGetErrorString(e));
    }
    std::lock_guard<std::mutex> lk(batch->mu);
    hipGraphExec_t exec = nullptr;
    for (auto& g : batch->graphs)
        if (g.in == in && g.out == out && g.dir == direction) exec = g.exec;
    if (!exec) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(batch->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t le = run_batched(*batch, direction, in, out, batch->cap);
            e = hipStreamEndCapture(batch->cap, &graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        if (batch->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(batch->graphs.front().exec);
            batch->graphs.erase(batch->graphs.begin());
        }
        batch->graphs.push_back({in, out, direction, exec});
    }
    const hipError_t e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? NSLCT_OK : fail(NSLCT_E_HIP, std::string("graph launch: ") + hipGetErrorString(e));
}

int nslct_forward_batched(nslct_batch_t batch, const void* in, void* out, void* stream) {
    return nslct_batch_run(batch, 0, 0, in, out, stream);
}

int nslct_inverse_batched(nslct_batch_t batch, const void* in, void* out, void* stream) {
    return nslct_batch_run(batch, 1, 0, in, out, stream);
}

void nslct_batch_destroy(nslct_batch_t batch) { delete batch; }


int nslct_backward(nslct_plan_t plan, int count, const void* G, const void* grad_out, void* work, void* grad_x,
                   double* sums, void* stream) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    if (count < 1 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [1, 65535]");
    int rc = check_ptrs(G, grad_out);
    if (!rc) rc = check_ptrs(work, grad_x);
    if (rc) return rc;
    if (!sums || ((uintptr_t)sums & 7)) return fail(NSLCT_E_ARG, "sums must be an 8-byte aligned device pointer");
    const PlanData& d = plan->d;
    if (d.precision != NSLCT_C64 && d.precision != NSLCT_C128)
        return fail(NSLCT_E_UNSUPPORTED, "backward runs complex64 or complex128 plans");
    if (!pair_size_ok(d.Nx) || !pair_size_ok(d.Ny))
        return fail(NSLCT_E_SIZE, "backward sides must be 8..1024 (2^k) or 48, 96, 192, 384, 768");
    if (work == grad_x || work == G || work == grad_out || grad_x == G)
        return fail(NSLCT_E_ARG, "work and grad_x must be distinct from each other and from G");
    rc = ensure_device_ready();
    if (rc) return rc;
    const hipError_t e = d.precision == NSLCT_C128
                             ? run_backward_t<double>(d, count, G, grad_out, work, grad_x, sums, (hipStream_t)stream)
                             : run_backward_t<float>(d, count, G, grad_out, work, grad_x, sums, (hipStream_t)stream);
    return e == hipSuccess ? NSLCT_OK : fail(NSLCT_E_HIP, std::string("backward launch: ") + hipGetErrorString(e));
}

int nslct_plan_stage_gradient(nslct_plan_t plan, const double sums[15], double grad_stages[12]) {
    if (!plan || !sums || !grad_stages) return fail(NSLCT_E_ARG, "null argument");
    stage_gradient(plan->d, sums, grad_stages);
    return NSLCT_OK;
}

int nslct_lie_point(const double abcd[16], const double theta[10], double out[16]) {
    if (!abcd || !theta || !out) return fail(NSLCT_E_ARG, "null argument");
    lie_point(abcd, theta, out);
    return NSLCT_OK;
}

int nslct_plan_jacobian(const double abcd[16], const double theta0[10], int Nx, int Ny, double dx, double dy,
                        const nslct_opts* opts, double h, double jac[12 * 10]) {
    if (!abcd || !theta0 || !jac) return fail(NSLCT_E_ARG, "null argument");
    nslct_opts o;
    nslct_opts_default(&o);
    if (opts) o = *opts;
    std::string err;
    const int rc = plan_jacobian(abcd, theta0, Nx, Ny, dx, dy, o, h, jac, &err);
    return rc ? fail(rc, err) : NSLCT_OK;
}

const char* nslct_last_error(void) { return g_last_error.c_str(); }

const char* nslct_strerror(int code) {
    switch (code) {
        case NSLCT_OK: return "ok";
        case NSLCT_E_ARG: return "invalid argument";
        case NSLCT_E_NOT_SYMPLECTIC: return "ABCD matrix is not symplectic";
        case NSLCT_E_NO_DECOMPOSITION: return "no CM-CC-CM-CC decomposition";
        case NSLCT_E_SIZE: return "unsupported size";
        case NSLCT_E_HIP: return "HIP runtime error";
        case NSLCT_E_UNSUPPORTED: return "unsupported";
        default: return "unknown error";
    }
}

const char* nslct_version(void) { return "nslct 0.1 gfx950"; }

}  // extern "C"
