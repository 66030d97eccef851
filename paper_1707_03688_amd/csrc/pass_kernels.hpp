// Device building blocks shared by the translation units of the library:
// per-device twiddle tables, the pass argument block, exact chirps, the
// fused line pass (pointwise products and line DFTs in registers) and the
// five-slot pass arguments of a plan.  Everything here has internal linkage,
// so each translation unit holds its own copy of the device tables and
// initialises it through its own init_tables_* entry (internal.hpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft_engine.hpp"
#include "planner.hpp"

namespace nslct {
namespace {

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
    uint64_t c00;  // constant phase (turns)
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

// Sample loads and stores of the passes; NT: non-temporal (streaming)
// accesses of complex64 samples, which skip keeping the lines in the
// caches (used where one image's pass is latency-bound, see launch_t).
typedef float nslct_f2 __attribute__((ext_vector_type(2)));
template <bool NT, typename T>
__device__ __forceinline__ cplx<T> load_sample(const cplx<T>* p) {
    if constexpr (NT && sizeof(T) == 4) {
        const nslct_f2 u = __builtin_nontemporal_load(reinterpret_cast<const nslct_f2*>(p));
        return {u.x, u.y};
    } else {
        return *p;
    }
}
template <bool NT, typename T>
__device__ __forceinline__ void store_sample(cplx<T>* p, cplx<T> v) {
    if constexpr (NT && sizeof(T) == 4) {
        nslct_f2 u;
        u.x = v.re;
        u.y = v.im;
        __builtin_nontemporal_store(u, reinterpret_cast<nslct_f2*>(p));
    } else {
        *p = v;
    }
}

// One fused pass over LINES lines of length N per workgroup.  Row passes
// (COL = false) read and write contiguous lines directly.  Column passes
// cover a tile of LINES adjacent columns; their stores (and, for lines
// longer than a wavefront, their loads) are staged through LDS so that the
// global accesses cover LINES consecutive samples of each row (coalesced),
// while each line's FFT work stays with the TPL threads that own it.
// `img`, when given, replaces a.in and a.out (an image held in LDS).
template <typename T, int N, bool COL, int LINES, int NS = 1, bool X3 = false, typename PP = LinePlan<N>,
          bool NT = false>
__device__ __forceinline__ void pass_body(const PassArgs<T>& a, int tile, size_t img_off, cplx<T>* lds_all,
                                          cplx<T>* img = nullptr) {
    constexpr int TPL = PP::TPL;
    using F = LineFFT<T, N, TPL, typename PP::L>;
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
    const cplx<T>* ins[2] = {img ? img : a.in + img_off, NS > 1 ? a.in2 + img_off : nullptr};
    cplx<T>* outs[2] = {img ? img : a.out + img_off, NS > 1 ? a.out2 + img_off : nullptr};

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
                    v[sg][r] = load_sample<NT>(in + (size_t)src * nl + line);
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
                lds_all[c * LL + lds_pad(i)] = cok ? load_sample<NT>(in + (size_t)p * nl + line0 + c) : cplx<T>{0, 0};
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
                    v[sg][r] = load_sample<NT>(in + (size_t)line * N + src);
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
        const uint64_t A = (COL ? c.c22 : c.c11) * (l64 * l64) + c.c00;
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
                    store_sample<NT>(out + (size_t)p * nl + line0 + c, lds_all[c * LL + lds_pad(p)]);
                }
            }
        } else if (active) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const int p = pos(r);
                const int dst = a.store_remap ? fft_to_store<N>(p) : p;
                store_sample<NT>(out + (size_t)line * N + dst, v[sg][r]);
            }
        }
    }
}



// Line plan of the single-image passes.  The alternative split of a line
// over threads (PlanVariant<N, 1>) trades per-line latency for occupancy:
// measured on gfx950 (complex64, square images, all counts alike), it is
// faster for 192 always, for 256, 384 and 768 when few lines are in flight,
// and for 64, 512 and 1024 when many are; `lines` = lines of the pass times
// images.  (Complex128: alt_plan_c128; the other lengths keep LinePlan<N>.)
// The backward sweep's paired passes follow the same rule except at 1024,
// where their two signals make the alternative slower at every count
// measured.
inline bool alt_plan(int N, long long lines) {
    switch (N) {
        case 64: return lines >= 1024;
        case 192: return true;
        case 256: return lines <= 4096;
        case 384: return lines <= 3072;
        case 512: return lines >= 2048;
        case 768: return lines <= 1536;
        case 1024: return lines >= 32768;
        default: return false;
    }
}

// Complex128 single-image passes: the alternative split is faster at every
// image count measured (1 to 64) for 64, 192, 256, 384 and 768 (FP64 line
// DFTs gain more from the shorter per-thread chains: one image of 192^2
// 69.5 -> 40.5 us, 256^2 42.7 -> 30.0, 768^2 99.5 -> 68.0) and slower for
// 128 (29.2 -> 46.0 us) and 512.
constexpr bool alt_plan_c128(int N) { return N == 64 || N == 192 || N == 256 || N == 384 || N == 768; }

template <typename P>
constexpr int row_lines_of() {
    return P::TPL >= 256 ? 1 : 256 / P::TPL;
}
template <typename T, int N>
constexpr int row_lines() {
    return row_lines_of<LinePlan<N>>();
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


ChirpArg to_arg(const ChirpTurns& c) { return {c.c11, c.c12, c.c22, c.c00, c.nonzero}; }

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

// Fills this translation unit's twiddle tables on the current device.
hipError_t init_twiddles_here() {
    hipLaunchKernelGGL(init_twiddles_kernel, dim3((kTwiddleN + 255) / 256), dim3(256), 0, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}

}  // namespace
}  // namespace nslct
