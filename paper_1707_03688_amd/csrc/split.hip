// Split-precision passes: line DFTs of 256 or 4096 samples as radix-16
// DFT-as-GEMM stages on the matrix cores with operands split into high + low
// FP16 / BF16 parts and FP32 accumulation (split_fft.hpp); storage complex64,
// chirps exact as in the FP32 path.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "pass_kernels.hpp"
#include "split_fft.hpp"

namespace nslct {
namespace {

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
                                (COL ? c.c11 : c.c22) * (e64 * e64) + c.c00;
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

}  // namespace

hipError_t init_tables_split() { return init_twiddles_here(); }

hipError_t launch_split_pass(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s) {
    const PassArgs<float> a = pass_args<float>(d, dir, pass, in, out);
    const bool col = (pass == 1 || pass == 3);
    const int N = col ? d.Nx : d.Ny;
    if (d.precision == NSLCT_C64_SPLIT_F16)
        return col ? launch_split_n<0, true>(N, a, count, s) : launch_split_n<0, false>(N, a, count, s);
    return col ? launch_split_n<1, true>(N, a, count, s) : launch_split_n<1, false>(N, a, count, s);
}

}  // namespace nslct
