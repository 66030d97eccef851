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

#include "internal.hpp"
#include "pass_kernels.hpp"
#include "bluestein.hpp"

using namespace nslct;

namespace nslct {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

}  // namespace nslct

namespace {

// Per-device one-time setup (the twiddle tables of every translation unit).
std::mutex g_init_mu;
bool g_inited[64] = {};

}  // namespace

int nslct::ensure_device_ready() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= 64) return fail(NSLCT_E_HIP, "device index out of range");
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (g_inited[dev]) return NSLCT_OK;
    e = init_twiddles_here();
    if (e == hipSuccess) e = init_tables_batched();
    if (e == hipSuccess) e = init_tables_split();
    if (e == hipSuccess) e = init_tables_backward();
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("twiddle init: ") + hipGetErrorString(e));
    g_inited[dev] = true;
    return NSLCT_OK;
}

namespace {

template <typename T, int N, bool COL, int LINES, bool X3, int V, bool NT = false>
__global__ void __launch_bounds__((PlanVariant<N, V>::TPL * LINES)) nslct_pass(PassArgs<T> a) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<N>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    pass_body<T, N, COL, LINES, 1, X3, PlanVariant<N, V>, NT>(a, tile, (size_t)blockIdx.y * a.img_stride,
                                                               lds_all);
}
template <typename T, int N, bool COL, bool X3, int V, bool NT = false>
hipError_t launch_tv(const PassArgs<T>& a, int count, hipStream_t s) {
    constexpr int TPL = PlanVariant<N, V>::TPL;
    // Column tiles keep the thread count of the LinePlan tile; row tiles
    // 256 threads.
    constexpr int L = COL ? (col_lines<T, N>() * LinePlan<N>::TPL + TPL - 1) / TPL : row_lines_of<PlanVariant<N, V>>();
    static_assert(L * lds_line_elems<N>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    dim3 grid((a.nlines + L - 1) / L, count);
    dim3 block(TPL * L);
    hipLaunchKernelGGL((nslct_pass<T, N, COL, L, X3, V, NT>), grid, block, 0, s, a);
    return hipGetLastError();
}
template <typename T, int N, bool COL, bool X3 = false>
hipError_t launch_t(const PassArgs<T>& a, int count, hipStream_t s) {
    if constexpr (sizeof(T) == 4 && PlanVariant<N, 1>::exists) {
        // 4096-long rows with one line DFT (the first and last pass of a
        // chain) run faster on 128 threads; the two-DFT middle pass and the
        // column tiles keep the 256-thread plan.
        const bool alt = N == 4096 ? (!COL && !X3 && !a.has_t2) : alt_plan(N, (long long)a.nlines * count);
        if (alt) return launch_tv<T, N, COL, X3, 1>(a, count, s);
    }
    if constexpr (sizeof(T) == 8 && alt_plan_c128(N)) return launch_tv<T, N, COL, X3, 1>(a, count, s);
    if constexpr (sizeof(T) == 4 && N == 1024 && !X3) {
        // One 1024^2 complex64 image: streaming sample loads and stores leave
        // less dirty data in the L2s for each pass's end to write back, which
        // took the five-pass chain from 54.5 to 51.6 us on gfx950 (with more
        // images per launch, where bandwidth rather than the pass boundaries
        // sets the time, they were slower: 8 images 37 k -> 21 k NsLCT/s).
        if (count == 1) return launch_tv<T, N, COL, X3, 0, true>(a, count, s);
    }
    return launch_tv<T, N, COL, X3, 0>(a, count, s);
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
        const uint64_t A0 = a.mid.c22 * (l64 * l64) + a.mid.c00;
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


template <typename T>
hipError_t launch_pass_typed(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s);
}  // namespace

// ---------------------------------------------------------------- Bluestein
// Host side of the Bluestein line DFTs (bluestein.hpp): which lengths need
// them, their padded length and the FFT_M(b) / M tables.
namespace nslct {

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

namespace {
std::mutex g_bs_mu;
std::vector<std::pair<std::array<int, 4>, void*>> g_bs;  // (device, N, M, fp64) -> table
}  // namespace

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

}  // namespace nslct

namespace {

// One Bluestein pass of a single-image launch: tile from the XCD-aware
// order, image from blockIdx.y.
template <typename T, int M, bool COL, int LINES>
__global__ void __launch_bounds__(BsPlan<M>::TPL* LINES) nslct_bs_pass(PassArgs<T> a, BsArgs<T> bs) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<M>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    bs_body<T, M, COL, LINES>(a, bs, tile, (size_t)blockIdx.y * a.img_stride, lds_all);
}

template <typename T, int M, bool COL>
hipError_t launch_bs_t(const PassArgs<T>& a, const BsArgs<T>& b, int count, hipStream_t s) {
    constexpr int L = bs_tile_lines<T, M, COL>();
    static_assert(L * lds_line_elems<M>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    hipLaunchKernelGGL((nslct_bs_pass<T, M, COL, L>), dim3((a.nlines + L - 1) / L, count),
                       dim3(BsPlan<M>::TPL * L), 0, s, a, b);
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
// chain (CM-CC-CM, LC) in c64 / c128 at native line lengths, else the
// five-pass chain (for a reduced chain its five-slot form, which the
// Bluestein pass kernels run at any length).
int plan_passes(const PlanData& d) {
    const bool split = d.precision == NSLCT_C64_SPLIT_F16 || d.precision == NSLCT_C64_SPLIT_BF16;
    const bool native = native_line(d.Nx) && native_line(d.Ny);
    return (!split && native && d.prog[0].npass > 0) ? d.prog[0].npass : 5;
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

// ------------------------------------------ small images resident in LDS
// A square image of 32 x 32 or 64 x 64 samples (complex64 or complex128)
// fits one workgroup's LDS together with the line-exchange buffer of all its
// lines: the whole chain then runs in one launch with one workgroup per
// image, each pass reading and writing the LDS copy through the same pass
// code as the global passes (line plan LinePlan<N>, so the results are those
// of the pass launches on that plan, bit for bit), and the image crosses
// global memory once each way instead of once per pass.  One workgroup does
// the work of every pass of its image, so this pays when the launches of the
// pass path are the cost (32 x 32) or when many images fill the chip
// (measured on gfx950, per image: 64 x 64 complex64 0.161 -> 0.092 us at 256
// images, on par at 16; complex128 0.207 -> 0.143 us at 256, slower at 64 and
// below; 32 x 32 faster at every count, 19 -> 12 us for one complex64
// image).  128 x 128 complex64 would leave room for only 16 lines per tile,
// and the serial tiles made it 6x slower.
template <typename T>
struct ResidentArgs {
    PassArgs<T> p[5];  // the passes of the chain, in order (in / out unused)
    int col[5];        // column pass
    int x3[5];         // three line DFTs (reduced schedules)
    int npass;
    const cplx<T>* in;
    cplx<T>* out;
};

template <typename T, int N>
__global__ void __launch_bounds__(N * LinePlan<N>::TPL) nslct_resident(ResidentArgs<T> r) {
    constexpr int NT = N * LinePlan<N>::TPL;  // all N lines of a pass at once
    __shared__ cplx<T> img[N * N];
    __shared__ cplx<T> xch[N * lds_line_elems<N>()];
    const size_t off = (size_t)blockIdx.x * (N * N);
    for (int i = threadIdx.x; i < N * N; i += NT) img[i] = r.in[off + i];
    __syncthreads();
#pragma nounroll
    for (int k = 0; k < r.npass; ++k) {
        // Every line of the pass is read into registers before any is
        // written (each line is one wavefront's), so the passes run in
        // place; the barrier orders the passes (the next reads other lines).
        const PassArgs<T>& a = r.p[k];
        if (r.col[k]) {
            if (r.x3[k])
                pass_body<T, N, true, N, 1, true>(a, 0, 0, xch, img);
            else
                pass_body<T, N, true, N>(a, 0, 0, xch, img);
        } else {
            if (r.x3[k])
                pass_body<T, N, false, N, 1, true>(a, 0, 0, xch, img);
            else
                pass_body<T, N, false, N>(a, 0, 0, xch, img);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < N * N; i += NT) r.out[off + i] = img[i];
}

template <typename T, int N>
hipError_t launch_resident_t(const ResidentArgs<T>& r, int count, hipStream_t s) {
    static_assert(N * LinePlan<N>::TPL <= 1024, "one workgroup per image");
    static_assert(N * N * sizeof(cplx<T>) + N * lds_line_elems<N>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    hipLaunchKernelGGL((nslct_resident<T, N>), dim3(count), dim3(N * LinePlan<N>::TPL), 0, s, r);
    return hipGetLastError();
}

// Where the resident kernel runs a chain (see above): square 32 x 32 always,
// 64 x 64 from 32 (complex64) or 128 (complex128) images per call.
bool resident_applies(const PlanData& d, int count) {
    if (d.Nx != d.Ny) return false;
    if (d.precision != NSLCT_C64 && d.precision != NSLCT_C128) return false;
    if (d.Nx == 32) return true;
    if (d.Nx == 64) return count >= (d.precision == NSLCT_C64 ? 32 : 128);
    return false;
}

template <typename T>
hipError_t launch_resident(const PlanData& d, int dir, int count, const void* in, void* out, hipStream_t s) {
    ResidentArgs<T> r{};
    r.npass = plan_passes(d);
    for (int k = 0; k < r.npass; ++k) {
        if (r.npass != 5) {  // the program of a reduced chain (as launch_pass)
            const ProgPass& q = d.prog[dir].p[k];
            r.p[k] = program_args<T>(d, dir, k, nullptr, nullptr);
            r.col[k] = q.col ? 1 : 0;
            r.x3[k] = q.ndft == 3 ? 1 : 0;
        } else {
            r.p[k] = pass_args<T>(d, dir, k, nullptr, nullptr);
            r.col[k] = (k == 1 || k == 3) ? 1 : 0;
        }
    }
    r.in = (const cplx<T>*)in;
    r.out = (cplx<T>*)out;
    return d.Nx == 32 ? launch_resident_t<T, 32>(r, count, s) : launch_resident_t<T, 64>(r, count, s);
}

hipError_t launch_pass(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                       hipStream_t s) {
    if (plan_passes(d) != 5)
        return d.precision == NSLCT_C128 ? launch_program_pass<double>(d, dir, pass, count, in, out, s)
                                         : launch_program_pass<float>(d, dir, pass, count, in, out, s);
    if (d.precision == NSLCT_C64_SPLIT_F16 || d.precision == NSLCT_C64_SPLIT_BF16)
        return launch_split_pass(d, dir, pass, count, in, out, s);
    return d.precision == NSLCT_C128 ? launch_pass_typed<double>(d, dir, pass, count, in, out, s)
                                     : launch_pass_typed<float>(d, dir, pass, count, in, out, s);
}

}  // namespace

namespace nslct {

int check_ptrs(const void* in, const void* out) {
    if (!in || !out) return fail(NSLCT_E_ARG, "null image pointer");
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15))
        return fail(NSLCT_E_ARG, "image pointers must be 16-byte aligned");
    return NSLCT_OK;
}

int run_chain(nslct_plan_t plan, int dir, int count, const void* in, void* out, void* stream, bool element_aligned) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    if (count < 0 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [0, 65535]");
    int rc = NSLCT_OK;
    if (element_aligned) {
        const uintptr_t es = plan->d.precision == NSLCT_C128 ? 16 : 8;
        if (!in || !out) rc = fail(NSLCT_E_ARG, "null image pointer");
        else if (((uintptr_t)in % es) || ((uintptr_t)out % es))
            rc = fail(NSLCT_E_ARG, "image pointers must be aligned to a sample");
    } else {
        rc = check_ptrs(in, out);
    }
    if (rc) return rc;
    if (count == 0) return NSLCT_OK;
    rc = ensure_device_ready();
    if (!rc) rc = prepare_plan_tables(plan->d);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (resident_applies(plan->d, count)) {
        const hipError_t e = plan->d.precision == NSLCT_C128
                                 ? launch_resident<double>(plan->d, dir, count, in, out, s)
                                 : launch_resident<float>(plan->d, dir, count, in, out, s);
        return e == hipSuccess ? NSLCT_OK : fail(NSLCT_E_HIP, std::string("resident launch: ") + hipGetErrorString(e));
    }
    const int np = plan_passes(plan->d);
    for (int pass = 0; pass < np; ++pass) {
        hipError_t e = launch_pass(plan->d, dir, pass, count, pass == 0 ? in : out, out, s);
        if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("pass launch: ") + hipGetErrorString(e));
    }
    return NSLCT_OK;
}

}  // namespace nslct

namespace {

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

void nslct_opts_default(nslct_opts* o) {
    if (!o) return;
    o->precision = NSLCT_C64;
    o->type_override = 0;
    o->symplectic_tol = 1e-9;
    o->det_min = 1e-6;
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

int nslct_plan_lie(const double abcd0[16], const double theta[10], int Nx, int Ny, double dx, double dy,
                   const nslct_opts* opts, nslct_plan_t* out) {
    if (!abcd0 || !theta || !out) return fail(NSLCT_E_ARG, "null argument");
    *out = nullptr;
    nslct_opts o;
    nslct_opts_default(&o);
    if (opts) o = *opts;
    auto* p = new (std::nothrow) nslct_plan_s;
    if (!p) return fail(NSLCT_E_ARG, "out of host memory");
    std::string err;
    const int rc = build_plan_lie(abcd0, theta, Nx, Ny, dx, dy, o, &p->d, &err);
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

int nslct_plan_prepare(nslct_plan_t plan) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    int rc = ensure_device_ready();
    if (!rc) rc = prepare_plan_tables(plan->d);
    return rc;
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
