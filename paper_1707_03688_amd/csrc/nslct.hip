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
#include <mutex>
#include <new>
#include <string>

#include "fft_engine.hpp"
#include "nslct.h"
#include "planner.hpp"

using namespace nslct;

struct nslct_plan_s {
    PlanData d;
};

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
        sincospi(2.0 * k / kTwiddleN, &s, &c);
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
};

// sin/cos of 2 pi * phase, phase in 64-bit fixed-point turns.
__device__ __forceinline__ cplx<float> turns_cs(uint64_t ph, float scale) {
    const float t = (float)(int32_t)(ph >> 32) * 0x1p-32f;  // [-1/2, 1/2)
    float s, c;
    sincospif(2.0f * t, &s, &c);
    return {c * scale, s * scale};
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

template <typename T, int N, bool COL, int LINES>
__global__ void __launch_bounds__(LinePlan<N>::TPL* LINES) nslct_pass(PassArgs<T> a) {
    constexpr int TPL = LinePlan<N>::TPL;
    using F = LineFFT<T, N, TPL>;
    constexpr int E = F::E;
    constexpr int R0 = F::R0;
    constexpr int LL = lds_line_elems<N>();
    __shared__ cplx<T> lds_all[LINES * LL];

    const int tid = threadIdx.x;
    const int slot = COL ? tid % LINES : tid / TPL;
    const int t = COL ? tid / LINES : tid % TPL;
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int line = tile * LINES + slot;
    const bool active = line < a.nlines;
    cplx<T>* lds = lds_all + slot * LL;
    const cplx<T>* __restrict__ tw = twiddles<T>();
    const size_t img = blockIdx.y;
    const cplx<T>* __restrict__ in = a.in + img * a.img_stride;
    cplx<T>* __restrict__ out = a.out + img * a.img_stride;

    auto addr = [&](int p) -> size_t {
        return COL ? (size_t)p * a.nlines + line : (size_t)line * N + p;
    };
    auto pos = [&](int r) { return t + TPL * (r / R0) + (r % R0) * (N / R0); };

    cplx<T> v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int p = pos(r);
        const int src = a.load_remap ? (p + N / 2) & (N - 1) : p;
        v[r] = active ? in[addr(src)] : cplx<T>{0, 0};
    }

    const int nl = a.nlines;
    const int lc = a.line_centered ? line - nl / 2 : (line >= (nl + 1) / 2 ? line - nl : line);
    auto chirp = [&](const ChirpArg& c, T scale) {
        const uint64_t l64 = (uint64_t)(int64_t)lc;
        const uint64_t A = (COL ? c.c22 : c.c11) * (l64 * l64);
        const uint64_t Bc = c.c12 * l64;
        const uint64_t Q = COL ? c.c11 : c.c22;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int e = p >= (N + 1) / 2 ? p - N : p;
            const uint64_t e64 = (uint64_t)(int64_t)e;
            const uint64_t ph = A + Bc * e64 + Q * (uint64_t)(uint32_t)(e * e);
            v[r] = cmul(v[r], turns_cs(ph, scale));
        }
    };

    if (a.pre.on) chirp(a.pre, (T)1);
    if (a.sign1 < 0)
        F::template dft<-1>(v, lds, t, tw);
    else
        F::template dft<+1>(v, lds, t, tw);
    if (a.mid_on) {
        if (a.mid.on) {
            chirp(a.mid, a.scale);
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) v[r] = {v[r].re * a.scale, v[r].im * a.scale};
        }
    }
    if (a.has_t2) {
        if (a.sign2 < 0)
            F::template dft<-1>(v, lds, t, tw);
        else
            F::template dft<+1>(v, lds, t, tw);
    }
    if (active) {
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = pos(r);
            const int dst = a.store_remap ? (p + N / 2) & (N - 1) : p;
            out[addr(dst)] = v[r];
        }
    }
}

template <typename T, int N>
constexpr int row_lines() {
    return LinePlan<N>::TPL >= 256 ? 1 : 256 / LinePlan<N>::TPL;
}
template <typename T, int N>
constexpr int col_lines() {
    constexpr int cmin = sizeof(T) == 4 ? 4 : 2;
    constexpr int c = 256 / LinePlan<N>::TPL;
    return c > cmin ? c : cmin;
}

template <typename T, int N, bool COL>
hipError_t launch_t(const PassArgs<T>& a, int count, hipStream_t s) {
    constexpr int L = COL ? col_lines<T, N>() : row_lines<T, N>();
    static_assert(L * lds_line_elems<N>() * sizeof(cplx<T>) <= 160 * 1024, "LDS budget");
    dim3 grid((a.nlines + L - 1) / L, count);
    dim3 block(LinePlan<N>::TPL * L);
    hipLaunchKernelGGL((nslct_pass<T, N, COL, L>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T, bool COL>
hipError_t launch_n(int N, const PassArgs<T>& a, int count, hipStream_t s) {
    switch (N) {
        case 2: return launch_t<T, 2, COL>(a, count, s);
        case 4: return launch_t<T, 4, COL>(a, count, s);
        case 8: return launch_t<T, 8, COL>(a, count, s);
        case 16: return launch_t<T, 16, COL>(a, count, s);
        case 32: return launch_t<T, 32, COL>(a, count, s);
        case 64: return launch_t<T, 64, COL>(a, count, s);
        case 128: return launch_t<T, 128, COL>(a, count, s);
        case 256: return launch_t<T, 256, COL>(a, count, s);
        case 512: return launch_t<T, 512, COL>(a, count, s);
        case 1024: return launch_t<T, 1024, COL>(a, count, s);
        case 2048: return launch_t<T, 2048, COL>(a, count, s);
        case 4096: return launch_t<T, 4096, COL>(a, count, s);
        default: return hipErrorInvalidValue;
    }
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

template <typename T>
PassArgs<T> pass_args(const PlanData& d, int dir, int pass, const void* in, void* out) {
    const Chain5& c = d.dir[dir];
    PassArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.in = (const cplx<T>*)in;
    a.out = (cplx<T>*)out;
    a.img_stride = (long long)d.Nx * d.Ny;
    const bool col = (pass == 1 || pass == 3);
    a.nlines = col ? d.Ny : d.Nx;
    a.pre.on = 0;
    a.mid.on = 0;
    a.scale = (T)1;
    switch (pass) {
        case 0:
            a.load_remap = 1;
            a.line_centered = 1;
            a.pre = to_arg(c.turns[0]);
            a.sign1 = -1;
            break;
        case 1:
        case 3:
            a.load_remap = pass == 1;
            a.store_remap = pass == 3;
            a.line_centered = 0;
            a.sign1 = -1;
            a.mid_on = 1;
            a.mid = to_arg(c.turns[pass]);
            a.scale = (T)(1.0 / d.Nx);
            a.has_t2 = 1;
            a.sign2 = +1;
            break;
        case 2:
            a.sign1 = +1;
            a.mid_on = 1;
            a.mid = to_arg(c.turns[2]);
            a.scale = (T)(1.0 / d.Ny);
            a.has_t2 = 1;
            a.sign2 = -1;
            break;
        case 4:
            a.store_remap = 1;
            a.line_centered = 1;
            a.sign1 = +1;
            a.mid_on = 1;
            a.mid = to_arg(c.turns[4]);
            a.scale = (T)(1.0 / d.Ny);
            break;
    }
    return a;
}

template <typename T>
hipError_t launch_pass_typed(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s) {
    const PassArgs<T> a = pass_args<T>(d, dir, pass, in, out);
    const bool col = (pass == 1 || pass == 3);
    return col ? launch_n<T, true>(d.Nx, a, count, s) : launch_n<T, false>(d.Ny, a, count, s);
}

hipError_t launch_pass(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                       hipStream_t s) {
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
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    for (int pass = 0; pass < 5; ++pass) {
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
    if (pass < 0 || pass > 4) return fail(NSLCT_E_ARG, "pass must be in [0, 4]");
    if (count < 1 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [1, 65535]");
    int rc = check_ptrs(in, out);
    if (rc) return rc;
    rc = ensure_device_ready();
    if (rc) return rc;
    hipError_t e = launch_pass(plan->d, direction, pass, count, in, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("pass launch: ") + hipGetErrorString(e));
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
