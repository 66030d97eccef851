// Backward sweep of the differentiable transform: the inverse chain run on
// the forward output and on the incoming gradient together, with the
// gradient sums of every chirp point, and the host steps that turn them into
// dLoss / dtheta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "internal.hpp"
#include "pass_kernels.hpp"
#include "bluestein.hpp"

using namespace nslct;

namespace {

// Backward sweep: the inverse chain applied to the forward output G and to
// the incoming gradient at once, with the gradient sums at every chirp point.
template <typename T, int N, bool COL, int LINES, int V>
__global__ void __launch_bounds__((PlanVariant<N, V>::TPL * LINES)) nslct_pair_pass(PassArgs<T> a) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<N>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    pass_body<T, N, COL, LINES, 2, false, PlanVariant<N, V>>(a, tile, (size_t)blockIdx.y * a.img_stride, lds_all);
}

#define NSLCT_PAIR_SIZES(X) X(8) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

bool pair_native_size(int n) {
    switch (n) {
#define NSLCT_PAIR_OK(v) case v:
        NSLCT_PAIR_SIZES(NSLCT_PAIR_OK)
#undef NSLCT_PAIR_OK
        return true;
        default:
            return false;
    }
}
// Sides of the backward sweep: the native ones above and every length up to
// 2048 without a native plan (Bluestein line DFTs).
bool pair_size_ok(int n) { return pair_native_size(n) || (n >= 2 && n <= 2048 && !native_line(n)); }

// Paired Bluestein pass (lines without a native plan).
template <typename T, int M, bool COL, int LINES>
__global__ void __launch_bounds__(BsPlan<M>::TPL* LINES) nslct_pair_bs_pass(PassArgs<T> a, BsArgs<T> bs) {
    __shared__ cplx<T> lds_all[LINES * lds_line_elems<M>()];
    const int tile = COL ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    bs_body<T, M, COL, LINES, 2>(a, bs, tile, (size_t)blockIdx.y * a.img_stride, lds_all);
}
template <typename T, int M, bool COL>
hipError_t launch_pair_bs_m(const PassArgs<T>& a, const BsArgs<T>& bs, int count, hipStream_t s) {
    constexpr int L = bs_tile_lines<T, M, COL>();
    hipLaunchKernelGGL((nslct_pair_bs_pass<T, M, COL, L>), dim3((a.nlines + L - 1) / L, count),
                       dim3(BsPlan<M>::TPL * L), 0, s, a, bs);
    return hipGetLastError();
}
template <typename T, bool COL>
hipError_t launch_pair_bs(int N, const PassArgs<T>& a, int count, hipStream_t s) {
    const int M = bluestein_length(N);
    const void* tabp = nullptr;
    if (bs_tables(N, M, sizeof(T) == 8, &tabp) != NSLCT_OK) return hipErrorInvalidValue;
    const BsArgs<T> bs{N, (const cplx<T>*)tabp};
    switch (M) {
        case 8: return launch_pair_bs_m<T, 8, COL>(a, bs, count, s);
        case 16: return launch_pair_bs_m<T, 16, COL>(a, bs, count, s);
        case 32: return launch_pair_bs_m<T, 32, COL>(a, bs, count, s);
        case 64: return launch_pair_bs_m<T, 64, COL>(a, bs, count, s);
        case 128: return launch_pair_bs_m<T, 128, COL>(a, bs, count, s);
        case 256: return launch_pair_bs_m<T, 256, COL>(a, bs, count, s);
        case 512: return launch_pair_bs_m<T, 512, COL>(a, bs, count, s);
        case 1024: return launch_pair_bs_m<T, 1024, COL>(a, bs, count, s);
        case 2048: return launch_pair_bs_m<T, 2048, COL>(a, bs, count, s);
        case 4096: return launch_pair_bs_m<T, 4096, COL>(a, bs, count, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int N, bool COL, int V>
hipError_t launch_pair_v(const PassArgs<T>& a, int count, hipStream_t s) {
    constexpr int TPL = PlanVariant<N, V>::TPL;
    constexpr int L = COL ? (col_lines<T, N>() * LinePlan<N>::TPL + TPL - 1) / TPL : row_lines_of<PlanVariant<N, V>>();
    hipLaunchKernelGGL((nslct_pair_pass<T, N, COL, L, V>), dim3((a.nlines + L - 1) / L, count), dim3(TPL * L), 0, s,
                       a);
    return hipGetLastError();
}

template <typename T, bool COL>
hipError_t launch_pair_n(int N, const PassArgs<T>& a, int count, int plan_count, hipStream_t s) {
    switch (N) {
#define NSLCT_PAIR_LAUNCH(v)                                                                   \
    case v:                                                                                    \
        if constexpr (sizeof(T) == 4 && PlanVariant<v, 1>::exists)                             \
            if (v != 1024 && alt_plan(v, (long long)a.nlines * plan_count))                   \
                return launch_pair_v<T, v, COL, 1>(a, count, s);                               \
        return launch_pair_v<T, v, COL, 0>(a, count, s);
        NSLCT_PAIR_SIZES(NSLCT_PAIR_LAUNCH)
#undef NSLCT_PAIR_LAUNCH
        default:
            return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t run_backward_t(const PlanData& d, int count, int plan_count, const void* G, const void* gout, void* work, void* gx,
                          double* sums, hipStream_t s) {
    for (int pass = 0; pass < 5; ++pass) {
        PassArgs<T> a = pass_args<T>(d, 1, pass, pass == 0 ? G : work, work);
        a.in2 = (const cplx<T>*)(pass == 0 ? gout : gx);
        a.out2 = (cplx<T>*)gx;
        a.acc = sums + 3 * pass;
        const bool col = (pass == 1 || pass == 3);
        const int N = col ? d.Nx : d.Ny;
        const hipError_t e = !pair_native_size(N) ? (col ? launch_pair_bs<T, true>(N, a, count, s)
                                                         : launch_pair_bs<T, false>(N, a, count, s))
                             : col ? launch_pair_n<T, true>(N, a, count, plan_count, s)
                                   : launch_pair_n<T, false>(N, a, count, plan_count, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

__global__ void zero_f64(double* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Argument checks shared by the backward entry points.
int check_backward(nslct_plan_t plan, int count, const void* G, const void* grad_out, const void* grad_x) {
    if (!plan) return fail(NSLCT_E_ARG, "null plan");
    if (count < 1 || count > 65535) return fail(NSLCT_E_ARG, "count must be in [1, 65535]");
    int rc = check_ptrs(G, grad_out);
    if (!rc) rc = check_ptrs(grad_x, grad_x);
    if (rc) return rc;
    const PlanData& d = plan->d;
    if (d.precision != NSLCT_C64 && d.precision != NSLCT_C128)
        return fail(NSLCT_E_UNSUPPORTED, "backward runs complex64 or complex128 plans");
    if (!pair_size_ok(d.Nx) || !pair_size_ok(d.Ny))
        return fail(NSLCT_E_SIZE, "backward sides must be 8..1024 (2^k), 48, 96, 192, 384, 768, or a length up to 2048 without a native plan");
    if (d.st.type == 7) return fail(NSLCT_E_UNSUPPORTED, "the backward sweep runs five-slot chains (not type 7)");
    if (grad_x == G) return fail(NSLCT_E_ARG, "grad_x must be distinct from G");
    return NSLCT_OK;
}

// Bluestein tables of the plan's non-native axes on the current device
// (made on first use; host work and a device allocation).
int pair_tables(const PlanData& d) {
    for (int n : {d.Nx, d.Ny}) {
        if (pair_native_size(n)) continue;
        const void* tabp = nullptr;
        const int rc = bs_tables(n, bluestein_length(n), d.precision == NSLCT_C128, &tabp);
        if (rc) return rc;
    }
    return NSLCT_OK;
}

// d(stage entries)/d(theta) of the plan, computed on first use.
int plan_jac(nslct_plan_t plan, const double** jac) {
    std::lock_guard<std::mutex> lk(plan->jac_mu);
    if (!plan->jac_done) {
        plan->jac_rc = plan_theta_jacobian(plan->d, plan->jac, &plan->jac_err);
        plan->jac_done = true;
    }
    if (plan->jac_rc) return fail(plan->jac_rc, plan->jac_err);
    *jac = plan->jac;
    return NSLCT_OK;
}

// The paired sweep of `count` images through a work image region of `chunk`
// images (work holds chunk images; the images are processed chunk by
// chunk), accumulating into the device sums[15] (cleared here first).  The
// line plan of the passes follows `count` (the images of the call), so a
// chunked sweep computes every image with the same code as a whole one.
hipError_t sweep_chunks(const PlanData& d, int count, int chunk, const void* G, const void* gout, void* work,
                        void* gx, double* sums, hipStream_t s) {
    hipLaunchKernelGGL(zero_f64, dim3(1), dim3(64), 0, s, sums, 15);
    hipError_t e = hipGetLastError();
    const size_t es = d.precision == NSLCT_C128 ? 16 : 8;
    const size_t img = (size_t)d.Nx * d.Ny * es;
    for (int i0 = 0; e == hipSuccess && i0 < count; i0 += chunk) {
        const int n = std::min(chunk, count - i0);
        const char* g = (const char*)G + i0 * img;
        const char* go = (const char*)gout + i0 * img;
        char* x = (char*)gx + i0 * img;
        e = d.precision == NSLCT_C128 ? run_backward_t<double>(d, n, count, g, go, work, x, sums, s)
                                      : run_backward_t<float>(d, n, count, g, go, work, x, sums, s);
    }
    return e;
}

// Host part: the 15 sums -> dLoss/d(stage entries) -> dLoss/dtheta.
void finish_theta(const PlanData& d, const double* jac, const double sums[15], double grad_theta[10]) {
    double gst[12];
    stage_gradient(d, sums, gst);
    theta_gradient(jac, gst, grad_theta);
}

constexpr size_t kNoallocWorkBytes = (size_t)16 << 20;
constexpr size_t kNoallocSumsBytes = 256;

void* g_scratch[64] = {};  // device address of `scratch`, written once per device under the set-up lock

}  // namespace

// Scratch of the allocation-free backward entry point: the 15 gradient sums
// (first 256 bytes) and a work region of kNoallocWorkBytes for the inverse
// chain of G.  Each device holds its own copy of the array.  Host code never
// passes `scratch` itself to a kernel or a copy (on the host the name is a
// stand-in, not a device address): it uses g_scratch[device], obtained with
// hipGetSymbolAddress at the device's set-up.
static __device__ __align__(256) unsigned char scratch[kNoallocSumsBytes + kNoallocWorkBytes];

namespace nslct {
hipError_t init_tables_backward() {
    hipError_t e = init_twiddles_here();
    if (e != hipSuccess) return e;
    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
    return hipSuccess;
}
}  // namespace nslct

extern "C" {

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
        return fail(NSLCT_E_SIZE, "backward sides must be 8..1024 (2^k), 48, 96, 192, 384, 768, or a length up to 2048 without a native plan");
    if (d.st.type == 7) return fail(NSLCT_E_UNSUPPORTED, "the backward sweep runs five-slot chains (not type 7)");
    if (work == grad_x || work == G || work == grad_out || grad_x == G)
        return fail(NSLCT_E_ARG, "work and grad_x must be distinct from each other and from G");
    rc = ensure_device_ready();
    if (!rc) rc = pair_tables(d);
    if (rc) return rc;
    const hipError_t e = d.precision == NSLCT_C128
                             ? run_backward_t<double>(d, count, count, G, grad_out, work, grad_x, sums, (hipStream_t)stream)
                             : run_backward_t<float>(d, count, count, G, grad_out, work, grad_x, sums, (hipStream_t)stream);
    return e == hipSuccess ? NSLCT_OK : fail(NSLCT_E_HIP, std::string("backward launch: ") + hipGetErrorString(e));
}

int nslct_backward_theta(nslct_plan_t plan, int count, const void* G, const void* grad_out, void* grad_x,
                         double grad_theta[10], void* stream) {
    int rc = check_backward(plan, count, G, grad_out, grad_x);
    if (rc) return rc;
    const PlanData& d = plan->d;
    const double* jac = nullptr;
    if (grad_theta) {
        rc = plan_jac(plan, &jac);
        if (rc) return rc;
    }
    rc = ensure_device_ready();
    if (!rc) rc = pair_tables(d);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t es = d.precision == NSLCT_C128 ? 16 : 8;
    const size_t work_bytes = (size_t)count * d.Nx * d.Ny * es;
    void* buf = nullptr;
    hipError_t e = hipMallocAsync(&buf, work_bytes + 256, s);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("backward work image: ") + hipGetErrorString(e));
    double* sums = (double*)buf;
    void* work = (char*)buf + 256;
    double host[15] = {};
    e = sweep_chunks(d, count, count, G, grad_out, work, grad_x, sums, s);
    if (e == hipSuccess && grad_theta) e = hipMemcpyAsync(host, sums, sizeof host, hipMemcpyDeviceToHost, s);
    const hipError_t ef = hipFreeAsync(buf, s);
    if (e == hipSuccess) e = ef;
    if (e == hipSuccess && grad_theta) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("backward: ") + hipGetErrorString(e));
    if (grad_theta) finish_theta(d, jac, host, grad_theta);
    return NSLCT_OK;
}

int nslct_backward_theta_noalloc(nslct_plan_t plan, int count, const void* G, const void* grad_out,
                                 void* grad_x, double grad_theta[10], void* stream) {
    int rc = check_backward(plan, count, G, grad_out, grad_x);
    if (rc) return rc;
    const PlanData& d = plan->d;
    const size_t es = d.precision == NSLCT_C128 ? 16 : 8;
    const size_t img = (size_t)d.Nx * d.Ny * es;
    if (img > kNoallocWorkBytes)
        return fail(NSLCT_E_SIZE, "an image is larger than the 16 MiB scratch work region");
    if (!pair_native_size(d.Nx) || !pair_native_size(d.Ny))
        return fail(NSLCT_E_SIZE, "the allocation-free backward takes native lengths (Bluestein tables are allocated)");
    const double* jac = nullptr;
    if (grad_theta) {
        rc = plan_jac(plan, &jac);
        if (rc) return rc;
    }
    rc = ensure_device_ready();
    if (rc) return rc;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    unsigned char* base = (unsigned char*)g_scratch[dev];
    if (!base) return fail(NSLCT_E_HIP, "scratch address of this device is unknown");
    hipStream_t s = (hipStream_t)stream;
    const int chunk = (int)std::min<size_t>((size_t)count, kNoallocWorkBytes / img);
    double host[15] = {};
    e = sweep_chunks(d, count, chunk, G, grad_out, base + kNoallocSumsBytes, grad_x, (double*)base, s);
    if (e == hipSuccess && grad_theta) e = hipMemcpyAsync(host, base, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && grad_theta) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("backward: ") + hipGetErrorString(e));
    if (grad_theta) finish_theta(d, jac, host, grad_theta);
    return NSLCT_OK;
}

int nslct_plan_theta_jacobian(nslct_plan_t plan, double jac[12 * 10]) {
    if (!plan || !jac) return fail(NSLCT_E_ARG, "null argument");
    const double* j = nullptr;
    const int rc = plan_jac(plan, &j);
    if (rc) return rc;
    std::memcpy(jac, j, sizeof(double) * 120);
    return NSLCT_OK;
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

}  // extern "C"
