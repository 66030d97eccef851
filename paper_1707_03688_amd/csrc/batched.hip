// Ragged batches: many images, each with its own size and matrix, over one
// packed buffer; per-(pass, line length) launches over XCD-balanced work
// lists, captured in a HIP graph; autotuned at creation.
#include <hip/hip_runtime.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pass_kernels.hpp"
#include "bluestein.hpp"

using namespace nslct;

namespace {

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

// Line lengths the batched kernel handles (all with TPL <= 64).
#define NSLCT_BATCH_SIZES(X) X(64) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

// Tile widths of a work item: W = 0, 1, 2 give 256, 512, 1024 threads, i.e.
// (256 << W) / TPL lines (row passes W <= 1), for line plan V (PlanVariant:
// 0 the single-image plan, 1 the alternative).  A (width, plan) pair is a
// candidate when the plan exists and its lines fit the 160 KB of LDS.
constexpr int kMaxWidth = 2;
constexpr int kPlans = 2;
template <int N, int W, int V>
constexpr int width_lines() {
    return (256 << W) / PlanVariant<N, V>::TPL;
}
template <typename T, int N, bool COL, int W, int V>
constexpr bool width_ok() {
    return PlanVariant<N, V>::exists && (COL || W <= 1) &&
           width_lines<N, W, V>() * lds_line_elems<N>() * (int)sizeof(cplx<T>) <= 160 * 1024;
}

bool batch_native_size(int n) {
    switch (n) {
#define NSLCT_CASE_OK(v) case v:
        NSLCT_BATCH_SIZES(NSLCT_CASE_OK)
#undef NSLCT_CASE_OK
        return true;
        default:
            return false;
    }
}
// Sides the batch takes: the native ones above, and every length up to 2048
// without a native plan (Bluestein line DFTs on M-point lines).
bool batch_size_ok(int n) { return batch_native_size(n) || (n >= 2 && n <= 2048 && !native_line(n)); }

// Lines per work item of a Bluestein group: the single-image tile of the
// M-point line.
template <typename T, int M, bool COL>
constexpr int bs_lines() {
    return bs_tile_lines<T, M, COL>();
}
int host_bs_lines(int M, bool col, bool dbl) {
    switch (M) {
#define NSLCT_CASE_BSL(m)                                                                              \
    case m:                                                                                            \
        return dbl ? (col ? bs_lines<double, m, true>() : bs_lines<double, m, false>())                \
                   : (col ? bs_lines<float, m, true>() : bs_lines<float, m, false>());
        NSLCT_CASE_BSL(8) NSLCT_CASE_BSL(16) NSLCT_CASE_BSL(32) NSLCT_CASE_BSL(64) NSLCT_CASE_BSL(128)
        NSLCT_CASE_BSL(256) NSLCT_CASE_BSL(512) NSLCT_CASE_BSL(1024) NSLCT_CASE_BSL(2048) NSLCT_CASE_BSL(4096)
#undef NSLCT_CASE_BSL
        default:
            return 1;
    }
}

template <int N, int V>
bool host_width_ok_v(int w, bool col, bool dbl) {
    switch (w) {
        case 0: return dbl ? (col ? width_ok<double, N, true, 0, V>() : width_ok<double, N, false, 0, V>())
                           : (col ? width_ok<float, N, true, 0, V>() : width_ok<float, N, false, 0, V>());
        case 1: return dbl ? (col ? width_ok<double, N, true, 1, V>() : width_ok<double, N, false, 1, V>())
                           : (col ? width_ok<float, N, true, 1, V>() : width_ok<float, N, false, 1, V>());
        case 2: return dbl ? (col ? width_ok<double, N, true, 2, V>() : width_ok<double, N, false, 2, V>())
                           : (col ? width_ok<float, N, true, 2, V>() : width_ok<float, N, false, 2, V>());
        default: return false;
    }
}
template <int N>
bool host_width_ok_n(int w, int v, bool col, bool dbl) {
    switch (v) {
        case 0: return host_width_ok_v<N, 0>(w, col, dbl);
        case 1: return host_width_ok_v<N, 1>(w, col, dbl);
        default: return false;
    }
}
bool host_width_ok(int n, int w, int v, bool col, bool dbl) {
    switch (n) {
#define NSLCT_CASE_W(x) \
    case x:           \
        return host_width_ok_n<x>(w, v, col, dbl);
        NSLCT_BATCH_SIZES(NSLCT_CASE_W)
#undef NSLCT_CASE_W
        default:
            return false;
    }
}
int host_width_lines(int n, int w, int v) {
    switch (n) {
#define NSLCT_CASE_L(x) \
    case x:           \
        return (256 << w) / (v ? PlanVariant<x, 1>::TPL : PlanVariant<x, 0>::TPL);
        NSLCT_BATCH_SIZES(NSLCT_CASE_L)
#undef NSLCT_CASE_L
        default:
            return 1;
    }
}
// The width used before (or without) tuning: 256 threads, complex64 column
// tiles twice as wide (1024-long columns: 8 columns, 64-byte row segments).
int default_width(bool col, bool dbl) { return (col && !dbl) ? 1 : 0; }

// Batched pass over the images of one line length N, L = width_lines<N, W>
// lines per work item.  LOOP: a persistent grid whose workgroups walk the
// group's item list with a grid stride (item i belongs to XCD i mod 8,
// which is also the XCD of every workgroup that visits it: the grid size is
// a multiple of 8); otherwise one workgroup per item, without the loop,
// whose loop-invariant values would otherwise stay in registers across
// iterations.
template <typename T, int N, bool COL, bool LOOP, int W, int V>
__global__ void __launch_bounds__((width_lines<N, W, V>() * PlanVariant<N, V>::TPL))
    nslct_batched_pass(BatchArgs<T> b, const BatchItem* __restrict__ items, const BatchPass<T>* __restrict__ passes) {
    constexpr int L = width_lines<N, W, V>();
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
            pass_body<T, N, COL, L, 1, false, PlanVariant<N, V>>(a, w.tile, (size_t)passes[k].off, lds);
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

// Batched Bluestein pass over the images of one non-native line length
// (all of one M): the same work list and grids as nslct_batched_pass, each
// item through the single-image Bluestein body.
template <typename T, int M, bool COL, bool LOOP>
__global__ void __launch_bounds__((bs_lines<T, M, COL>() * BsPlan<M>::TPL))
    nslct_batched_bs_pass(BatchArgs<T> b, const BatchItem* __restrict__ items, const BatchPass<T>* __restrict__ passes,
                          BsArgs<T> bs) {
    constexpr int L = bs_lines<T, M, COL>();
    __shared__ cplx<T> lds[L * lds_line_elems<M>()];
    auto item = [&](int it) {
        const BatchItem w = items[it];
        if (w.img >= 0) {
            const int k = (w.img * 2 + b.dir) * 5 + b.pass;
            PassArgs<T> a = passes[k].a;
            a.in = b.in;
            a.out = b.out;
            bs_body<T, M, COL, L>(a, bs, w.tile, (size_t)passes[k].off, lds);
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

template <typename T, int M, bool COL>
hipError_t launch_batched_bs_m(const BatchArgs<T>& a, const BsArgs<T>& bs, int grid, hipStream_t s) {
    const dim3 block(bs_lines<T, M, COL>() * BsPlan<M>::TPL);
    if (grid >= a.nitems)
        hipLaunchKernelGGL((nslct_batched_bs_pass<T, M, COL, false>), dim3(a.nitems), block, 0, s, a, a.items,
                           a.passes, bs);
    else
        hipLaunchKernelGGL((nslct_batched_bs_pass<T, M, COL, true>), dim3(grid), block, 0, s, a, a.items, a.passes,
                           bs);
    return hipGetLastError();
}

template <typename T, bool COL>
hipError_t launch_batched_bs(int M, const BatchArgs<T>& a, const BsArgs<T>& bs, int grid, hipStream_t s) {
    switch (M) {
        case 8: return launch_batched_bs_m<T, 8, COL>(a, bs, grid, s);
        case 16: return launch_batched_bs_m<T, 16, COL>(a, bs, grid, s);
        case 32: return launch_batched_bs_m<T, 32, COL>(a, bs, grid, s);
        case 64: return launch_batched_bs_m<T, 64, COL>(a, bs, grid, s);
        case 128: return launch_batched_bs_m<T, 128, COL>(a, bs, grid, s);
        case 256: return launch_batched_bs_m<T, 256, COL>(a, bs, grid, s);
        case 512: return launch_batched_bs_m<T, 512, COL>(a, bs, grid, s);
        case 1024: return launch_batched_bs_m<T, 1024, COL>(a, bs, grid, s);
        case 2048: return launch_batched_bs_m<T, 2048, COL>(a, bs, grid, s);
        case 4096: return launch_batched_bs_m<T, 4096, COL>(a, bs, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int N, bool COL, int W, int V>
hipError_t launch_batched_w(const BatchArgs<T>& a, int grid, hipStream_t s) {
    if constexpr (width_ok<T, N, COL, W, V>()) {
        const dim3 block(width_lines<N, W, V>() * PlanVariant<N, V>::TPL);
        if (grid >= a.nitems)
            hipLaunchKernelGGL((nslct_batched_pass<T, N, COL, false, W, V>), dim3(a.nitems), block, 0, s, a, a.items,
                               a.passes);
        else
            hipLaunchKernelGGL((nslct_batched_pass<T, N, COL, true, W, V>), dim3(grid), block, 0, s, a, a.items,
                               a.passes);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T, bool COL, int N, int V>
hipError_t launch_batched_v(int w, const BatchArgs<T>& a, int grid, hipStream_t s) {
    switch (w) {
        case 0: return launch_batched_w<T, N, COL, 0, V>(a, grid, s);
        case 1: return launch_batched_w<T, N, COL, 1, V>(a, grid, s);
        case 2: return launch_batched_w<T, N, COL, 2, V>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool COL, int N>
hipError_t launch_batched_n(int v, int w, const BatchArgs<T>& a, int grid, hipStream_t s) {
    switch (v) {
        case 0: return launch_batched_v<T, COL, N, 0>(w, a, grid, s);
        case 1: return launch_batched_v<T, COL, N, 1>(w, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool COL>
hipError_t launch_batched_group(int N, int v, int w, const BatchArgs<T>& a, int grid, hipStream_t s) {
    switch (N) {
#define NSLCT_CASE_LAUNCH(x) \
    case x:                  \
        return launch_batched_n<T, COL, x>(v, w, a, grid, s);
        NSLCT_BATCH_SIZES(NSLCT_CASE_LAUNCH)
#undef NSLCT_CASE_LAUNCH
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace

struct nslct_batch_s {
    int count = 0;
    int precision = NSLCT_C64;
    int device = 0;
    size_t total = 0;                 // samples in the packed buffer
    std::vector<long long> offsets;
    std::unique_ptr<nslct_plan_s[]> plans;  // copies of the input plans
    void* d_passes = nullptr;  // BatchPass<T>[count * 10], T by precision
    // Work groups: one per (pass kind, line length).  Row passes ([0]) take
    // lines of length Ny, column passes ([1]) lines of length Nx.
    struct Group {
        int N;
        int nitems;
        int grid;
        BatchItem* items;
        int width;    // tile width index (width_lines)
        int plan;     // line plan (PlanVariant index)
        int M;        // Bluestein line length (0: native N)
        const void* bs_tab;  // Bluestein table of N (device)
        int mult;     // persistent workgroups per CU (0: one per item)
        int cached;   // schedule taken from the schedule cache
        double us;    // measured time of one launch of this group while tuning
    };
    std::vector<Group> groups[2];
    // chain_col[k]: the column group holding exactly the images of row group
    // k, when every row group has one (then each (row group, column group)
    // pair is a set of chains that no other group touches); else empty.
    std::vector<int> chain_col;
    int mult = 0;  // grid override of nslct_batch_set_grid (-1: per-group tuned grids)
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

// One pass of one group (axis col, one line length) on stream st.
template <typename T>
hipError_t launch_group_pass(const nslct_batch_s& b, int col, const nslct_batch_s::Group& g, int dir, int pass,
                             const void* in, void* out, hipStream_t st) {
    BatchArgs<T> a;
    a.in = (const cplx<T>*)in;
    a.out = (cplx<T>*)out;
    a.passes = (const BatchPass<T>*)b.d_passes;
    a.items = g.items;
    a.nitems = g.nitems;
    a.dir = dir;
    a.pass = pass;
    if (g.M) {
        const BsArgs<T> bs{g.N, (const cplx<T>*)g.bs_tab};
        return col ? launch_batched_bs<T, true>(g.M, a, bs, g.grid, st) : launch_batched_bs<T, false>(g.M, a, bs, g.grid, st);
    }
    return col ? launch_batched_group<T, true>(g.N, g.plan, g.width, a, g.grid, st)
               : launch_batched_group<T, false>(g.N, g.plan, g.width, a, g.grid, st);
}

template <typename T>
hipError_t run_batched_t(const nslct_batch_s& b, int dir, const void* in, void* out, hipStream_t s) {
    const size_t nch = b.chain_col.size();
    if (nch > 1 && b.side.size() >= nch) {
        // Independent image sets: each runs its five passes on its own fork
        // stream, joined once at the end, so a set that finishes a pass
        // early goes on to the next instead of waiting for the others.
        hipError_t e = hipEventRecord(b.ev[0], s);
        for (size_t k = 0; k < nch && e == hipSuccess; ++k) e = hipStreamWaitEvent(b.side[k], b.ev[0], 0);
        for (size_t k = 0; k < nch && e == hipSuccess; ++k) {
            for (int pass = 0; pass < 5 && e == hipSuccess; ++pass) {
                const int col = (pass == 1 || pass == 3) ? 1 : 0;
                const auto& g = col ? b.groups[1][b.chain_col[k]] : b.groups[0][k];
                e = launch_group_pass<T>(b, col, g, dir, pass, pass == 0 ? in : out, out, b.side[k]);
            }
            if (e == hipSuccess) e = hipEventRecord(b.ev[1 + k], b.side[k]);
        }
        for (size_t k = 0; k < nch && e == hipSuccess; ++k) e = hipStreamWaitEvent(s, b.ev[1 + k], 0);
        return e;
    }
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
            hipStream_t st = fork ? b.side[k] : s;
            e = launch_group_pass<T>(b, col, gs[k], dir, pass, pass == 0 ? in : out, out, st);
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
std::vector<BatchItem> build_items(const nslct_batch_s& b, bool col, int N, int L) {
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

// (w, v) is a schedule candidate of group g: for a Bluestein group only its
// single tile (w = 0, v = 0).
bool candidate_ok(const nslct_batch_s::Group& g, int w, int v, bool col, bool dbl) {
    return g.M ? (w == 0 && v == 0) : host_width_ok(g.N, w, v, col, dbl);
}
int group_lines(const nslct_batch_s::Group& g, bool col, bool dbl) {
    return g.M ? host_bs_lines(g.M, col, dbl) : host_width_lines(g.N, g.width, g.plan);
}

int grid_for(int mult, int cus, int nitems) {
    const int want = mult == 0 ? nitems : ((mult * cus + 7) / 8) * 8;
    return std::max(8, std::min(want, nitems));
}

// Every group on `mult` workgroups per CU (nslct_batch_set_grid).
void set_grids(nslct_batch_s* b, int mult, int cus) {
    b->mult = mult;
    for (auto& gs : b->groups)
        for (auto& g : gs) {
            g.mult = mult;
            g.grid = grid_for(mult, cus, g.nitems);
        }
}

// (Re)builds and uploads the work list of group g for tile width w and
// line plan v.
hipError_t set_group_width(nslct_batch_s& b, int col, nslct_batch_s::Group& g, int w, int v) {
    const int L = g.M ? host_bs_lines(g.M, col == 1, b.precision == NSLCT_C128) : host_width_lines(g.N, w, v);
    const std::vector<BatchItem> items = build_items(b, col == 1, g.N, L);
    if (g.items) {
        hipError_t e = hipFree(g.items);
        g.items = nullptr;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&g.items, sizeof(BatchItem) * items.size());
    if (e == hipSuccess)
        e = hipMemcpy(g.items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice);
    g.nitems = (int)items.size();
    g.width = w;
    g.plan = v;
    return e;
}

// ------------------------------------------------------------ schedule cache
// The tuned schedule of a group is kept in a text file, one line per
//   <gfx arch> <precision> <axis 0 rows / 1 columns> <N> <items, rounded up
//   to a power of two> <line plan> <width> <mult> <microseconds>
// (lines of any other shape are skipped)
// (file NSLCT_TUNE_CACHE, default $HOME/.cache/nslct/batch_schedule.txt;
// NSLCT_TUNE_CACHE=off disables it).  A batch whose groups are all found
// there is not tuned again.
struct CacheKey {
    std::string arch;
    int prec, col, N, bucket;
};

std::mutex g_cache_mu;

std::string cache_path() {
    const char* env = std::getenv("NSLCT_TUNE_CACHE");
    if (env) return std::string(env) == "off" ? std::string() : std::string(env);
    const char* home = std::getenv("HOME");
    if (!home || !*home) return std::string();
    return std::string(home) + "/.cache/nslct/batch_schedule.txt";
}

int bucket_of(int nitems) {
    int b = 1;
    while (b < nitems) b <<= 1;
    return b;
}

bool cache_lookup(const std::string& path, const CacheKey& k, int* v, int* w, int* mult) {
    if (path.empty()) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string arch, extra;
        int prec, col, N, bucket, vv, ww, mm;
        double us;
        if (!(in >> arch >> prec >> col >> N >> bucket >> vv >> ww >> mm >> us) || (in >> extra)) continue;
        if (arch == k.arch && prec == k.prec && col == k.col && N == k.N && bucket == k.bucket) {
            *v = vv;  // the last entry for a key wins
            *w = ww;
            *mult = mm;
            found = true;
        }
    }
    return found;
}

void cache_store(const std::string& path, const CacheKey& k, int v, int w, int mult, double us) {
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // Create the parent directories (best effort; errors only skip caching).
        std::string dir = path.substr(0, slash);
        for (size_t p = 1; p <= dir.size(); ++p)
            if (p == dir.size() || dir[p] == '/') (void)mkdir(dir.substr(0, p).c_str(), 0755);
    }
    std::ofstream f(path, std::ios::app);
    if (f) f << k.arch << ' ' << k.prec << ' ' << k.col << ' ' << k.N << ' ' << k.bucket << ' ' << v << ' ' << w
             << ' ' << mult << ' ' << us << '\n';
}

std::string device_arch(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a(prop.gcnArchName);
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
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

namespace nslct {
hipError_t init_tables_batched() { return init_twiddles_here(); }
}  // namespace nslct

extern "C" {

int nslct_batch_create(const nslct_plan_t* plans, int count, nslct_batch_t* out) {
    if (!plans || !out || count < 1) return fail(NSLCT_E_ARG, "need plans, count >= 1 and out");
    *out = nullptr;
    auto* b = new (std::nothrow) nslct_batch_s;
    if (!b) return fail(NSLCT_E_ARG, "out of host memory");
    b->count = count;
    b->precision = plans[0] ? plans[0]->d.precision : NSLCT_C64;
    b->plans.reset(new (std::nothrow) nslct_plan_s[count]);
    if (!b->plans) {
        delete b;
        return fail(NSLCT_E_ARG, "out of host memory");
    }
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
            return fail(NSLCT_E_SIZE, "batched sides must be 64, 128, 192, 256, 384, 512, 768, 1024 or a length up to 2048 without a native plan");
        }
        if (d.st.type == 7) {
            delete b;
            return fail(NSLCT_E_UNSUPPORTED, "batches run five-slot chains (not the IDFT route, type 7)");
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
    const bool dbl = b->precision == NSLCT_C128;
    for (int col = 0; col < 2; ++col) {
        std::vector<int> sizes;
        for (int i = 0; i < count; ++i) {
            const int N = col ? b->plans[i].d.Nx : b->plans[i].d.Ny;
            if (std::find(sizes.begin(), sizes.end(), N) == sizes.end()) sizes.push_back(N);
        }
        std::sort(sizes.begin(), sizes.end(), std::greater<int>());
        for (int N : sizes) {
            nslct_batch_s::Group g{};
            g.N = N;
            g.grid = 8;
            if (!batch_native_size(N)) {  // Bluestein group: its table on this device
                g.M = bluestein_length(N);
                rc = bs_tables(N, g.M, dbl, &g.bs_tab);
                if (rc) {
                    delete b;
                    return rc;
                }
            } else {
                g.width = default_width(col == 1, dbl);
            }
            b->groups[col].push_back(g);
            e = set_group_width(*b, col, b->groups[col].back(), b->groups[col].back().width, 0);
            if (e != hipSuccess) return batch_fail(b, e, "work list upload");
        }
    }
    {  // Pair row and column groups that hold the same images (chain_col).
        auto index_of = [&](int col, int N) {
            for (size_t k = 0; k < b->groups[col].size(); ++k)
                if (b->groups[col][k].N == N) return (int)k;
            return -1;
        };
        std::vector<int> pc(b->groups[0].size(), -1), pr(b->groups[1].size(), -1);
        bool paired = b->groups[0].size() == b->groups[1].size();
        for (int i = 0; i < count && paired; ++i) {
            const int r = index_of(0, b->plans[i].d.Ny), c = index_of(1, b->plans[i].d.Nx);
            if ((pc[r] >= 0 && pc[r] != c) || (pr[c] >= 0 && pr[c] != r)) paired = false;
            pc[r] = c;
            pr[c] = r;
        }
        if (paired) b->chain_col = pc;
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

    // Schedule of every group (pass axis, line length): tile width and grid,
    // from the schedule cache, else measured here on scratch images.
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) cus = 256;
    b->cus = cus;
    b->mult = -1;
    const int mults[] = {0, 1, 2, 4, 8};  // 0: one workgroup per item
    const std::string path = cache_path();
    const std::string arch = device_arch(b->device);
    auto key_of = [&](int col, const nslct_batch_s::Group& g) {
        long long lines = 0;  // lines of this group over the batch (independent of the width)
        for (int i = 0; i < count; ++i) {
            const PlanData& d = b->plans[i].d;
            if ((col ? d.Nx : d.Ny) == g.N) lines += col ? d.Ny : d.Nx;
        }
        return CacheKey{arch, b->precision, col, g.N, bucket_of((int)std::min<long long>(lines, 1 << 30))};
    };
    bool all_cached = true;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        for (int col = 0; col < 2; ++col)
            for (auto& g : b->groups[col]) {
                int v = 0, w = 0, m = 0;
                const bool hit = cache_lookup(path, key_of(col, g), &v, &w, &m) &&
                                 candidate_ok(g, w, v, col == 1, dbl) &&
                                 std::find(std::begin(mults), std::end(mults), m) != std::end(mults);
                if (hit) {
                    if (w != g.width || v != g.plan) e = set_group_width(*b, col, g, w, v);
                    if (e != hipSuccess) return batch_fail(b, e, "work list upload");
                    g.mult = m;
                    g.grid = grid_for(m, cus, g.nitems);
                    g.cached = 1;
                } else {
                    all_cached = false;
                }
            }
    }
    if (!all_cached) {
        const size_t bytes = b->total * (dbl ? 16 : 8);
        void* scratch = nullptr;
        e = hipMalloc(&scratch, bytes);
        if (e != hipSuccess) return batch_fail(b, e, "hipMalloc (autotune scratch)");
        e = hipMemsetAsync(scratch, 0, bytes, b->cap);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        for (int col = 0; col < 2 && e == hipSuccess; ++col)
            for (auto& g : b->groups[col]) {
                if (g.cached || e != hipSuccess) continue;
                // The heavier pass of the axis (two line DFTs around a chirp).
                const int pass = col ? 1 : 2;
                double best = 1e30;
                int bv = g.plan, bw = g.width, bm = 0;
                for (int v = 0; v < kPlans && e == hipSuccess; ++v)
                for (int w = 0; w <= kMaxWidth && e == hipSuccess; ++w) {
                    if (!candidate_ok(g, w, v, col == 1, dbl)) continue;
                    e = set_group_width(*b, col, g, w, v);
                    for (int m : mults) {
                        if (e != hipSuccess) break;
                        g.grid = grid_for(m, cus, g.nitems);
                        auto launch = [&]() {
                            return dbl ? launch_group_pass<double>(*b, col, g, 0, pass, scratch, scratch, b->cap)
                                       : launch_group_pass<float>(*b, col, g, 0, pass, scratch, scratch, b->cap);
                        };
                        e = launch();  // warm-up
                        if (e == hipSuccess) e = hipEventRecord(e0, b->cap);
                        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
                        if (e == hipSuccess) e = hipEventRecord(e1, b->cap);
                        if (e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0;
                        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        if (e == hipSuccess && ms / 3 * 1e3 < best) {
                            best = ms / 3 * 1e3;
                            bv = v;
                            bw = w;
                            bm = m;
                        }
                    }
                }
                if (e != hipSuccess) break;
                if (bw != g.width || bv != g.plan) e = set_group_width(*b, col, g, bw, bv);
                g.mult = bm;
                g.grid = grid_for(bm, cus, g.nitems);
                g.us = best;
                std::lock_guard<std::mutex> lk(g_cache_mu);
                cache_store(path, key_of(col, g), bv, bw, bm, best);
            }
        // The whole batch with the chosen schedule.
        if (e == hipSuccess) e = run_batched(*b, 0, scratch, scratch, b->cap);
        if (e == hipSuccess) e = hipEventRecord(e0, b->cap);
        for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run_batched(*b, 0, scratch, scratch, b->cap);
        if (e == hipSuccess) e = hipEventRecord(e1, b->cap);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        b->tuned_us = ms / 3 * 1e3;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(scratch);
        if (e != hipSuccess) return batch_fail(b, e, "autotune");
    }
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

int nslct_batch_group(nslct_batch_t batch, int col, int N, int* plan, int* lines, int* mult, int* cached) {
    if (!batch) return fail(NSLCT_E_ARG, "null batch");
    if (col != 0 && col != 1) return fail(NSLCT_E_ARG, "col must be 0 (rows) or 1 (columns)");
    std::lock_guard<std::mutex> lk(batch->mu);
    for (const auto& g : batch->groups[col])
        if (g.N == N) {
            if (plan) *plan = g.plan;
            if (lines) *lines = group_lines(g, col == 1, batch->precision == NSLCT_C128);
            if (mult) *mult = g.mult;
            if (cached) *cached = g.cached;
            return NSLCT_OK;
        }
    return fail(NSLCT_E_ARG, "no group of that axis and line length in the batch");
}

int nslct_batch_set_group(nslct_batch_t batch, int col, int N, int plan, int lines, int mult) {
    if (!batch) return fail(NSLCT_E_ARG, "null batch");
    if (col != 0 && col != 1) return fail(NSLCT_E_ARG, "col must be 0 (rows) or 1 (columns)");
    if (plan < 0 || plan >= kPlans) return fail(NSLCT_E_ARG, "plan must be 0 or 1");
    if (mult != 0 && mult != 1 && mult != 2 && mult != 4 && mult != 8)
        return fail(NSLCT_E_ARG, "mult must be 0, 1, 2, 4 or 8");
    std::lock_guard<std::mutex> lk(batch->mu);
    for (auto& g : batch->groups[col]) {
        if (g.N != N) continue;
        const bool dbl = batch->precision == NSLCT_C128;
        int w = -1;
        for (int k = 0; k <= kMaxWidth; ++k)
            if (candidate_ok(g, k, plan, col == 1, dbl) &&
                (g.M ? host_bs_lines(g.M, col == 1, dbl) : host_width_lines(N, k, plan)) == lines)
                w = k;
        if (w < 0) return fail(NSLCT_E_ARG, "not a (line plan, tile width) of this group");
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess && dev != batch->device) e = hipSetDevice(batch->device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess && (w != g.width || plan != g.plan)) e = set_group_width(*batch, col, g, w, plan);
        if (dev >= 0 && dev != batch->device) (void)hipSetDevice(dev);
        if (e != hipSuccess) return fail(NSLCT_E_HIP, std::string("set group: ") + hipGetErrorString(e));
        g.mult = mult;
        g.grid = grid_for(mult, batch->cus, g.nitems);
        for (auto& gr : batch->graphs) (void)hipGraphExecDestroy(gr.exec);
        batch->graphs.clear();
        return NSLCT_OK;
    }
    return fail(NSLCT_E_ARG, "no group of that axis and line length in the batch");
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
            rc = run_chain(&batch->plans[i], direction, 1, pi, po, stream, true);
            if (rc) return rc;
        }
        return NSLCT_OK;
    }
    if (mode == 1) {
        // The batch's fork streams and events are shared: one call at a time.
        std::lock_guard<std::mutex> lk(batch->mu);
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

}  // extern "C"
