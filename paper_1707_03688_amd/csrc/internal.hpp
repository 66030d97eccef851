// Host-side declarations shared by the library's translation units (not part
// of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "nslct.h"
#include "planner.hpp"

struct nslct_plan_s {
    nslct::PlanData d;
    // d(stage entries)/d(theta), computed on the first backward call that
    // needs it (the plan stays logically immutable).
    std::mutex jac_mu;
    bool jac_done = false;
    int jac_rc = 0;
    std::string jac_err;
    double jac[12 * 10] = {};
};

namespace nslct {

// Records `msg` as this thread's last error and returns `code`.
int fail(int code, const std::string& msg);

// One-time per-device setup of every translation unit's device tables.
int ensure_device_ready();

// NSLCT_E_ARG unless both image pointers are non-null and 16-byte aligned.
int check_ptrs(const void* in, const void* out);

// The passes of one plan (forward dir 0, inverse dir 1) on `count` images.
// The entry points require 16-byte aligned images; element_aligned accepts
// any sample-aligned pointer (the images of a packed batch).
int run_chain(nslct_plan_t plan, int dir, int count, const void* in, void* out, void* stream,
              bool element_aligned = false);

// Per translation unit: fill its device tables on the current device.
hipError_t init_tables_batched();
hipError_t init_tables_split();
hipError_t init_tables_backward();

// Line lengths with a native mixed-radix plan (2^k up to 4096, 3 * 2^k up
// to 768); the Bluestein line length of the others (smallest power of two
// >= 2n - 1); the device table FFT_M(b) / M of both signs for (N, M,
// precision) on the current device, made on first use and kept.
bool native_line(int n);
int bluestein_length(int n);
int bs_tables(int N, int M, bool dbl, const void** out);

// Pass `pass` (0..4) of a split-precision plan.
hipError_t launch_split_pass(const PlanData& d, int dir, int pass, int count, const void* in, void* out,
                             hipStream_t s);

}  // namespace nslct
