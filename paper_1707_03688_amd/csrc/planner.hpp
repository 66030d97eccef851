// Host-side planning of the 2D HA-NsDLCT (FP64): validation of the ABCD
// matrix, decomposition type, HA gauge search and the stage coefficients the
// device passes consume.  No HIP calls: planning runs without a GPU.
#pragma once

#include <cstdint>
#include <string>

#include "nslct.h"

namespace nslct {

// Quadratic phase phi(a, b) = c11*a^2 + c12*a*b + c22*b^2 in fixed-point
// turns: 2^64 units = one turn, so integer wrap-around is the reduction
// modulo 2*pi and a product with exact integer sample indices is exact.
struct ChirpTurns {
    uint64_t c11, c12, c22;
    uint64_t c00;  // constant phase (turns), added once per line
    int nonzero;
};

// One of the chain's five "slots" in application order:
//   CM(S0) -> F -> CM_w(C1) -> F^-1 -> CM(S2) -> F -> CM_w(C3) -> F^-1 -> CM(S4)
// S slots act on the space grid (dx, dy), C slots on the frequency grid.
struct Chain5 {
    double slot[5][3];
    ChirpTurns turns[5];
};

// One pass of a reduced schedule: a line pass over rows (y lines) or
// columns (x lines) doing [pre] DFT [mid] [DFT] [post] [DFT] in registers.
struct ProgPass {
    int col;            // 0: rows (y lines, contiguous), 1: columns (x lines)
    int load_remap;     // centred -> FFT order along the line at load
    int store_remap;    // FFT -> centred order along the line at store
    int line_centered;  // the line index is stored in centred order
    int ndft;           // 1..3 line DFTs
    int sign[3];        // exponent signs of the DFTs
    int pre_on, mid_on, post_on;  // pointwise products (chirp and/or scale)
    double scale_mid, scale_post;
    ChirpTurns pre, mid, post;
};

// Reduced schedule of the CM-CC-CM and LC chains: three passes.
struct Program {
    int npass;  // 0: the five-pass chain of Chain5 is used
    ProgPass p[5];
};

struct PlanData {
    nslct_stages st;
    int Nx, Ny;
    int precision;
    Chain5 dir[2];     // [0] forward, [1] inverse (adjoint): five-slot form
    Program prog[2];   // reduced three-pass schedule of the same chain
    // The planned matrix as M = M0 expm(J S(theta)) (theta = 0 for a plan of
    // M itself) and the options it was planned with, for the derivative of
    // the stage matrices along theta; has_lie = 0 for plans made from stages.
    int has_lie;
    double abcd0[16];
    double theta[10];
    nslct_opts opts;
};

// Symmetric 2x2 (x11, x12, x22) helpers exposed for tests of the planner.
double gamma_ratio(const double x[3]);

// Builds a plan; returns an NSLCT_* code and fills `err` on failure.
int build_plan(const double abcd[16], int Nx, int Ny, double dx, double dy, const nslct_opts& o,
               PlanData* out, std::string* err);
int build_plan_from_stages(const nslct_stages& st, int Nx, int Ny, const nslct_opts& o,
                           PlanData* out, std::string* err);
// Plans M = M0 expm(J S(theta)) and records (M0, theta).
int build_plan_lie(const double abcd0[16], const double theta[10], int Nx, int Ny, double dx, double dy,
                   const nslct_opts& o, PlanData* out, std::string* err);
// M expm(J S(theta)) (10 Lie coordinates theta).
void lie_point(const double abcd[16], const double theta[10], double* M);
// d(stage entries)/d(theta) at theta0 for M(theta) = M expm(J S(theta)),
// central differences of the planner with step h.
int plan_jacobian(const double abcd[16], const double theta0[10], int Nx, int Ny, double dx, double dy,
                  const nslct_opts& o, double h, double jac[12 * 10], std::string* err);
// d(stage entries)/d(theta) of a plan at its own (M0, theta), with the
// difference step of its decomposition type.
int plan_theta_jacobian(const PlanData& p, double jac[12 * 10], std::string* err);
// Raw backward sums (15) -> d loss / d(stage entries) (12, order of st.mats).
void stage_gradient(const PlanData& p, const double sums[15], double g[12]);
// d loss / d theta = jac^T (d loss / d stages).
void theta_gradient(const double jac[12 * 10], const double gst[12], double out[10]);
// Phase-space box check (eqs. HA12-HA20) with the input in fraction `frac`.
bool box_check(const PlanData& p, double frac);

}  // namespace nslct
