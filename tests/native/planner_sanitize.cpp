// Host driver for the sanitizer test of the planner (tests/test_planner_sanitizers.py):
// reads 4x4 matrices (16 numbers per line) and runs every host entry of
// the planner on each: planning under every type option, the stage round
// trip, Lie plans with their theta-Jacobian and gradient contraction, the
// box check.  Built with AddressSanitizer and UndefinedBehaviorSanitizer;
// any report aborts the process.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "planner.hpp"

using namespace nslct;

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    std::vector<std::vector<double>> mats;
    for (;;) {
        std::vector<double> m(16);
        int got = 0;
        for (double& v : m) got += std::fscanf(f, "%lf", &v) == 1;
        if (got != 16) break;
        mats.push_back(m);
    }
    std::fclose(f);
    const double two_pi = 6.283185307179586;
    const int shapes[3][2] = {{16, 16}, {30, 45}, {64, 48}};
    int planned = 0, refused = 0, lie = 0, jac = 0;
    for (size_t i = 0; i < mats.size(); ++i) {
        const double* M = mats[i].data();
        const int Nx = shapes[i % 3][0], Ny = shapes[i % 3][1];
        // Spacing of the IDFT route on every third shape, free elsewhere.
        const double dx = i % 3 == 2 ? std::sqrt(two_pi / Nx) : 0.45, dy = i % 3 == 2 ? std::sqrt(two_pi / Ny) : 0.6;
        for (int t = 0; t <= 7; ++t) {
            nslct_opts o{NSLCT_C64, t, 1e-8, 1e-6};
            PlanData p;
            std::string err;
            if (build_plan(M, Nx, Ny, dx, dy, o, &p, &err) != NSLCT_OK) {
                ++refused;
                continue;
            }
            ++planned;
            PlanData q;
            if (build_plan_from_stages(p.st, Nx, Ny, o, &q, &err) != NSLCT_OK && p.st.type != 0) return 3;
            (void)box_check(p, 0.5);
        }
        double theta[10];
        for (int k = 0; k < 10; ++k) theta[k] = 0.01 * std::sin(1.7 * (double)(i * 10 + k));
        nslct_opts o{NSLCT_C64, 0, 1e-8, 1e-6};
        PlanData p;
        std::string err;
        if (build_plan_lie(M, theta, Nx, Ny, dx, dy, o, &p, &err) != NSLCT_OK) continue;
        ++lie;
        double J[120];
        if (plan_theta_jacobian(p, J, &err) != NSLCT_OK) continue;
        ++jac;
        double sums[15], g[12], out[10];
        for (int k = 0; k < 15; ++k) sums[k] = std::cos((double)k + (double)i);
        stage_gradient(p, sums, g);
        theta_gradient(J, g, out);
        for (double v : out)
            if (!std::isfinite(v)) return 4;
    }
    std::printf("matrices %zu planned %d refused %d lie %d jacobian %d\n", mats.size(), planned, refused, lie, jac);
    return 0;
}
