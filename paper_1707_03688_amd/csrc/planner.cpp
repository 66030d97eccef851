// Host planner of the 2D HA-NsDLCT (FP64).
//
// Steps (Pei & Huang, CM-CC-CM-CC NsDLCT):
//   1. M J M^T = J within tolerance (Sec. 1, eq. Intro12).
//   2. B = 0: a pure chirp multiplication when A = D = I (eq. BasicCM12);
//      otherwise an affine map (eq. Intro20), which is rejected.
//   3. Type from the sign of tr B (Sec. 4.4, eq. Reversible08), tr B = 0 read
//      as type 1; a type whose gauge equation has no solution falls back to
//      the other type.
//   4. Gauge: minimise the product of the growth ratios gamma (eq. HA16) of
//      the four stage matrices (eq. HA24) over symmetric H with B' = B - A H
//      symmetric (type 1, eq. Bnonsym32) or B1' = B - H1 D symmetric (type 2,
//      eq. CCCMCCCM08), |det B'| >= det_min max(1, max|B_ij|^2) (det_min
//      an option, default 1e-6).  The feasible
//      set is a plane (or all of Sym(2)); the objective is piecewise smooth
//      with minima on |.| kinks, so the search is exhaustive on a grid, then
//      Nelder-Mead, then Newton "snapping" onto the kinks.  Ties within
//      relative 1e-9 go to the smallest ||H||_F, then lexicographic order.
//   5. Stage matrices (type 1: P1 = (D'-I)B'^-1, B', P3 = B'^-1(A-I), H,
//      eq. Bnonsym12; type 2: H1, Q1 = (D-I)B1'^-1, B1', Q3 = B1'^-1(A1'-I),
//      eq. CCCMCCCM16), symmetrised, then the five-slot chain and its adjoint
//      (eq. CCCMCCCM30) with phase coefficients in fixed-point turns.
// Reduced decompositions:
//   * CM-CC-CM when B is symmetric and invertible (Sec. 4.1, eqs. Bsym04-12):
//     P1 = (D - I) B^-1, B, P3 = B^-1 (A - I).  Chosen without an override
//     when B = B^T and |det B| >= the det_min bound (the case split of
//     Secs. 4.1 / 4.2), or on request (type_override 3).
//   * LC-NsDLCT (Sec. 4.2.2, eqs. LC04-LC12), on request (type_override 4..6):
//     the type-1 form with the rank-one gauge H = (h, 0; 0, 0),
//     h = (b21 - b12) / a21 (eq. LC08), or H = (0, 0; 0, h),
//     h = (b12 - b21) / a12 (eq. LC10); with both available, the smaller
//     eq. HA24 objective (6); with neither giving an invertible B', option 6
//     falls back to the HA-NsDLCT as the paper prescribes.
//   Both are five-slot chains with zero slots, run as three passes.
#include "planner.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

namespace nslct {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct M2 {
    double a11, a12, a21, a22;
};

M2 mul(const M2& x, const M2& y) {
    return {x.a11 * y.a11 + x.a12 * y.a21, x.a11 * y.a12 + x.a12 * y.a22,
            x.a21 * y.a11 + x.a22 * y.a21, x.a21 * y.a12 + x.a22 * y.a22};
}
M2 sub(const M2& x, const M2& y) { return {x.a11 - y.a11, x.a12 - y.a12, x.a21 - y.a21, x.a22 - y.a22}; }
M2 minus_eye(const M2& x) { return {x.a11 - 1.0, x.a12, x.a21, x.a22 - 1.0}; }
double det(const M2& x) { return x.a11 * x.a22 - x.a12 * x.a21; }

struct Blocks {
    M2 A, B, C, D;
};

Blocks split(const double m[16]) {
    auto at = [&](int r, int c) { return m[4 * r + c]; };
    return {{at(0, 0), at(0, 1), at(1, 0), at(1, 1)},
            {at(0, 2), at(0, 3), at(1, 2), at(1, 3)},
            {at(2, 0), at(2, 1), at(3, 0), at(3, 1)},
            {at(2, 2), at(2, 3), at(3, 2), at(3, 3)}};
}

double symplectic_residual(const double m[16]) {
    // max |M J M^T - J| with J = (0, I; -I, 0).
    double J[16] = {0, 0, 1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, -1, 0, 0};
    double MJ[16], R = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0;
            for (int k = 0; k < 4; ++k) s += m[4 * i + k] * J[4 * k + j];
            MJ[4 * i + j] = s;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0;
            for (int k = 0; k < 4; ++k) s += MJ[4 * i + k] * m[4 * j + k];
            R = std::max(R, std::fabs(s - J[4 * i + j]));
        }
    return R;
}

void sym3(const M2& x, double out[3]) {
    out[0] = x.a11;
    out[1] = 0.5 * (x.a12 + x.a21);
    out[2] = x.a22;
}

// The decomposition of one matrix for one type, evaluated at gauge h.
struct Gauge {
    Blocks b;
    int type;
    double dmin;

    // Stage matrices in formula order (leftmost first), symmetrised.
    bool stages(const double h[3], double out[4][3], double* dt) const {
        const M2 H{h[0], h[1], h[1], h[2]};
        M2 Bp, X1, X3;
        if (type == 1) {
            Bp = sub(b.B, mul(b.A, H));
            const M2 Dp = sub(b.D, mul(b.C, H));
            *dt = det(Bp);
            if (!(std::fabs(*dt) >= dmin)) return false;
            const double r = 1.0 / *dt;
            const M2 Bi{Bp.a22 * r, -Bp.a12 * r, -Bp.a21 * r, Bp.a11 * r};
            X1 = mul(minus_eye(Dp), Bi);   // P1 = (D' - I) B'^-1
            X3 = mul(Bi, minus_eye(b.A));  // P3 = B'^-1 (A - I)
            sym3(X1, out[0]);
            sym3(Bp, out[1]);
            sym3(X3, out[2]);
            sym3(H, out[3]);
        } else {
            Bp = sub(b.B, mul(H, b.D));
            const M2 Ap = sub(b.A, mul(H, b.C));
            *dt = det(Bp);
            if (!(std::fabs(*dt) >= dmin)) return false;
            const double r = 1.0 / *dt;
            const M2 Bi{Bp.a22 * r, -Bp.a12 * r, -Bp.a21 * r, Bp.a11 * r};
            X1 = mul(minus_eye(b.D), Bi);  // Q1 = (D - I) B1'^-1
            X3 = mul(Bi, minus_eye(Ap));   // Q3 = B1'^-1 (A1' - I)
            sym3(H, out[0]);
            sym3(X1, out[1]);
            sym3(Bp, out[2]);
            sym3(X3, out[3]);
        }
        return true;
    }

    double objective(const double h[3]) const {
        double st[4][3], dt;
        if (!stages(h, st, &dt)) return INFINITY;
        double f = 1.0;
        for (auto& x : st) f *= gamma_ratio(x);
        return f;
    }

    // The feasibility equation c . h = rhs.
    void equation(double c[3], double* rhs) const {
        *rhs = b.B.a12 - b.B.a21;
        if (type == 1) {
            c[0] = -b.A.a21;
            c[1] = b.A.a11 - b.A.a22;
            c[2] = b.A.a12;
        } else {
            c[0] = b.D.a12;
            c[1] = b.D.a22 - b.D.a11;
            c[2] = -b.D.a21;
        }
    }
};

struct Cand {
    double f;
    double h[3];
};

bool better_tie(const Cand& x, const Cand& y) {
    auto key = [](const Cand& c) {
        std::array<double, 4> k{c.h[0] * c.h[0] + 2 * c.h[1] * c.h[1] + c.h[2] * c.h[2], c.h[0], c.h[1],
                                c.h[2]};
        for (auto& v : k) v = std::round(v * 1e12) / 1e12;
        return k;
    };
    return key(x) < key(y);
}

struct GaugeOut {
    bool feasible = false;
    bool found = false;
    double h[3] = {0, 0, 0};
    double f = INFINITY;
};

// Nelder-Mead minimisation in dim (2 or 3) coordinates from s with an
// axis-aligned initial simplex of size `size`; s is overwritten by the best
// vertex, whose value is returned.
template <class Fn>
double nelder_mead(Fn& f, double* s, int dim, double size) {
    const int n = dim;
    double X[4][3], F[4];
    for (int i = 0; i <= n; ++i) {
        for (int k = 0; k < 3; ++k) X[i][k] = s[k];
        if (i > 0) X[i][i - 1] += size;
        F[i] = f(X[i]);
    }
    for (int it = 0; it < 20000; ++it) {
        // Order vertices by value.
        for (int i = 1; i <= n; ++i)
            for (int j = i; j > 0 && F[j] < F[j - 1]; --j) {
                std::swap(F[j], F[j - 1]);
                for (int k = 0; k < 3; ++k) std::swap(X[j][k], X[j - 1][k]);
            }
        double xspan = 0;
        for (int i = 1; i <= n; ++i)
            for (int k = 0; k < n; ++k) xspan = std::max(xspan, std::fabs(X[i][k] - X[0][k]));
        if (xspan <= 1e-12 * (1.0 + std::fabs(X[0][0]) + std::fabs(X[0][1])) ||
            (std::isfinite(F[n]) && F[n] - F[0] <= 1e-14 * F[0] && xspan <= 1e-9))
            break;
        double c[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) c[k] += X[i][k] / n;
        auto along = [&](double t, double* out) {
            for (int k = 0; k < 3; ++k) out[k] = k < n ? c[k] + t * (X[n][k] - c[k]) : X[0][k];
        };
        double xr[3], xe[3], xc[3];
        along(-1.0, xr);
        const double fr = f(xr);
        if (fr < F[0]) {
            along(-2.0, xe);
            const double fe = f(xe);
            if (fe < fr) {
                std::memcpy(X[n], xe, sizeof xe);
                F[n] = fe;
            } else {
                std::memcpy(X[n], xr, sizeof xr);
                F[n] = fr;
            }
        } else if (fr < F[n - 1]) {
            std::memcpy(X[n], xr, sizeof xr);
            F[n] = fr;
        } else {
            const bool outside = fr < F[n];
            along(outside ? -0.5 : 0.5, xc);
            const double fc = f(xc);
            if (fc < (outside ? fr : F[n])) {
                std::memcpy(X[n], xc, sizeof xc);
                F[n] = fc;
            } else {
                for (int i = 1; i <= n; ++i) {
                    for (int k = 0; k < n; ++k) X[i][k] = X[0][k] + 0.5 * (X[i][k] - X[0][k]);
                    F[i] = f(X[i]);
                }
            }
        }
    }
    int b = 0;
    for (int i = 1; i <= n; ++i)
        if (F[i] < F[b]) b = i;
    for (int k = 0; k < 3; ++k) s[k] = X[b][k];
    return F[b];
}

// Exhaustive HA gauge search (eq. HA24).
// Gauge search of eq. HA24.  With `start` == nullptr: exhaustive grid over
// the feasible set, then Nelder-Mead from the best distinct cells.  With a
// start gauge (a neighbouring optimum, used by the Jacobian's difference
// quotients): Nelder-Mead from its projection onto this feasible set only.
// Kink snapping follows in both cases.
GaugeOut solve(const Gauge& g, double mmax, const double* start = nullptr) {
    GaugeOut out;
    double c[3], rhs;
    g.equation(c, &rhs);
    const double scale = std::max(1.0, mmax);
    const double cn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    double h0[3] = {0, 0, 0};
    double U[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};  // columns span the feasible set
    int dim;
    if (cn <= 1e-12 * scale) {
        if (std::fabs(rhs) > 1e-12 * scale) return out;  // 0 = rhs != 0: empty
        dim = 3;
    } else {
        dim = 2;
        const double u[3] = {c[0] / cn, c[1] / cn, c[2] / cn};
        for (int i = 0; i < 3; ++i) h0[i] = u[i] * rhs / cn;
        // Gram-Schmidt: start from the axis least aligned with c.
        int ax = 0;
        for (int i = 1; i < 3; ++i)
            if (std::fabs(u[i]) < std::fabs(u[ax])) ax = i;
        double e[3] = {0, 0, 0};
        e[ax] = 1;
        double d = u[ax];
        double v1[3] = {e[0] - d * u[0], e[1] - d * u[1], e[2] - d * u[2]};
        double n1 = std::sqrt(v1[0] * v1[0] + v1[1] * v1[1] + v1[2] * v1[2]);
        for (auto& x : v1) x /= n1;
        double v2[3] = {u[1] * v1[2] - u[2] * v1[1], u[2] * v1[0] - u[0] * v1[2], u[0] * v1[1] - u[1] * v1[0]};
        for (int i = 0; i < 3; ++i) {
            U[i][0] = v1[i];
            U[i][1] = v2[i];
            U[i][2] = 0;
        }
    }
    out.feasible = true;
    auto to_h = [&](const double* s, double* h) {
        for (int i = 0; i < 3; ++i) {
            h[i] = h0[i];
            for (int k = 0; k < dim; ++k) h[i] += U[i][k] * s[k];
        }
    };
    auto fs = [&](const double* s) {
        double h[3];
        to_h(s, h);
        return g.objective(h);
    };

    const double R = 4.0 * (1.0 + mmax);
    const int G = dim == 2 ? 513 : 81;
    double step = 2.0 * R / (G - 1);
    std::vector<std::array<double, 3>> starts;
    if (start) {
        // Coordinates of the start gauge's projection onto the feasible set.
        std::array<double, 3> s0{0, 0, 0};
        for (int k = 0; k < dim; ++k)
            for (int i = 0; i < 3; ++i) s0[k] += U[i][k] * (start[i] - h0[i]);
        starts.push_back(s0);
        step = 1e-3 * (1.0 + std::fabs(s0[0]) + std::fabs(s0[1]) + std::fabs(s0[2]));
    }
    // Grid evaluation.
    using Cell = std::pair<double, std::array<int, 3>>;
    // Cells ordered by objective, ties by cell index: a strict total order,
    // so the selections below do not depend on how the grid was split.
    auto less = [](const Cell& x, const Cell& y) {
        return x.first < y.first || (x.first == y.first && x.second < y.second);
    };
    constexpr size_t kHead = 4096;
    std::vector<std::vector<Cell>> part;
    std::vector<Cell> cells;  // the best cells, in order
    if (!start) {
        // The grid's rows are swept by up to 16 host threads, each into a
        // vector of its own (moved into `part` at the end, so no two threads
        // write to neighbouring memory), which it also partially orders: its
        // best kHead cells first.  The best kHead cells of the grid are among
        // the union of those heads.
        const int G3 = dim == 3 ? G : 1;
        const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        part.resize(nth);
        auto rows = [&](int t) {
            std::vector<Cell> local;
            local.reserve((size_t)(G / nth + 1) * G * G3);
            double s[3] = {0, 0, 0};
            for (int i = t; i < G; i += nth)
                for (int j = 0; j < G; ++j)
                    for (int k = 0; k < G3; ++k) {
                        s[0] = -R + step * i;
                        s[1] = -R + step * j;
                        s[2] = -R + step * k;
                        const double f = fs(s);
                        if (std::isfinite(f)) local.push_back({f, {i, j, k}});
                    }
            if (local.size() > kHead) std::nth_element(local.begin(), local.begin() + (kHead - 1), local.end(), less);
            part[t] = std::move(local);
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nth; ++t) pool.emplace_back(rows, t);
        rows(0);
        for (auto& th : pool) th.join();
        for (const auto& pv : part) cells.insert(cells.end(), pv.begin(), pv.begin() + std::min(pv.size(), kHead));
    }
    if (!start) {
        if (cells.empty()) return out;
        // Seeds: the best cells in increasing objective, each more than three
        // cells away from the seeds already taken, at most 16.  Only the head
        // of the order is needed: the best kHead cells are sorted, and the
        // whole grid is sorted only if they hold fewer than 16 seeds (same
        // seeds either way).
        auto pick = [&](size_t n, std::vector<std::array<int, 3>>& seeds) {
            seeds.clear();
            for (size_t c = 0; c < n; ++c) {
                const auto& cell = cells[c];
                bool far = true;
                for (const auto& sd : seeds) {
                    int dmax = 0;
                    for (int k = 0; k < dim; ++k) dmax = std::max(dmax, std::abs(cell.second[k] - sd[k]));
                    if (dmax <= 3) far = false;
                }
                if (far) seeds.push_back(cell.second);
                if (seeds.size() >= 16) return true;
            }
            return false;
        };
        size_t total = 0;
        for (const auto& pv : part) total += pv.size();
        std::vector<std::array<int, 3>> seeds;
        const size_t head = std::min(cells.size(), kHead);
        std::nth_element(cells.begin(), cells.begin() + (head - 1), cells.end(), less);
        std::sort(cells.begin(), cells.begin() + head, less);
        if (!pick(head, seeds) && head < total) {
            cells.clear();
            cells.reserve(total);
            for (const auto& pv : part) cells.insert(cells.end(), pv.begin(), pv.end());
            std::sort(cells.begin(), cells.end(), less);
            pick(cells.size(), seeds);
        }
        for (const auto& sd : seeds) starts.push_back({-R + step * sd[0], -R + step * sd[1], -R + step * sd[2]});
    }

    std::vector<Cand> cands;
    for (const auto& st0 : starts) {
        double s[3] = {st0[0], st0[1], st0[2]};
        if (dim == 2) s[2] = 0;
        double f = nelder_mead(fs, s, dim, step);
        // Restart from the result with a fresh simplex: Nelder-Mead can
        // collapse early next to a kink.
        for (int rs = 0; rs < 3; ++rs) f = nelder_mead(fs, s, dim, step * std::pow(0.1, rs + 1));
        Cand cd;
        cd.f = f;
        to_h(s, cd.h);
        cands.push_back(cd);

        // Kink snapping: Newton on subsets of the near-zero stage entries.
        double stg[4][3], dt;
        if (!g.stages(cd.h, stg, &dt)) continue;
        double emax = 0;
        for (auto& x : stg)
            for (double v : x) emax = std::max(emax, std::fabs(v));
        std::vector<int> near;
        for (int i = 0; i < 12; ++i)
            if (std::fabs(stg[i / 3][i % 3]) < 1e-4 * (1 + emax)) near.push_back(i);
        if (near.size() > 8) near.resize(8);
        const int nn = (int)near.size();
        auto entries = [&](const double* x, const int* idx, double* e) {
            double h[3], st2[4][3], dd;
            to_h(x, h);
            if (!g.stages(h, st2, &dd)) return false;
            for (int k = 0; k < dim; ++k) e[k] = st2[idx[k] / 3][idx[k] % 3];
            return true;
        };
        std::vector<int> comb(dim);
        std::function<void(int, int)> rec;
        auto newton = [&](const int* idx) {
            double x[3] = {s[0], s[1], s[2]};
            double e[3];
            if (!entries(x, idx, e)) return;
            for (int it = 0; it < 60; ++it) {
                double Jm[3][3];
                for (int k = 0; k < dim; ++k) {
                    const double hstep = 1e-7 * (1.0 + std::fabs(x[k]));
                    double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
                    xp[k] += hstep;
                    xm[k] -= hstep;
                    double ep[3], em[3];
                    if (!entries(xp, idx, ep) || !entries(xm, idx, em)) return;
                    for (int r = 0; r < dim; ++r) Jm[r][k] = (ep[r] - em[r]) / (2 * hstep);
                }
                // Solve Jm dx = -e (dim 2 or 3) by Cramer's rule.
                double dx[3] = {0, 0, 0};
                if (dim == 2) {
                    const double dj = Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0];
                    if (std::fabs(dj) < 1e-300) return;
                    dx[0] = (-e[0] * Jm[1][1] + e[1] * Jm[0][1]) / dj;
                    dx[1] = (-e[1] * Jm[0][0] + e[0] * Jm[1][0]) / dj;
                } else {
                    auto d3 = [](double a[3][3]) {
                        return a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
                               a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
                               a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
                    };
                    const double dj = d3(Jm);
                    if (std::fabs(dj) < 1e-300) return;
                    for (int k = 0; k < 3; ++k) {
                        double Mk[3][3];
                        for (int r = 0; r < 3; ++r)
                            for (int q = 0; q < 3; ++q) Mk[r][q] = (q == k) ? -e[r] : Jm[r][q];
                        dx[k] = d3(Mk) / dj;
                    }
                }
                for (int k = 0; k < dim; ++k) x[k] += dx[k];
                if (!entries(x, idx, e)) return;
                double em = 0;
                for (int k = 0; k < dim; ++k) em = std::max(em, std::fabs(e[k]));
                if (em <= 1e-13 * (1 + emax)) {
                    Cand c2;
                    to_h(x, c2.h);
                    c2.f = g.objective(c2.h);
                    if (std::isfinite(c2.f)) cands.push_back(c2);
                    return;
                }
            }
        };
        rec = [&](int start, int depth) {
            if (depth == dim) {
                newton(comb.data());
                return;
            }
            for (int i = start; i < nn; ++i) {
                comb[depth] = near[i];
                rec(i + 1, depth + 1);
            }
        };
        rec(0, 0);
    }
    double fmin = INFINITY;
    for (const auto& cd : cands) fmin = std::min(fmin, cd.f);
    if (!std::isfinite(fmin)) return out;
    const Cand* best = nullptr;
    for (const auto& cd : cands) {
        if (cd.f > fmin * (1.0 + 1e-9)) continue;
        if (!best || better_tie(cd, *best)) best = &cd;
    }
    out.found = true;
    out.f = best->f;
    std::memcpy(out.h, best->h, sizeof out.h);
    return out;
}

uint64_t turns_fixed(long double kappa) {
    // frac(kappa / 2 pi) as a 64-bit fixed-point fraction of a turn.  The
    // host's long double (64-bit significand) keeps the coefficient's own
    // rounding near 2^-64 turns: the device multiplies it by exact squared
    // sample indices (up to ~2^22), which would lift a 53-bit coefficient's
    // rounding to ~1e-10 turns at N = 2048.
    const long double two_pi = 6.283185307179586476925286766559005768L;
    const long double t = kappa / two_pi;
    long double f = t - floorl(t);
    if (!(f < 1.0L)) f = 0.0L;
    return (uint64_t)ldexpl(f, 64);
}

ChirpTurns make_turns(const double p[3], double du, double dv) {
    ChirpTurns c;
    const long double u = du, v = dv;
    c.c11 = turns_fixed(0.5L * (long double)p[0] * u * u);
    c.c12 = turns_fixed((long double)p[1] * u * v);
    c.c22 = turns_fixed(0.5L * (long double)p[2] * v * v);
    c.c00 = 0;
    c.nonzero = (p[0] != 0.0 || p[1] != 0.0 || p[2] != 0.0) ? 1 : 0;
    return c;
}

// Line lengths with a native plan: 2^k (2..4096) and 3 * 2^k (6..768).
bool native_size(int n) {
    if (n >= 2 && n <= 4096 && (n & (n - 1)) == 0) return true;
    if (n % 3 == 0 && n >= 6 && n <= 768) {
        const int m = n / 3;
        return (m & (m - 1)) == 0;
    }
    return false;
}

// Supported: native lengths, and any other length up to 2048 (Bluestein's
// chirp-z form on a power-of-two line of at least 2N - 1 samples).
bool supported_size(int n) { return native_size(n) || (n >= 2 && n <= 2048); }

ProgPass prog_pass(int col, int lr, int sr, int lcn, int ndft, int s0, int s1, int s2) {
    ProgPass q{};
    q.col = col;
    q.load_remap = lr;
    q.store_remap = sr;
    q.line_centered = lcn;
    q.ndft = ndft;
    q.sign[0] = s0;
    q.sign[1] = s1;
    q.sign[2] = s2;
    q.scale_mid = q.scale_post = 1.0;
    return q;
}

// Three-pass schedules of the reduced chains (rightmost factor first).
// CM-CC-CM, slots (S0, C1, S4):
//   rows   [CM(S0)] F_y
//   cols   F_x CM_w(C1) / Nx F_x^-1          (x centred in, centred out)
//   rows   F_y^-1 CM(S4) / Ny
// LC along y (H = (0,0;0,h)):  CM(P1) U^H CM_w(-B') U CM(P3) U_y^H CM_wy(-h) U_y
//   rows   F_y CM_wy(-h) / Ny F_y^-1 CM(P3) F_y
//   cols   F_x CM_w(-B') / Nx F_x^-1
//   rows   F_y^-1 CM(P1) / Ny
// LC along x swaps the roles of rows and columns.  The inverse (adjoint) runs
// the reversed factors with negated matrices.
void fill_program(PlanData* p) {
    const nslct_stages& s = p->st;
    p->prog[0].npass = p->prog[1].npass = 0;
    if (!native_size(p->Nx) || !native_size(p->Ny)) return;  // Bluestein axes: the five-slot chain
    const double iNx = 1.0 / p->Nx, iNy = 1.0 / p->Ny;
    auto turns = [&](const double* m, double sign, bool freq) {
        double x[3] = {sign * m[0], sign * m[1], sign * m[2]};
        return make_turns(x, freq ? s.dwx : s.dx, freq ? s.dwy : s.dy);
    };
    for (int d = 0; d < 2; ++d) {
        Program& g = p->prog[d];
        g.npass = 0;
        const double sg = d == 0 ? 1.0 : -1.0;  // the inverse negates every matrix
        if (s.type == 3) {  // mats {P1, B, P3}
            const double* first = d == 0 ? s.mats[2] : s.mats[0];
            const double* last = d == 0 ? s.mats[0] : s.mats[2];
            ProgPass a = prog_pass(0, 1, 0, 1, 1, -1, 0, 0);
            a.pre = turns(first, sg, false);
            a.pre_on = a.pre.nonzero;
            ProgPass b = prog_pass(1, 1, 1, 0, 2, -1, +1, 0);
            b.mid = turns(s.mats[1], -sg, true);
            b.mid_on = 1;
            b.scale_mid = iNx;
            ProgPass c = prog_pass(0, 0, 1, 1, 1, +1, 0, 0);
            c.mid = turns(last, sg, false);
            c.mid_on = 1;
            c.scale_mid = iNy;
            g.p[0] = a;
            g.p[1] = b;
            g.p[2] = c;
            g.npass = 3;
        } else if (s.type == 4 || s.type == 5) {  // mats {P1, B', P3, H}
            const int lc = s.type == 4 ? 1 : 0;  // LC line axis: x lines are columns
            const double iNl = lc ? iNx : iNy, iNo = lc ? iNy : iNx;
            if (d == 0) {
                ProgPass a = prog_pass(lc, 1, 0, 1, 3, -1, +1, -1);
                a.mid = turns(s.mats[3], -1.0, true);
                a.mid_on = 1;
                a.scale_mid = iNl;
                a.post = turns(s.mats[2], 1.0, false);
                a.post_on = a.post.nonzero;
                ProgPass b = prog_pass(1 - lc, 1, 1, 0, 2, -1, +1, 0);
                b.mid = turns(s.mats[1], -1.0, true);
                b.mid_on = 1;
                b.scale_mid = iNo;
                ProgPass c = prog_pass(lc, 0, 1, 1, 1, +1, 0, 0);
                c.mid = turns(s.mats[0], 1.0, false);
                c.mid_on = 1;
                c.scale_mid = iNl;
                g.p[0] = a;
                g.p[1] = b;
                g.p[2] = c;
            } else {
                ProgPass a = prog_pass(lc, 1, 0, 1, 1, -1, 0, 0);
                a.pre = turns(s.mats[0], -1.0, false);
                a.pre_on = a.pre.nonzero;
                ProgPass b = prog_pass(1 - lc, 1, 1, 0, 2, -1, +1, 0);
                b.mid = turns(s.mats[1], 1.0, true);
                b.mid_on = 1;
                b.scale_mid = iNo;
                ProgPass c = prog_pass(lc, 0, 1, 1, 3, +1, -1, +1);
                c.mid = turns(s.mats[2], -1.0, false);
                c.mid_on = 1;
                c.scale_mid = iNl;
                c.post = turns(s.mats[3], 1.0, true);
                c.post_on = 1;
                c.scale_post = iNl;
                g.p[0] = a;
                g.p[1] = b;
                g.p[2] = c;
            }
            g.npass = 3;
        } else if (s.type == 7) {  // mats {P1', A, P3'}: j^q CM(P1') U^H CM_w(-A) U CM(P3') U^H
            // Three line DFTs per axis (unnormalised): (Nx Ny)^(-3/2) in total.
            const double sx = std::pow((double)p->Nx, -1.5), sy = std::pow((double)p->Ny, -1.5);
            const uint64_t q = (uint64_t)(s.phase_q & 3);
            if (d == 0) {
                ProgPass a = prog_pass(0, 1, 0, 1, 1, +1, 0, 0);   // rows: IDFT_y
                ProgPass b = prog_pass(1, 1, 0, 0, 2, +1, -1, 0);  // cols: IDFT_x CM(P3') DFT_x
                b.mid = turns(s.mats[2], 1.0, false);
                b.mid_on = 1;
                ProgPass c = prog_pass(0, 0, 1, 0, 2, -1, +1, 0);  // rows: DFT_y CM_w(-A) IDFT_y
                c.mid = turns(s.mats[1], -1.0, true);
                c.mid_on = 1;
                c.scale_mid = sy;
                ProgPass e = prog_pass(1, 0, 1, 1, 1, +1, 0, 0);   // cols: IDFT_x CM(P1') j^q
                e.mid = turns(s.mats[0], 1.0, false);
                e.mid.c00 = q << 62;
                e.mid.nonzero = e.mid.nonzero || q != 0;
                e.mid_on = 1;
                e.scale_mid = sx;
                g.p[0] = a;
                g.p[1] = b;
                g.p[2] = c;
                g.p[3] = e;
            } else {  // adjoint: j^-q U CM(-P3') U^H CM_w(A) U CM(-P1')
                ProgPass a = prog_pass(1, 1, 0, 1, 1, -1, 0, 0);   // cols: j^-q CM(-P1') DFT_x
                a.pre = turns(s.mats[0], -1.0, false);
                a.pre.c00 = ((4 - q) & 3) << 62;
                a.pre_on = a.pre.nonzero || q != 0;
                a.pre.nonzero = a.pre_on;
                ProgPass b = prog_pass(0, 1, 0, 0, 2, -1, +1, 0);  // rows: DFT_y CM_w(A) IDFT_y
                b.mid = turns(s.mats[1], 1.0, true);
                b.mid_on = 1;
                b.scale_mid = sy;
                ProgPass c = prog_pass(1, 0, 1, 0, 2, +1, -1, 0);  // cols: IDFT_x CM(-P3') DFT_x
                c.mid = turns(s.mats[2], -1.0, false);
                c.mid_on = 1;
                c.scale_mid = sx;
                ProgPass e = prog_pass(0, 0, 1, 1, 1, -1, 0, 0);   // rows: DFT_y
                g.p[0] = a;
                g.p[1] = b;
                g.p[2] = c;
                g.p[3] = e;
            }
            g.npass = 4;
        }
    }
}

void fill_chains(PlanData* p) {
    const nslct_stages& s = p->st;
    double S[5][3] = {};
    auto put = [&](int slot, const double* x, double sign) {
        for (int k = 0; k < 3; ++k) S[slot][k] = sign * x[k];
    };
    // Generic form CM(S0) U CM_w(C1) U^H CM(S2) U CM_w(C3) U^H CM(S4), rightmost first.
    if (s.type == 1 || s.type == 4 || s.type == 5) {  // CM(P1) CC(B') CM(P3) CC(H), CC(X) = F^-1 CM(-X) F
        put(1, s.mats[3], -1.0);
        put(2, s.mats[2], 1.0);
        put(3, s.mats[1], -1.0);
        put(4, s.mats[0], 1.0);
    } else if (s.type == 2) {  // CC(H1) CM(Q1) CC(B1') CM(Q3)
        put(0, s.mats[3], 1.0);
        put(1, s.mats[2], -1.0);
        put(2, s.mats[1], 1.0);
        put(3, s.mats[0], -1.0);
    } else if (s.type == 3) {  // CM(P1) CC(B) CM(P3), overall constant +1
        put(0, s.mats[2], 1.0);
        put(1, s.mats[1], -1.0);
        put(4, s.mats[0], 1.0);
    } else if (s.type == 7) {  // no five-slot form (an IDFT is one of its factors)
    } else {  // CM(C)
        put(0, s.mats[0], 1.0);
    }
    for (int d = 0; d < 2; ++d) {
        for (int k = 0; k < 5; ++k) {
            // Adjoint: reversed order, negated matrices (eq. CCCMCCCM30).
            const double* src = d == 0 ? S[k] : S[4 - k];
            const double sg = d == 0 ? 1.0 : -1.0;
            for (int q = 0; q < 3; ++q) p->dir[d].slot[k][q] = sg * src[q];
            const bool freq = (k == 1 || k == 3);
            p->dir[d].turns[k] = make_turns(p->dir[d].slot[k], freq ? s.dwx : s.dx, freq ? s.dwy : s.dy);
        }
    }
    fill_program(p);
}

int check_common(int Nx, int Ny, double dx, double dy, const nslct_opts& o, std::string* err) {
    if (!(dx > 0) || !(dy > 0) || !std::isfinite(dx) || !std::isfinite(dy)) {
        *err = "sampling intervals must be finite and positive";
        return NSLCT_E_ARG;
    }
    if (!supported_size(Nx) || !supported_size(Ny)) {
        *err = "Nx and Ny must be in [2, 2048], or 2^k up to 4096";
        return NSLCT_E_SIZE;
    }
    if (o.precision < NSLCT_C64 || o.precision > NSLCT_C64_SPLIT_BF16) {
        *err = "unknown precision";
        return NSLCT_E_ARG;
    }
    if (o.precision >= NSLCT_C64_SPLIT_F16 && !((Nx == 256 || Nx == 4096) && (Ny == 256 || Ny == 4096))) {
        *err = "split-precision sides must be 256 or 4096";
        return NSLCT_E_SIZE;
    }
    if (o.type_override < 0 || o.type_override > 7) {
        *err = "type_override must be in 0..7";
        return NSLCT_E_ARG;
    }
    if (!(o.det_min > 0) || !std::isfinite(o.det_min)) {
        *err = "det_min must be finite and positive";
        return NSLCT_E_ARG;
    }
    return NSLCT_OK;
}

}  // namespace

double gamma_ratio(const double x[3]) {
    return (std::fabs(x[0]) + std::fabs(x[1]) + 1.0) * (std::fabs(x[1]) + std::fabs(x[2]) + 1.0);
}

namespace {

// ------------------------------------------- constant of the IDFT route
// A Gaussian exp(-1/2 z^T S z) (S complex symmetric, Re S > 0) stays a
// Gaussian under every factor of a chain; tracking its amplitude through two
// factorisations of one matrix gives the ratio of their overall constants.
//   CM(P):           S -> S - j P
//   CC(B) (unitary): S -> (S^-1 + j B)^-1, amplitude / det(I + j S B)^(1/2),
//                    the root continued from B = 0 along t B
//   unitary IDFT:    S -> S^-1, amplitude / det(S)^(1/2), the root continued
//                    from S = I along (1 - t) I + t S
using cplxd = std::complex<double>;
struct C2 {
    cplxd a, b, c, d;  // [[a, b], [c, d]]
};
C2 c2_mul(const C2& x, const C2& y) {
    return {x.a * y.a + x.b * y.c, x.a * y.b + x.b * y.d, x.c * y.a + x.d * y.c, x.c * y.b + x.d * y.d};
}
cplxd c2_det(const C2& x) { return x.a * x.d - x.b * x.c; }
C2 c2_inv(const C2& x) {
    const cplxd r = 1.0 / c2_det(x);
    return {x.d * r, -x.b * r, -x.c * r, x.a * r};
}
C2 c2_real(const double m[3]) { return {m[0], m[1], m[1], m[2]}; }

template <class Fn>
cplxd root_continued(Fn at) {
    cplxd prev = 1.0;
    const int steps = 512;
    for (int k = 1; k <= steps; ++k) {
        cplxd r = std::sqrt(c2_det(at((double)k / steps)));
        if (std::abs(r - prev) > std::abs(r + prev)) r = -r;
        prev = r;
    }
    return prev;
}

struct Factor {
    int kind;  // 0 CM, 1 unitary CC, 2 unitary IDFT
    const double* m;
};

cplxd track_amplitude(const Factor* f, int n, C2* S) {
    cplxd amp = 1.0;
    const cplxd j(0.0, 1.0);
    for (int i = 0; i < n; ++i) {
        if (f[i].kind == 0) {
            const C2 P = c2_real(f[i].m);
            *S = {S->a - j * P.a, S->b - j * P.b, S->c - j * P.c, S->d - j * P.d};
        } else if (f[i].kind == 1) {
            const C2 B = c2_real(f[i].m);
            const C2 S0 = *S;
            const C2 SB = c2_mul(S0, B);
            amp /= root_continued([&](double t) {
                return C2{1.0 + j * t * SB.a, j * t * SB.b, j * t * SB.c, 1.0 + j * t * SB.d};
            });
            const C2 Si = c2_inv(S0);
            *S = c2_inv({Si.a + j * B.a, Si.b + j * B.b, Si.c + j * B.c, Si.d + j * B.d});
        } else {
            const C2 S0 = *S;
            amp /= root_continued([&](double t) {
                return C2{(1.0 - t) + t * S0.a, t * S0.b, t * S0.c, (1.0 - t) + t * S0.d};
            });
            *S = c2_inv(S0);
        }
    }
    return amp;
}

// j^q with the route (type 7) equal to the HA chain `ha` of the same matrix;
// -1 if the ratio of the amplitudes is not a power of j (not the same matrix).
int route_phase(const nslct_stages& ha, const double mats[4][3]) {
    const C2 S0{1.1, -0.2, -0.2, 0.9};
    Factor fh[4];
    if (ha.type == 1) {  // CC(H), CM(P3), CC(B'), CM(P1) in application order
        fh[0] = {1, ha.mats[3]};
        fh[1] = {0, ha.mats[2]};
        fh[2] = {1, ha.mats[1]};
        fh[3] = {0, ha.mats[0]};
    } else {  // CM(Q3), CC(B1'), CM(Q1), CC(H1)
        fh[0] = {0, ha.mats[3]};
        fh[1] = {1, ha.mats[2]};
        fh[2] = {0, ha.mats[1]};
        fh[3] = {1, ha.mats[0]};
    }
    const Factor fr[4] = {{2, nullptr}, {0, mats[2]}, {1, mats[1]}, {0, mats[0]}};
    C2 Sh = S0, Sr = S0;
    const cplxd ah = track_amplitude(fh, 4, &Sh);
    const cplxd ar = track_amplitude(fr, 4, &Sr);
    const double smax = std::max({std::abs(Sh.a), std::abs(Sh.b), std::abs(Sh.d), 1.0});
    if (std::max({std::abs(Sh.a - Sr.a), std::abs(Sh.b - Sr.b), std::abs(Sh.d - Sr.d)}) > 1e-8 * smax) return -1;
    const cplxd k = ah / ar;
    const int q = ((int)std::lround(std::arg(k) / (0.25 * kTwoPi)) % 4 + 4) % 4;
    const cplxd jq = q == 0 ? cplxd(1, 0) : q == 1 ? cplxd(0, 1) : q == 2 ? cplxd(-1, 0) : cplxd(0, -1);
    return std::abs(k - jq) <= 1e-6 ? q : -1;
}

bool route_spacing_ok(int N, double d) { return std::fabs(d * d * N / kTwoPi - 1.0) <= 1e-12; }

}  // namespace

namespace {
int build_plan_from(const double abcd[16], int Nx, int Ny, double dx, double dy, const nslct_opts& o,
                    PlanData* out, std::string* err, const double* start_gauge, bool auto_bsym);
}  // namespace

int build_plan(const double abcd[16], int Nx, int Ny, double dx, double dy, const nslct_opts& o,
               PlanData* out, std::string* err) {
    const int rc = build_plan_from(abcd, Nx, Ny, dx, dy, o, out, err, nullptr, true);
    if (rc) return rc;
    out->has_lie = 1;
    std::memcpy(out->abcd0, abcd, sizeof out->abcd0);
    std::memset(out->theta, 0, sizeof out->theta);
    out->opts = o;
    return NSLCT_OK;
}

// A plan that is to be differentiated keeps one decomposition type in a
// neighbourhood of theta: the automatic choice of CM-CC-CM for a symmetric B
// (which a perturbation of theta breaks) is not made, the trace rule picks
// the CM-CC-CM-CC or CC-CM-CC-CM form instead.
int build_plan_lie(const double abcd0[16], const double theta[10], int Nx, int Ny, double dx, double dy,
                   const nslct_opts& o, PlanData* out, std::string* err) {
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(abcd0[i])) {
            *err = "ABCD matrix has a non-finite entry";
            return NSLCT_E_ARG;
        }
    for (int i = 0; i < 10; ++i)
        if (!std::isfinite(theta[i])) {
            *err = "theta has a non-finite entry";
            return NSLCT_E_ARG;
        }
    double M[16];
    lie_point(abcd0, theta, M);
    const int rc = build_plan_from(M, Nx, Ny, dx, dy, o, out, err, nullptr, false);
    if (rc) return rc;
    out->has_lie = 1;
    std::memcpy(out->abcd0, abcd0, sizeof out->abcd0);
    std::memcpy(out->theta, theta, sizeof out->theta);
    out->opts = o;
    return NSLCT_OK;
}

namespace {
// start_gauge: a gauge of a neighbouring matrix to follow locally (HA types
// with type_override 1 or 2 only), else the full search.
int build_plan_from(const double abcd[16], int Nx, int Ny, double dx, double dy, const nslct_opts& o,
                    PlanData* out, std::string* err, const double* start_gauge, bool auto_bsym) {
    int rc = check_common(Nx, Ny, dx, dy, o, err);
    if (rc) return rc;
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(abcd[i])) {
            *err = "ABCD matrix has a non-finite entry";
            return NSLCT_E_ARG;
        }
    const double res = symplectic_residual(abcd);
    if (!(res <= o.symplectic_tol)) {
        *err = "ABCD matrix is not symplectic: max|M J M^T - J| = " + std::to_string(res);
        return NSLCT_E_NOT_SYMPLECTIC;
    }
    std::memset(out, 0, sizeof *out);
    out->Nx = Nx;
    out->Ny = Ny;
    out->precision = o.precision;
    nslct_stages& s = out->st;
    s.dx = dx;
    s.dy = dy;
    s.dwx = kTwoPi / (Nx * dx);
    s.dwy = kTwoPi / (Ny * dy);
    s.symplectic_residual = res;
    const Blocks b = split(abcd);
    double bmax = std::max({std::fabs(b.B.a11), std::fabs(b.B.a12), std::fabs(b.B.a21), std::fabs(b.B.a22)});
    double mmax = 0;
    for (int i = 0; i < 16; ++i) mmax = std::max(mmax, std::fabs(abcd[i]));
    if (bmax < 1e-12) {
        const double ea = std::max({std::fabs(b.A.a11 - 1), std::fabs(b.A.a12), std::fabs(b.A.a21),
                                    std::fabs(b.A.a22 - 1)});
        const double ed = std::max({std::fabs(b.D.a11 - 1), std::fabs(b.D.a12), std::fabs(b.D.a21),
                                    std::fabs(b.D.a22 - 1)});
        if (ea < 1e-12 && ed < 1e-12) {
            s.type = 0;
            sym3(b.C, s.mats[0]);
            s.gauge_objective = gamma_ratio(s.mats[0]);
            fill_chains(out);
            return NSLCT_OK;
        }
        *err = "B = 0 with A or D != I is an affine map, not decomposable into CMs and CCs";
        return NSLCT_E_NO_DECOMPOSITION;
    }
    const double dmin = o.det_min * std::max(1.0, bmax * bmax);
    // Sec. 4.1 covers B = B^T with det B != 0 (eq. Bsym08) by CM-CC-CM, Sec.
    // 4.2 the other matrices by CM-CC-CM-CC: without an override a
    // symmetric invertible B is planned as CM-CC-CM.  (CM-CC-CM is the type-1
    // chain at the gauge H = 0, which is feasible exactly when B is symmetric.)
    const bool bsym_auto = auto_bsym && o.type_override == 0 &&
                           std::fabs(b.B.a12 - b.B.a21) <= 1e-12 * std::max(1.0, bmax) &&
                           std::fabs(det(b.B)) >= dmin;
    if (o.type_override == 3 || bsym_auto) {  // CM-CC-CM (eq. Bsym08: B symmetric, invertible)
        if (std::fabs(b.B.a12 - b.B.a21) > 1e-9 * std::max(1.0, bmax)) {
            *err = "CM-CC-CM needs a symmetric B (eq. Bsym08)";
            return NSLCT_E_NO_DECOMPOSITION;
        }
        const double dt = det(b.B);
        if (!(std::fabs(dt) >= dmin)) {
            *err = "CM-CC-CM needs an invertible B (eq. Bsym08)";
            return NSLCT_E_NO_DECOMPOSITION;
        }
        const M2 Bi{b.B.a22 / dt, -b.B.a12 / dt, -b.B.a21 / dt, b.B.a11 / dt};
        s.type = 3;
        sym3(mul(minus_eye(b.D), Bi), s.mats[0]);
        sym3(b.B, s.mats[1]);
        sym3(mul(Bi, minus_eye(b.A)), s.mats[2]);
        s.gauge_objective = gamma_ratio(s.mats[0]) * gamma_ratio(s.mats[1]) * gamma_ratio(s.mats[2]);
        fill_chains(out);
        return NSLCT_OK;
    }
    if (o.type_override >= 4 && o.type_override <= 6) {  // LC-NsDLCT: rank-one gauge (eqs. LC04-LC10)
        Gauge g{b, 1, dmin};
        double best = INFINITY, bh[3] = {0, 0, 0};
        int btype = 0;
        for (int t = 4; t <= 5; ++t) {
            if (o.type_override != 6 && o.type_override != t) continue;
            const double a = t == 4 ? b.A.a21 : b.A.a12;
            if (std::fabs(a) < 1e-12) continue;
            double h[3] = {0, 0, 0};
            if (t == 4)
                h[0] = (b.B.a21 - b.B.a12) / a;  // eq. LC08
            else
                h[2] = (b.B.a12 - b.B.a21) / a;  // eq. LC10
            const double f = g.objective(h);
            if (f < best) {
                best = f;
                btype = t;
                std::memcpy(bh, h, sizeof bh);
            }
        }
        if (btype) {
            double dt;
            g.stages(bh, s.mats, &dt);
            s.type = btype;
            std::memcpy(s.h, bh, sizeof s.h);
            s.gauge_objective = best;
            fill_chains(out);
            return NSLCT_OK;
        }
        if (o.type_override != 6) {
            *err = "no rank-one gauge with invertible B' (eqs. LC08, LC10)";
            return NSLCT_E_NO_DECOMPOSITION;
        }
        // Neither rank-one form gives an invertible B' (Sec. 4.2.2): for
        // a12 = a21 = 0 the IDFT route where it applies, else the HA-NsDLCT,
        // its type by the trace rule.
    }
    if (o.type_override == 7 || o.type_override == 6) {
        const double amax = std::max({std::fabs(b.A.a11), std::fabs(b.A.a12), std::fabs(b.A.a21), std::fabs(b.A.a22)});
        const double sc = std::max(1.0, mmax);
        std::string why;
        int wrc = NSLCT_OK;
        if (std::fabs(b.A.a12) > 1e-12 * sc || std::fabs(b.A.a21) > 1e-12 * sc) {
            why = "the IDFT route needs a12 = a21 = 0 (Sec. 4.2.2)";
            wrc = NSLCT_E_NO_DECOMPOSITION;
        } else if (!(std::fabs(det(b.A)) >= o.det_min * std::max(1.0, amax * amax))) {
            why = "the IDFT route needs an invertible A (eq. Bsym08 for (-B, A; -D, C))";
            wrc = NSLCT_E_NO_DECOMPOSITION;
        } else if (!route_spacing_ok(Nx, dx) || !route_spacing_ok(Ny, dy)) {
            why = "the IDFT route keeps the grid only at dx = sqrt(2 pi / Nx), dy = sqrt(2 pi / Ny)";
            wrc = NSLCT_E_UNSUPPORTED;
        } else if (!native_size(Nx) || !native_size(Ny)) {
            why = "the IDFT route runs native lengths (2^k, 3 * 2^k) only";
            wrc = NSLCT_E_SIZE;
        } else if (o.precision != NSLCT_C64 && o.precision != NSLCT_C128) {
            why = "the IDFT route runs complex64 / complex128 only";
            wrc = NSLCT_E_UNSUPPORTED;
        }
        if (wrc == NSLCT_OK) {
            // The HA chain of M fixes the operator the route must equal.
            nslct_opts oh = o;
            oh.type_override = 0;
            PlanData ha;
            const int hrc = build_plan_from(abcd, Nx, Ny, dx, dy, oh, &ha, err, nullptr, false);
            if (hrc) return hrc;
            const double dt = det(b.A);
            const M2 Ai{b.A.a22 / dt, -b.A.a12 / dt, -b.A.a21 / dt, b.A.a11 / dt};
            const M2 mB{-b.B.a11, -b.B.a12, -b.B.a21, -b.B.a22};
            double mats[4][3] = {};
            sym3(mul(minus_eye(b.C), Ai), mats[0]);  // P1' = (C - I) A^-1
            sym3(b.A, mats[1]);
            sym3(mul(Ai, minus_eye(mB)), mats[2]);   // P3' = A^-1 (-B - I)
            const int q = route_phase(ha.st, mats);
            if (q < 0) {
                *err = "IDFT route: the two factorisations do not reach the same matrix";
                return NSLCT_E_NO_DECOMPOSITION;
            }
            s.type = 7;
            s.phase_q = q;
            std::memcpy(s.mats, mats, sizeof mats);
            s.gauge_objective = gamma_ratio(mats[0]) * gamma_ratio(mats[1]) * gamma_ratio(mats[2]);
            fill_chains(out);
            return NSLCT_OK;
        }
        if (o.type_override == 7) {
            *err = why;
            return wrc;
        }
    }
    int type = o.type_override >= 4 ? 0 : o.type_override;  // 6 (and 7 handled above): trace rule
    if (type == 0) type = (b.B.a11 + b.B.a22) < 0 ? 2 : 1;
    Gauge g{b, type, dmin};
    GaugeOut go;
    if (start_gauge && o.type_override != 0) go = solve(g, mmax, start_gauge);
    if (!go.found) go = solve(g, mmax);
    if ((o.type_override == 0 || o.type_override == 6) && !go.feasible) {
        g.type = type = 3 - type;
        go = solve(g, mmax);
    }
    if (!go.found) {
        *err = "no symmetric gauge H with invertible middle CC matrix (eqs. Bnonsym32, HA24)";
        return NSLCT_E_NO_DECOMPOSITION;
    }
    s.type = type;
    double dt;
    g.stages(go.h, s.mats, &dt);
    std::memcpy(s.h, go.h, sizeof s.h);
    s.gauge_objective = go.f;
    fill_chains(out);
    return NSLCT_OK;
}

}  // namespace

int build_plan_from_stages(const nslct_stages& st, int Nx, int Ny, const nslct_opts& o, PlanData* out,
                           std::string* err) {
    int rc = check_common(Nx, Ny, st.dx, st.dy, o, err);
    if (rc) return rc;
    if (st.type < 0 || st.type > 7 || st.type == 6) {
        *err = "stage type must be in 0..5 or 7";
        return NSLCT_E_ARG;
    }
    if (st.type == 7) {
        if (!route_spacing_ok(Nx, st.dx) || !route_spacing_ok(Ny, st.dy)) {
            *err = "the IDFT route keeps the grid only at dx = sqrt(2 pi / Nx), dy = sqrt(2 pi / Ny)";
            return NSLCT_E_UNSUPPORTED;
        }
        if (!native_size(Nx) || !native_size(Ny)) {
            *err = "the IDFT route runs native lengths (2^k, 3 * 2^k) only";
            return NSLCT_E_SIZE;
        }
        if (o.precision != NSLCT_C64 && o.precision != NSLCT_C128) {
            *err = "the IDFT route runs complex64 / complex128 only";
            return NSLCT_E_UNSUPPORTED;
        }
    }
    const int nm = st.type == 0 ? 1 : (st.type == 3 || st.type == 7) ? 3 : 4;
    if ((st.type == 4 && (st.mats[3][1] != 0 || st.mats[3][2] != 0)) ||
        (st.type == 5 && (st.mats[3][0] != 0 || st.mats[3][1] != 0))) {
        *err = "LC stages need H = (h, 0; 0, 0) (type 4) or (0, 0; 0, h) (type 5)";
        return NSLCT_E_ARG;
    }
    for (int i = 0; i < nm; ++i)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(st.mats[i][k])) {
                *err = "stage matrix has a non-finite entry";
                return NSLCT_E_ARG;
            }
    std::memset(out, 0, sizeof *out);
    out->Nx = Nx;
    out->Ny = Ny;
    out->precision = o.precision;
    nslct_stages& s = out->st;
    s.type = st.type;
    for (int i = 0; i < nm; ++i)
        for (int k = 0; k < 3; ++k) s.mats[i][k] = st.mats[i][k];
    if (st.type == 4 || st.type == 5)
        for (int k = 0; k < 3; ++k) s.h[k] = st.mats[3][k];
    if (st.type == 7) s.phase_q = st.phase_q & 3;
    s.dx = st.dx;
    s.dy = st.dy;
    s.dwx = kTwoPi / (Nx * st.dx);
    s.dwy = kTwoPi / (Ny * st.dy);
    double f = 1.0;
    for (int i = 0; i < nm; ++i) f *= gamma_ratio(s.mats[i]);
    s.gauge_objective = f;
    s.symplectic_residual = 0.0;
    fill_chains(out);
    return NSLCT_OK;
}

namespace {

void mat4_mul(const double* a, const double* b, double* c) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double t = 0;
            for (int k = 0; k < 4; ++k) t += a[4 * i + k] * b[4 * k + j];
            c[4 * i + j] = t;
        }
}

// exp(X) for a 4x4 X: scaling and squaring around a degree-14 Taylor series.
void mat4_exp(const double* X, double* out) {
    double nrm = 0;
    for (int i = 0; i < 4; ++i) {
        double r = 0;
        for (int j = 0; j < 4; ++j) r += std::fabs(X[4 * i + j]);
        nrm = std::max(nrm, r);
    }
    int sq = 0;
    while (nrm > 0.25 && sq < 60) {
        nrm *= 0.5;
        ++sq;
    }
    const double sc = std::ldexp(1.0, -sq);
    double Y[16], term[16], tmp[16];
    for (int i = 0; i < 16; ++i) Y[i] = X[i] * sc;
    for (int i = 0; i < 16; ++i) out[i] = term[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int k = 1; k <= 14; ++k) {
        mat4_mul(term, Y, tmp);
        for (int i = 0; i < 16; ++i) {
            term[i] = tmp[i] / k;
            out[i] += term[i];
        }
    }
    for (int k = 0; k < sq; ++k) {
        mat4_mul(out, out, tmp);
        std::memcpy(out, tmp, sizeof tmp);
    }
}

// J S(theta): S symmetric 4x4 whose upper triangle, row by row, is theta
// (s11, s12, s13, s14, s22, s23, s24, s33, s34, s44).
void lie_matrix(const double theta[10], double* X) {
    double S[16] = {0};
    int k = 0;
    for (int r = 0; r < 4; ++r)
        for (int c = r; c < 4; ++c, ++k) S[4 * r + c] = S[4 * c + r] = theta[k];
    const double J[16] = {0, 0, 1, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, -1, 0, 0};
    mat4_mul(J, S, X);
}

}  // namespace

void lie_point(const double abcd[16], const double theta[10], double* M) {
    double X[16], E[16];
    lie_matrix(theta, X);
    mat4_exp(X, E);
    mat4_mul(abcd, E, M);
}

namespace {

// Central differences of the planner along theta with the decomposition type
// held and the gauge followed from `base_h` (the minimiser at theta0).
int jacobian_followed(const double abcd[16], const double theta0[10], int Nx, int Ny, double dx, double dy,
                      const nslct_opts& o, int base_type, const double base_h[3], double h,
                      double jac[12 * 10], std::string* err) {
    int rc = 0;
    nslct_opts of = o;
    of.type_override = base_type;  // stay on one decomposition type
    for (int i = 0; i < 10; ++i) {
        double tp[10], tm[10], Mp[16], Mm[16];
        for (int k = 0; k < 10; ++k) tp[k] = tm[k] = theta0[k];
        tp[i] += h;
        tm[i] -= h;
        lie_point(abcd, tp, Mp);
        lie_point(abcd, tm, Mm);
        PlanData pp, pm;
        rc = build_plan_from(Mp, Nx, Ny, dx, dy, of, &pp, err, base_h, false);
        if (!rc) rc = build_plan_from(Mm, Nx, Ny, dx, dy, of, &pm, err, base_h, false);
        if (rc) return rc;
        if (pp.st.type != pm.st.type) {
            *err = "decomposition type changes within the difference step";
            return NSLCT_E_NO_DECOMPOSITION;
        }
        for (int m = 0; m < 4; ++m)
            for (int k = 0; k < 3; ++k) jac[(3 * m + k) * 10 + i] = (pp.st.mats[m][k] - pm.st.mats[m][k]) / (2 * h);
    }
    return NSLCT_OK;
}

// The twelve stage entries (order of nslct_stages.mats) of a type-1/2 gauge
// h for the matrix M(theta); false where B' is not invertible.
bool stage_entries(const Gauge& g, const double h[3], double e[12]) {
    double st[4][3], dt;
    if (!g.stages(h, st, &dt)) return false;
    for (int m = 0; m < 4; ++m)
        for (int k = 0; k < 3; ++k) e[3 * m + k] = st[m][k];
    return true;
}

// Solves the 3 x 3 system A x = b (Gaussian elimination, partial pivoting);
// false when A is singular to working precision.
bool solve3(double A[3][3], double b[3], double x[3]) {
    int p[3] = {0, 1, 2};
    double a[3][4];
    double amax = 0;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            a[r][c] = A[r][c];
            amax = std::max(amax, std::fabs(A[r][c]));
        }
        a[r][3] = b[r];
    }
    if (!(amax > 0)) return false;
    for (int c = 0; c < 3; ++c) {
        int best = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(a[p[r]][c]) > std::fabs(a[p[best]][c])) best = r;
        std::swap(p[c], p[best]);
        const double piv = a[p[c]][c];
        if (std::fabs(piv) <= 1e-13 * amax) return false;
        for (int r = c + 1; r < 3; ++r) {
            const double f = a[p[r]][c] / piv;
            for (int k = c; k < 4; ++k) a[p[r]][k] -= f * a[p[c]][k];
        }
    }
    for (int c = 2; c >= 0; --c) {
        double v = a[p[c]][3];
        for (int k = c + 1; k < 3; ++k) v -= a[p[c]][k] * x[k];
        x[c] = v / a[p[c]][c];
    }
    return true;
}

// d(stage entries)/d(theta) of a type-1/2 plan by the implicit function
// theorem.  The eq. HA24 minimiser sits where `need` stage entries vanish
// (the |.| kinks of the gamma ratios), need = 3 - (number of feasibility
// equations): with the kink set held, the gauge H(theta) is the solution of
//   F(H, theta) = [feasibility c(M) . h - rhs(M); e_k(H, M), k in the kink set] = 0,
// so dH/dtheta = -F_H^-1 F_theta and d(stages)/dtheta = S_theta + S_H dH/dtheta.
// The partial derivatives of these closed-form functions are central
// differences with steps of 1e-6 (no gauge search is repeated).  Returns
// false (the caller falls back to re-solved differences) when fewer than
// `need` entries vanish or no choice of them gives a regular F_H.
bool jacobian_implicit(const PlanData& p, double jac[12 * 10]) {
    const int type = p.st.type;
    if (type != 1 && type != 2) return false;
    double M[16];
    lie_point(p.abcd0, p.theta, M);
    const Blocks b0 = split(M);
    double bmax = std::max({std::fabs(b0.B.a11), std::fabs(b0.B.a12), std::fabs(b0.B.a21), std::fabs(b0.B.a22)});
    const double dmin = p.opts.det_min * std::max(1.0, bmax * bmax);
    auto gauge_at = [&](const double* theta) {
        double Mt[16];
        lie_point(p.abcd0, theta, Mt);
        return Gauge{split(Mt), type, dmin};
    };
    const double* h0 = p.st.h;
    const Gauge g0 = gauge_at(p.theta);
    double c[3], rhs;
    g0.equation(c, &rhs);
    double mmax = 0;
    for (double v : M) mmax = std::max(mmax, std::fabs(v));
    const bool plane = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) > 1e-12 * std::max(1.0, mmax);
    const int need = plane ? 2 : 3;
    double e0[12];
    if (!stage_entries(g0, h0, e0)) return false;
    double emax = 0;
    for (double v : e0) emax = std::max(emax, std::fabs(v));
    std::vector<int> kink;
    for (int k = 0; k < 12; ++k)
        if (std::fabs(e0[k]) <= 1e-9 * (1 + emax)) kink.push_back(k);
    if ((int)kink.size() < need) return false;
    // F(H, theta) for a chosen kink subset.
    auto F = [&](const Gauge& g, const double* h, const int* ks, double* out) {
        double e[12];
        if (!stage_entries(g, h, e)) return false;
        int n = 0;
        if (plane) {
            double cc[3], rr;
            g.equation(cc, &rr);
            out[n++] = cc[0] * h[0] + cc[1] * h[1] + cc[2] * h[2] - rr;
        }
        for (int i = 0; i < need; ++i) out[n++] = e[ks[i]];
        return true;
    };
    const double sh = 1e-6 * (1 + std::fabs(h0[0]) + std::fabs(h0[1]) + std::fabs(h0[2]));
    const double st = 1e-6;
    // Pick the kink subset with the best-conditioned F_H.
    double FH[3][3] = {};
    int best[3] = {0, 0, 0};
    double best_det = 0;
    const int nk = (int)kink.size();
    for (int a = 0; a < nk; ++a)
        for (int bb = a + 1; bb < nk; ++bb)
            for (int cc3 = need == 3 ? bb + 1 : nk - 1; cc3 < nk; ++cc3) {
                int ks[3] = {kink[a], kink[bb], need == 3 ? kink[cc3] : 0};
                double J[3][3];
                bool ok = true;
                for (int j = 0; j < 3 && ok; ++j) {
                    double hp[3] = {h0[0], h0[1], h0[2]}, hm[3] = {h0[0], h0[1], h0[2]};
                    hp[j] += sh;
                    hm[j] -= sh;
                    double fp[3], fm[3];
                    ok = F(g0, hp, ks, fp) && F(g0, hm, ks, fm);
                    for (int r = 0; r < 3 && ok; ++r) J[r][j] = (fp[r] - fm[r]) / (2 * sh);
                }
                if (!ok) continue;
                const double d = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                if (std::fabs(d) > std::fabs(best_det)) {
                    best_det = d;
                    std::memcpy(best, ks, sizeof best);
                    std::memcpy(FH, J, sizeof FH);
                }
                if (need == 2) break;  // the inner index is unused
            }
    if (!(std::fabs(best_det) > 0)) return false;
    double dH[3][10];
    double S_theta[12][10];
    for (int i = 0; i < 10; ++i) {
        double tp[10], tm[10];
        for (int k = 0; k < 10; ++k) tp[k] = tm[k] = p.theta[k];
        tp[i] += st;
        tm[i] -= st;
        const Gauge gp = gauge_at(tp), gm = gauge_at(tm);
        double fp[3], fm[3], ep[12], em[12];
        if (!F(gp, h0, best, fp) || !F(gm, h0, best, fm)) return false;
        if (!stage_entries(gp, h0, ep) || !stage_entries(gm, h0, em)) return false;
        double Ft[3], x[3];
        for (int r = 0; r < 3; ++r) Ft[r] = -(fp[r] - fm[r]) / (2 * st);
        double A[3][3];
        std::memcpy(A, FH, sizeof A);
        if (!solve3(A, Ft, x)) return false;
        for (int r = 0; r < 3; ++r) dH[r][i] = x[r];
        for (int m = 0; m < 12; ++m) S_theta[m][i] = (ep[m] - em[m]) / (2 * st);
    }
    double S_H[12][3];
    for (int j = 0; j < 3; ++j) {
        double hp[3] = {h0[0], h0[1], h0[2]}, hm[3] = {h0[0], h0[1], h0[2]};
        hp[j] += sh;
        hm[j] -= sh;
        double ep[12], em[12];
        if (!stage_entries(g0, hp, ep) || !stage_entries(g0, hm, em)) return false;
        for (int m = 0; m < 12; ++m) S_H[m][j] = (ep[m] - em[m]) / (2 * sh);
    }
    for (int m = 0; m < 12; ++m)
        for (int i = 0; i < 10; ++i) {
            double v = S_theta[m][i];
            for (int j = 0; j < 3; ++j) v += S_H[m][j] * dH[j][i];
            jac[m * 10 + i] = v;
        }
    return true;
}

}  // namespace

int plan_jacobian(const double abcd[16], const double theta0[10], int Nx, int Ny, double dx, double dy,
                  const nslct_opts& o, double h, double jac[12 * 10], std::string* err) {
    if (!(h > 0) || h > 1e-2) {
        *err = "step must be in (0, 1e-2]";
        return NSLCT_E_ARG;
    }
    double M0[16];
    lie_point(abcd, theta0, M0);
    PlanData base;
    int rc = build_plan_from(M0, Nx, Ny, dx, dy, o, &base, err, nullptr, false);
    if (rc) return rc;
    return jacobian_followed(abcd, theta0, Nx, Ny, dx, dy, o, base.st.type == 0 ? 0 : base.st.type, base.st.h,
                             h, jac, err);
}

int plan_theta_jacobian(const PlanData& p, double jac[12 * 10], std::string* err) {
    if (!p.has_lie) {
        *err = "the plan was made from stage matrices: no ABCD parameterisation to differentiate";
        return NSLCT_E_UNSUPPORTED;
    }
    if (p.st.type == 7) {
        *err = "the IDFT route (type 7) has no decomposition of the same type at perturbed matrices";
        return NSLCT_E_UNSUPPORTED;
    }
    if (p.st.type == 3 && p.opts.type_override == 0) {
        *err = "a CM-CC-CM plan chosen for a symmetric B has no decomposition of the same type at "
               "perturbed matrices; plan with nslct_plan_lie to differentiate";
        return NSLCT_E_UNSUPPORTED;
    }
    // A searched gauge on a full kink set: the implicit-function derivative.
    if (jacobian_implicit(p, jac)) return NSLCT_OK;
    // Otherwise central differences of the planner, the gauge followed from
    // the plan's own; closed-form stages (types 3-5) take a smaller step than
    // a searched gauge, whose minimiser is resolved to about 1e-12.
    const double h = p.st.type >= 3 ? 1e-5 : 1e-4;
    return jacobian_followed(p.abcd0, p.theta, p.Nx, p.Ny, p.st.dx, p.st.dy, p.opts,
                             p.st.type == 0 ? 0 : p.st.type, p.st.h, h, jac, err);
}

void theta_gradient(const double jac[12 * 10], const double gst[12], double out[10]) {
    for (int i = 0; i < 10; ++i) {
        double acc = 0;
        for (int m = 0; m < 12; ++m) acc += jac[m * 10 + i] * gst[m];
        out[i] = acc;
    }
}

void stage_gradient(const PlanData& p, const double sums[15], double g[12]) {
    // sums[3k..3k+2]: inverse-chain pass k, weights x^2, x y, y^2 in index
    // units, values scaled by s^2 relative to the unitary chain.
    const double Nx = p.Nx, Ny = p.Ny;
    const double s2[5] = {1.0, Nx * Ny, Ny * Ny, Nx * Ny, Ny * Ny};
    double slot[5][3];
    for (int k = 0; k < 5; ++k) {
        const int j = 4 - k;  // forward slot at this point of the inverse chain
        const bool freq = (j == 1 || j == 3);
        const double da = freq ? p.st.dwx : p.st.dx, db = freq ? p.st.dwy : p.st.dy;
        // d loss / d p = Re sum conj(r) i (d phi / d p) u = -(d phi / d p) Im(conj(r) u)
        slot[j][0] = -0.5 * da * da * sums[3 * k + 0] / s2[k];
        slot[j][1] = -da * db * sums[3 * k + 1] / s2[k];
        slot[j][2] = -0.5 * db * db * sums[3 * k + 2] / s2[k];
    }
    auto put = [&](int m, int j, double sg) {
        for (int k = 0; k < 3; ++k) g[3 * m + k] = sg * slot[j][k];
    };
    for (int k = 0; k < 12; ++k) g[k] = 0;
    if (p.st.type == 1 || p.st.type == 4 || p.st.type == 5) {  // {P1, B', P3, H} = {S4, -C3, S2, -C1}
        put(0, 4, 1.0);
        put(1, 3, -1.0);
        put(2, 2, 1.0);
        put(3, 1, -1.0);
    } else if (p.st.type == 2) {  // {H1, Q1, B1', Q3} = {-C3, S2, -C1, S0}
        put(0, 3, -1.0);
        put(1, 2, 1.0);
        put(2, 1, -1.0);
        put(3, 0, 1.0);
    } else if (p.st.type == 3) {  // {P1, B, P3} = {S4, -C1, S0}
        put(0, 4, 1.0);
        put(1, 1, -1.0);
        put(2, 0, 1.0);
    } else {
        put(0, 0, 1.0);
    }
}

bool box_check(const PlanData& p, double frac) {
    const nslct_stages& s = p.st;
    double X = frac * p.Nx * s.dx / 2, Y = frac * p.Ny * s.dy / 2;
    double Wx = frac * (0.5 * kTwoPi) / s.dx, Wy = frac * (0.5 * kTwoPi) / s.dy;
    const double lX = p.Nx * s.dx / 2, lY = p.Ny * s.dy / 2, lWx = (0.5 * kTwoPi) / s.dx, lWy = (0.5 * kTwoPi) / s.dy;
    // Forward chain slots in application order: CM(S0), CC via C1, CM(S2), CC via C3, CM(S4).
    // A CC with chirp -X in the frequency domain shears positions by X (eq. HA20);
    // a CM with matrix P shears frequencies by P z (eq. HA12).
    const Chain5& c = p.dir[0];
    auto ok = [&]() {
        const double e = 1 + 1e-12;
        return X <= lX * e && Y <= lY * e && Wx <= lWx * e && Wy <= lWy * e;
    };
    for (int k = 0; k < 5; ++k) {
        const double* m = c.slot[k];
        if (k == 1 || k == 3) {
            const double nx = X + std::fabs(m[0]) * Wx + std::fabs(m[1]) * Wy;
            const double ny = Y + std::fabs(m[1]) * Wx + std::fabs(m[2]) * Wy;
            X = nx;
            Y = ny;
        } else {
            if (m[0] == 0 && m[1] == 0 && m[2] == 0) continue;
            const double nx = Wx + std::fabs(m[0]) * X + std::fabs(m[1]) * Y;
            const double ny = Wy + std::fabs(m[1]) * X + std::fabs(m[2]) * Y;
            Wx = nx;
            Wy = ny;
        }
        if (!ok()) return false;
    }
    return true;
}

}  // namespace nslct
