"""Decompositions and the HA gauge problem (oracle; test infrastructure only).

CM-CC-CM-CC (Sec. 4.2, eqs. Bnonsym04-Bnonsym12): M = (A, B'; C, D')(I, H; 0, I)
with H = H^T, B' = B - A H, D' = D - C H; B' must be symmetric and
invertible.  The chain, rightmost applied first, is
    CM((D' - I) B'^-1) . CC(B') . CM(B'^-1 (A - I)) . CC(H).

CC-CM-CC-CM (Sec. 4.3, eqs. CCCMCCCM08-CCCMCCCM16): M = (I, H1; 0, I)(A1', B1'; C, D)
with B1' = B - H1 D, A1' = A - H1 C, giving
    CC(H1) . CM((D - I) B1'^-1) . CC(B1') . CM(B1'^-1 (A1' - I)).

Feasibility: B' symmetric is one linear equation in (h11, h12, h22)
(eq. Bnonsym32); the same holds for B1' in the second type.

Objective: the HA gauge minimises the product of the phase-space growth ratios
gamma(X) = (|x11| + |x12| + 1)(|x12| + |x22| + 1) (eq. HA16) of the four stage
matrices (eq. HA24).  The paper states the second type's gauge is found by a
"similar" approach; the reading used here is the same product over that
type's four stage matrices.

The problem is not convex and its minima sit on the |.| kinks, so it is solved
by brute force: a dense grid over the feasible plane (or the whole of Sym(2)
when the equation is void), Nelder-Mead polishing of the best cells, then
"kink snapping" (solving for the points where the near-zero entries vanish
exactly).  Ties within relative 1e-9 go to the smallest ||H||_F, then the
lexicographically smallest (h11, h12, h22).  The box is
|coordinate| <= 4 (1 + max|M_ij|).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import optimize

from .symplectic import blocks

TIE_RTOL = 1e-9


def det_bound(M) -> float:
    """Smallest |det B'| accepted: 1e-6 * max(1, max|B_ij|^2)."""
    _, B, _, _ = blocks(M)
    return 1e-6 * max(1.0, float(np.max(np.abs(B))) ** 2)


def gamma(X) -> float:
    """Phase-space growth ratio of a symmetric 2x2 matrix (eq. HA16)."""
    x11, x22 = X[0][0], X[1][1]
    x12 = 0.5 * (X[0][1] + X[1][0])
    return (abs(x11) + abs(x12) + 1.0) * (abs(x12) + abs(x22) + 1.0)


def trace_type(M) -> int:
    """Decomposition type by the trace rule of eq. Reversible08.

    1 (CM-CC-CM-CC) when tr B > 0, 2 (CC-CM-CC-CM) when tr B < 0; the paper
    does not cover tr B = 0, which is read as type 1.
    """
    _, B, _, _ = blocks(M)
    return 2 if (B[0, 0] + B[1, 1]) < 0 else 1


def feasible_equation(M, typ: int):
    """Coefficients (c, rhs) of the linear feasibility equation c . h = rhs.

    Type 1: (B - A H)_12 = (B - A H)_21
        -a21 h11 + (a11 - a22) h12 + a12 h22 = b12 - b21.
    Type 2: (B - H1 D)_12 = (B - H1 D)_21
        d12 h11 + (d22 - d11) h12 - d21 h22 = b12 - b21.
    """
    A, B, _, D = blocks(M)
    rhs = B[0, 1] - B[1, 0]
    if typ == 1:
        c = np.array([-A[1, 0], A[0, 0] - A[1, 1], A[0, 1]])
    else:
        c = np.array([D[0, 1], D[1, 1] - D[0, 0], -D[1, 0]])
    return c, float(rhs)


def _sym(h):
    return np.array([[h[0], h[1]], [h[1], h[2]]], dtype=np.float64)


def stage_matrices(M, typ: int, h):
    """The four chirp matrices of the decomposition at gauge h = (h11,h12,h22).

    Returned in the order they appear in the formula (leftmost first):
      type 1: P1 = (D'-I)B'^-1, B', P3 = B'^-1(A-I), H      (eq. Bnonsym12)
      type 2: H1, Q1 = (D-I)B1'^-1, B1', Q3 = B1'^-1(A1'-I) (eq. CCCMCCCM16)
    plus det of the middle CC matrix.  Matrices are not symmetrised here.
    """
    A, B, C, D = blocks(M)
    I2 = np.eye(2)
    Hm = _sym(h)
    if typ == 1:
        Bp = B - A @ Hm
        Dp = D - C @ Hm
        det = Bp[0, 0] * Bp[1, 1] - Bp[0, 1] * Bp[1, 0]
        if det == 0.0:
            return None, det
        Bi = np.array([[Bp[1, 1], -Bp[0, 1]], [-Bp[1, 0], Bp[0, 0]]]) / det
        P1 = (Dp - I2) @ Bi
        P3 = Bi @ (A - I2)
        return (P1, Bp, P3, Hm), det
    Bp = B - Hm @ D
    Ap = A - Hm @ C
    det = Bp[0, 0] * Bp[1, 1] - Bp[0, 1] * Bp[1, 0]
    if det == 0.0:
        return None, det
    Bi = np.array([[Bp[1, 1], -Bp[0, 1]], [-Bp[1, 0], Bp[0, 0]]]) / det
    Q1 = (D - I2) @ Bi
    Q3 = Bi @ (Ap - I2)
    return (Hm, Q1, Bp, Q3), det


def objective(M, typ: int, h, dmin: float | None = None) -> float:
    """HA objective of eq. HA24 (product of four gamma ratios), inf if infeasible."""
    if dmin is None:
        dmin = det_bound(M)
    mats, det = stage_matrices(M, typ, h)
    if mats is None or abs(det) < dmin:
        return math.inf
    f = 1.0
    for X in mats:
        f *= gamma(X)
    return f


def _objective_grid(M, typ, h11, h12, h22, dmin):
    """Vectorised objective over arrays of gauges (same formulas as above)."""
    A, B, C, D = blocks(M)
    # Stack the gauges as (K, 2, 2) symmetric matrices.
    K = h11.shape[0]
    Hm = np.empty((K, 2, 2))
    Hm[:, 0, 0] = h11
    Hm[:, 0, 1] = h12
    Hm[:, 1, 0] = h12
    Hm[:, 1, 1] = h22
    I2 = np.eye(2)
    if typ == 1:
        Bp = B[None] - A[None] @ Hm
        Dp = D[None] - C[None] @ Hm
    else:
        Bp = B[None] - Hm @ D[None]
        Ap = A[None] - Hm @ C[None]
    det = Bp[:, 0, 0] * Bp[:, 1, 1] - Bp[:, 0, 1] * Bp[:, 1, 0]
    ok = np.abs(det) >= dmin
    safe = np.where(ok, det, 1.0)
    Bi = np.empty_like(Bp)
    Bi[:, 0, 0] = Bp[:, 1, 1] / safe
    Bi[:, 0, 1] = -Bp[:, 0, 1] / safe
    Bi[:, 1, 0] = -Bp[:, 1, 0] / safe
    Bi[:, 1, 1] = Bp[:, 0, 0] / safe
    if typ == 1:
        mats = ((Dp - I2) @ Bi, Bp, Bi @ (A - I2)[None], Hm)
    else:
        mats = (Hm, (D - I2)[None] @ Bi, Bp, Bi @ (Ap - I2))
    f = np.ones(K)
    for X in mats:
        x12 = 0.5 * (X[:, 0, 1] + X[:, 1, 0])
        f *= (np.abs(X[:, 0, 0]) + np.abs(x12) + 1.0) * (np.abs(x12) + np.abs(X[:, 1, 1]) + 1.0)
    return np.where(ok, f, np.inf)


def _entries(M, typ, h):
    """The 12 distinct entries of the four stage matrices (kink locations)."""
    mats, det = stage_matrices(M, typ, h)
    if mats is None:
        return None
    out = []
    for X in mats:
        out += [X[0, 0], 0.5 * (X[0, 1] + X[1, 0]), X[1, 1]]
    return np.array(out)


class GaugeResult:
    """Outcome of the brute-force gauge search."""

    def __init__(self, typ, h, f, feasible, dim):
        self.typ = typ
        self.h = None if h is None else np.asarray(h, dtype=np.float64)
        self.f = f
        self.feasible = feasible
        self.dim = dim

    def __repr__(self):
        return f"GaugeResult(type={self.typ}, h={self.h}, f={self.f}, dim={self.dim})"


def _param(M, typ):
    """Affine parametrisation h = h0 + U s of the feasible set, or None."""
    c, rhs = feasible_equation(M, typ)
    scale = max(1.0, float(np.max(np.abs(M))))
    if np.linalg.norm(c) <= 1e-12 * scale:
        if abs(rhs) > 1e-12 * scale:
            return None                       # empty: 0 = rhs != 0
        return np.zeros(3), np.eye(3)         # all of Sym(2)
    h0 = c * rhs / float(c @ c)
    # Orthonormal basis of the plane c . h = 0 (the last two right-singular vectors).
    _, _, vt = np.linalg.svd(c[None, :])
    return h0, vt[1:].T


def _pick(cands):
    """Tie-break: smallest f (relative 1e-9), then ||H||_F, then lexicographic."""
    cands = [(f, h) for f, h in cands if math.isfinite(f)]
    if not cands:
        return None
    fmin = min(f for f, _ in cands)
    tied = [(f, h) for f, h in cands if f <= fmin * (1.0 + TIE_RTOL)]
    tied.sort(key=lambda fh: (round(float(fh[1][0] ** 2 + 2 * fh[1][1] ** 2 + fh[1][2] ** 2), 12),
                              round(float(fh[1][0]), 12), round(float(fh[1][1]), 12),
                              round(float(fh[1][2]), 12)))
    return tied[0]


def solve_gauge(M, typ: int, grid: int | None = None, starts: int = 8) -> GaugeResult:
    """Brute-force minimiser of eq. HA24 over the feasible gauge set."""
    M = np.asarray(M, dtype=np.float64)
    pr = _param(M, typ)
    if pr is None:
        return GaugeResult(typ, None, math.inf, False, 0)
    h0, U = pr
    dim = U.shape[1]
    dmin = det_bound(M)
    R = 4.0 * (1.0 + float(np.max(np.abs(M))))
    if grid is None:
        grid = 401 if dim == 2 else 101
    ax = np.linspace(-R, R, grid)
    mesh = np.meshgrid(*([ax] * dim), indexing="ij")
    S = np.stack([g.ravel() for g in mesh], axis=1)          # (K, dim)
    Hs = h0[None, :] + S @ U.T
    F = _objective_grid(M, typ, Hs[:, 0], Hs[:, 1], Hs[:, 2], dmin)
    if not np.any(np.isfinite(F)):
        return GaugeResult(typ, None, math.inf, True, dim)

    def fs(s):
        return objective(M, typ, h0 + U @ np.asarray(s), dmin)

    # Best grid cells, kept at least 3 cells apart.
    order = np.argsort(F)
    step = ax[1] - ax[0]
    seeds = []
    for idx in order:
        if not math.isfinite(F[idx]):
            break
        s = S[idx]
        if all(np.max(np.abs(s - t)) > 3 * step for t in seeds):
            seeds.append(s)
        if len(seeds) >= starts:
            break
    cands = []
    for s in seeds:
        simplex = np.vstack([s] + [s + step * e for e in np.eye(dim)])
        f0 = fs(s)
        res = optimize.minimize(fs, s, method="Nelder-Mead",
                                options=dict(xatol=1e-11, fatol=1e-13 * f0, maxiter=20000,
                                             maxfev=20000, initial_simplex=simplex))
        s_best = res.x
        cands.append((fs(s_best), h0 + U @ s_best))
        cands.extend(_snap(M, typ, h0, U, s_best, dmin))
    best = _pick(cands)
    return GaugeResult(typ, best[1], best[0], True, dim)


def _snap(M, typ, h0, U, s, dmin):
    """Solve for the nearby points where dim of the near-zero entries vanish."""
    dim = U.shape[1]
    e = _entries(M, typ, h0 + U @ s)
    if e is None:
        return []
    scale = 1.0 + float(np.max(np.abs(e)))
    near = [i for i in range(12) if abs(e[i]) < 1e-4 * scale]
    out = []
    for sub in itertools.combinations(near, dim):
        def eqs(x, sub=sub):
            v = _entries(M, typ, h0 + U @ x)
            return np.full(dim, 1e6) if v is None else v[list(sub)]
        try:
            sol = optimize.root(eqs, s, method="hybr", options=dict(xtol=1e-15))
        except Exception:  # pragma: no cover - singular Jacobian paths
            continue
        if not sol.success:
            continue
        if np.max(np.abs(eqs(sol.x))) > 1e-12 * scale:
            continue
        h = h0 + U @ sol.x
        # Exact zeros where the snap put them (removes 1e-17 residue).
        out.append((objective(M, typ, h, dmin), h))
    return out
