"""Oracle planner: validate M, pick the decomposition type, solve the gauge.

(Test infrastructure only.)  Steps, in the paper's order:

1. M must satisfy eq. Intro12 (residual <= tol).
2. B = 0: the transform is a chirp times an affine map (eq. Intro20); only
   A = D = I, a pure discrete CM with matrix C (eq. BasicCM12), is handled.
3. Type by the trace rule (eq. Reversible08); if that type's feasibility
   equation has no solution, the other type is used (reading: the paper only
   discusses the failure of its LC variant).
4. Gauge by the brute-force HA search (eq. HA24, ``gauge.solve_gauge``).
5. Stage matrices, each symmetrised as (X + X^T)/2 (they are symmetric in
   exact arithmetic; the asymmetry is recorded).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import gauge
from .symplectic import blocks, residual


class NoDecomposition(ValueError):
    pass


class NotSymplectic(ValueError):
    pass


@dataclass
class Plan:
    """Stage matrices of one NsDLCT, in formula order (leftmost first).

    typ 1: mats = (P1, B', P3, H)     -> CM(P1) CC(B') CM(P3) CC(H)
    typ 2: mats = (H1, Q1, B1', Q3)   -> CC(H1) CM(Q1) CC(B1') CM(Q3)
    typ 0: mats = (C,)                -> CM(C)     (B = 0, A = D = I)
    """
    typ: int
    mats: tuple
    Nx: int
    Ny: int
    dx: float
    dy: float
    h: np.ndarray | None = None
    f: float = math.nan
    asym: float = 0.0
    M: np.ndarray | None = field(default=None, repr=False)

    @property
    def dwx(self):
        return 2.0 * math.pi / (self.Nx * self.dx)

    @property
    def dwy(self):
        return 2.0 * math.pi / (self.Ny * self.dy)


def _symm(X):
    X = np.asarray(X, dtype=np.float64)
    return 0.5 * (X + X.T)


def plan_from_stages(typ: int, mats, Nx: int, Ny: int, dx: float, dy: float) -> Plan:
    """A plan at injected stage matrices (used for fixed-stage parity)."""
    return Plan(typ, tuple(_symm(X) for X in mats), Nx, Ny, dx, dy)


def plan(M, Nx: int, Ny: int, dx: float = 1.0, dy: float = 1.0, typ: int | None = None,
         tol: float = 1e-9) -> Plan:
    M = np.asarray(M, dtype=np.float64)
    r = residual(M)
    if r > tol:
        raise NotSymplectic(f"M J M^T - J residual {r:.3e} > {tol:.1e}")
    A, B, C, D = blocks(M)
    if np.max(np.abs(B)) < 1e-12:
        if np.max(np.abs(A - np.eye(2))) < 1e-12 and np.max(np.abs(D - np.eye(2))) < 1e-12:
            return Plan(0, (_symm(C),), Nx, Ny, dx, dy, M=M)
        raise NoDecomposition("B = 0 with A, D != I is an affine map (not supported)")
    t = gauge.trace_type(M) if typ is None else typ
    res = gauge.solve_gauge(M, t)
    if typ is None and not res.feasible:
        t = 3 - t
        res = gauge.solve_gauge(M, t)
    if not res.feasible or res.h is None or not math.isfinite(res.f):
        raise NoDecomposition("no symmetric gauge with invertible middle CC matrix")
    mats, _ = gauge.stage_matrices(M, t, res.h)
    asym = max(float(np.max(np.abs(X - X.T))) for X in mats)
    return Plan(t, tuple(_symm(X) for X in mats), Nx, Ny, dx, dy, h=res.h, f=res.f,
                asym=asym, M=M)
