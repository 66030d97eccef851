"""The decomposition (A, B; C, D) = (-B, A; -D, C)(0, -I; I, 0) of Sec. 4.2.2
for a12 = a21 = 0 (oracle; test infrastructure only).

When a12 = a21 = 0 neither rank-one gauge of the LC-NsDLCT exists (eqs.
LC08, LC10); the paper then factors M into the inverse Fourier transform
matrix (0, -I; I, 0) followed by M' = (-B, A; -D, C), whose B-block A is
symmetric (diagonal), so that M' has the CM-CC-CM decomposition of eq.
Bsym04 when A is invertible (eq. Bsym08).  The transform is the IDFT of eq.
BasicDFT20 followed by the CM-CC-CM chain of M' (eq. Bsym12):

    G = kappa CM((C - I) A^-1) CC(A) CM(A^-1 (-B - I)) F^-1 g,

with the paper's F^-1 (constant dw dw / (j 2 pi)) and CC (eq. BasicCC20).

Readings (the paper writes neither):

* Grid.  F^-1 maps an input spacing d to 2 pi / (N d) (Sec. 2.2); the
  route keeps the grid of the other chains (output spacing = input spacing)
  only at d = sqrt(2 pi / N) on each axis, which it requires.
* Overall constant kappa.  Operators of the same ABCD matrix built from
  different factorisations can differ by a constant (a sign for two
  factorisations of one matrix into chirps and Fresnel-type factors: the
  metaplectic ambiguity), and the paper fixes none.  kappa makes the route
  the same operator as the HA chain of M (the reference of this library).
  Both are applied in closed form to a Gaussian exp(-1/2 z^T S z), Re S > 0:
  a CM with matrix P maps S -> S - jP; a CC whose transfer function is
  exp(-j/2 w^T B w) between unitary Fourier transforms multiplies the
  amplitude by det(I + j S B)^(-1/2), the root continued from B = 0 along
  t B, t in [0, 1], and maps S -> (S^-1 + j B)^-1; the paper's F^-1 of a
  Gaussian is -j det(S)^(-1/2) exp(-1/2 w^T S^-1 w) (root continued from
  S = I), and its CC is -1 times the unitary one (eq. BasicCC20 with the
  constants of eqs. BasicDFT16/20).  Both chains reach the same Gaussian
  (same M); kappa is the ratio of their amplitudes, a unit complex number.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import gauge
from .ops import cc, cm, dft2, freq_spacing, idft2
from .symplectic import blocks

TWO_PI = 2.0 * math.pi


class NotApplicable(ValueError):
    pass


@dataclass
class RoutePlan:
    mats: tuple       # (P1', A, P3') of M' = (-B, A; -D, C), eq. Bsym04
    kappa: complex
    Nx: int
    Ny: int
    dx: float
    dy: float


def _symm(X):
    X = np.asarray(X, dtype=np.float64)
    return 0.5 * (X + X.T)


def _root_along(fn, steps: int = 400) -> complex:
    """sqrt(det fn(t)) at t = 1, continued from fn(0) = I (det 1, root 1)."""
    prev = 1.0 + 0j
    for k in range(1, steps + 1):
        r = np.sqrt(complex(np.linalg.det(fn(k / steps))))
        if abs(r - prev) > abs(r + prev):
            r = -r
        prev = r
    return prev


def gaussian_amplitude(factors, S) -> tuple:
    """(amplitude, S) of the Gaussian exp(-1/2 z^T S z) after `factors`,
    applied first to last: ('cm', P), ('cc', B) (unitary, transfer function
    exp(-j/2 w^T B w)), ('cc_paper', B) (eq. BasicCC20: -1 times 'cc'),
    ('idft_paper', None) (eq. BasicDFT20: -j times the unitary inverse FT)."""
    a = 1.0 + 0j
    S = np.asarray(S, dtype=np.complex128)
    I2 = np.eye(2)
    for kind, X in factors:
        if kind == "cm":
            S = S - 1j * np.asarray(X, dtype=np.float64)
        elif kind in ("cc", "cc_paper"):
            B = np.asarray(X, dtype=np.float64)
            a = a / _root_along(lambda t: I2 + 1j * t * S @ B)
            S = np.linalg.inv(np.linalg.inv(S) + 1j * B)
            if kind == "cc_paper":
                a = -a
        elif kind == "idft_paper":
            S0 = S.copy()
            a = a * (-1j) / _root_along(lambda t: (1 - t) * I2 + t * S0)
            S = np.linalg.inv(S)
        else:
            raise ValueError(kind)
    return a, S


def ha_factors(p):
    """The HA chain of an oracle plan as ('cm' / 'cc') factors, first applied
    first (the chain's CCs are unitary: two paper CCs give +1, Sec. A3)."""
    if p.typ == 1:
        P1, Bp, P3, H = p.mats
        return [("cc", H), ("cm", P3), ("cc", Bp), ("cm", P1)]
    H1, Q1, B1, Q3 = p.mats
    return [("cm", Q3), ("cc", B1), ("cm", Q1), ("cc", H1)]


REF_S = np.array([[0.8, 0.15], [0.15, 1.3]])  # any S with Re S > 0


def route_plan(M, Nx: int, Ny: int, dx: float, dy: float, ha_plan) -> RoutePlan:
    """Stages of the route and its constant kappa against the HA plan of M."""
    M = np.asarray(M, dtype=np.float64)
    A, B, C, D = blocks(M)
    scale = max(1.0, float(np.max(np.abs(M))))
    if abs(A[0, 1]) > 1e-12 * scale or abs(A[1, 0]) > 1e-12 * scale:
        raise NotApplicable("the route is for a12 = a21 = 0")
    if abs(np.linalg.det(A)) < 1e-6 * max(1.0, float(np.max(np.abs(A)))) ** 2:
        raise NotApplicable("the route needs an invertible A (eq. Bsym08 for M')")
    for N, d in ((Nx, dx), (Ny, dy)):
        if abs(d * d * N / TWO_PI - 1.0) > 1e-12:
            raise NotApplicable("the route needs the spacing sqrt(2 pi / N) on each axis")
    I2 = np.eye(2)
    Ai = np.linalg.inv(A)
    mats = (_symm((C - I2) @ Ai), _symm(A), _symm(Ai @ (-B - I2)))
    a_ha, S_ha = gaussian_amplitude(ha_factors(ha_plan), REF_S)
    a_r, S_r = gaussian_amplitude([("idft_paper", None), ("cm", mats[2]), ("cc_paper", mats[1]),
                                   ("cm", mats[0])], REF_S)
    assert np.max(np.abs(S_ha - S_r)) <= 1e-8 * (1 + np.max(np.abs(S_ha))), "not the same matrix"
    return RoutePlan(mats, complex(a_ha / a_r), Nx, Ny, dx, dy)


def forward(p: RoutePlan, g) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    P1, A, P3 = p.mats
    dwx, dwy = freq_spacing(p.Nx, p.dx), freq_spacing(p.Ny, p.dy)
    x = idft2(g, dwx, dwy)           # eq. BasicDFT20 (output spacing = dx at this spacing)
    x = cm(x, P3, p.dx, p.dy)
    x = cc(x, A, p.dx, p.dy)
    return p.kappa * cm(x, P1, p.dx, p.dy)


def inverse(p: RoutePlan, G) -> np.ndarray:
    """The inverse of forward: F^-1 F = -I and CC(-A) CC(A) = I with the
    paper's constants, so F^-1 has the inverse -F."""
    G = np.asarray(G, dtype=np.complex128)
    P1, A, P3 = p.mats
    x = cm(G / p.kappa, -P1, p.dx, p.dy)
    x = cc(x, -A, p.dx, p.dy)
    x = cm(x, -P3, p.dx, p.dy)
    return -dft2(x, p.dx, p.dy)
