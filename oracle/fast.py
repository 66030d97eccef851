"""Reduced decompositions of the NsDLCT (oracle; test infrastructure only).

* CM-CC-CM (Sec. 4.1, eqs. Bsym04-Bsym12), valid when B is symmetric and
  invertible:  G = CM((D - I) B^-1) CC(B) CM(B^-1 (A - I)) g.
* LC-NsDLCT (Sec. 4.2.2, eqs. LC04-LC12): the CM-CC-CM-CC form of eq. HA28
  with a rank-one gauge H = (h, 0; 0, 0) (h from eq. LC08, needs a21 != 0) or
  H = (0, 0; 0, h) (eq. LC10, needs a12 != 0), so that the last CC acts
  along one axis only:
      G = CM(P1) CC(B') CM(P3) F_a^-1 CM_a(-h) F_a g,
  B' = B - A H, D' = D - C H, P1 = (D' - I) B'^-1, P3 = B'^-1 (A - I).
  When both forms exist the one with the smaller eq. HA24 objective is used.

Readings (the paper does not write these out):

* The 1D DFT / IDFT along one axis carry the constants that make them the
  factors of the unitary centred DFT scaled to the continuous Fourier
  transform with kernel exp(-j w x) / sqrt(2 pi): F_a = da / sqrt(2 pi) sum
  exp(-j 2 pi k m / N), F_a^-1 = dw / sqrt(2 pi) sum exp(+j 2 pi k m / N), so
  F_a^-1 F_a = I and a 1D CC with h = 0 is the identity, as the continuous
  chirp convolution with kernel matrix (1, 0; 0, 1) is.
* A single 2D CC with the paper's constants (eqs. BasicDFT16/20) equals
  -U^H CM U; the HA chain has two of them and its overall constant is +1.
  The CM-CC-CM and LC chains have one 2D CC: taken literally they are the
  negative of the continuous transform (checked against the closed-form
  NsLCT of a Gaussian).  Reading: their overall constant is +1 like the HA
  chain's, i.e. the 2D CC inside them is used as U^H CM U.  ``literal=True``
  keeps the paper's sign for the pin that documents this.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import gauge
from .ops import cc, cm, centered, dft_kernel, freq_spacing
from .symplectic import blocks


class NotApplicable(ValueError):
    pass


@dataclass
class FastPlan:
    """kind 'cmccm': mats = (P1, B, P3);  kind 'lc': mats = (P1, B', P3, H),
    axis 0 (H = (h,0;0,0), x) or 1 (H = (0,0;0,h), y)."""
    kind: str
    mats: tuple
    Nx: int
    Ny: int
    dx: float
    dy: float
    axis: int = -1
    h: float = 0.0
    f: float = math.nan


def _symm(X):
    X = np.asarray(X, dtype=np.float64)
    return 0.5 * (X + X.T)


def cmccm_plan(M, Nx, Ny, dx, dy, tol=1e-9) -> FastPlan:
    """Stage matrices of eq. Bsym04 (requires eq. Bsym08)."""
    A, B, C, D = blocks(np.asarray(M, dtype=np.float64))
    scale = max(1.0, float(np.max(np.abs(B))))
    if np.max(np.abs(B - B.T)) > tol * scale:
        raise NotApplicable("CM-CC-CM needs a symmetric B")
    if abs(np.linalg.det(B)) < gauge.det_bound(M):
        raise NotApplicable("CM-CC-CM needs an invertible B")
    Bi = np.linalg.inv(B)
    I2 = np.eye(2)
    return FastPlan("cmccm", (_symm((D - I2) @ Bi), _symm(B), _symm(Bi @ (A - I2))), Nx, Ny, dx, dy)


def lc_candidates(M):
    """(axis, h, stage matrices) of every valid rank-one gauge (eqs. LC08, LC10)."""
    A, B, C, D = blocks(np.asarray(M, dtype=np.float64))
    I2 = np.eye(2)
    out = []
    for axis in (0, 1):
        a = A[1, 0] if axis == 0 else A[0, 1]
        if abs(a) < 1e-12:
            continue
        h = (B[1, 0] - B[0, 1]) / a if axis == 0 else (B[0, 1] - B[1, 0]) / a
        H = np.zeros((2, 2))
        H[axis, axis] = h
        Bp = B - A @ H
        if abs(np.linalg.det(Bp)) < gauge.det_bound(M):
            continue
        Dp = D - C @ H
        Bpi = np.linalg.inv(Bp)
        mats = (_symm((Dp - I2) @ Bpi), _symm(Bp), _symm(Bpi @ (A - I2)), H)
        f = gauge.gamma(mats[0]) * gauge.gamma(mats[1]) * gauge.gamma(mats[2]) * gauge.gamma(H)
        out.append((axis, h, mats, f))
    return out


def lc_plan(M, Nx, Ny, dx, dy, axis=None) -> FastPlan:
    cands = lc_candidates(M)
    if axis is not None:
        cands = [c for c in cands if c[0] == axis]
    if not cands:
        raise NotApplicable("no rank-one gauge with invertible B'")
    axis, h, mats, f = min(cands, key=lambda c: (c[3], c[0]))
    return FastPlan("lc", mats, Nx, Ny, dx, dy, axis=axis, h=h, f=f)


def dft1(g, axis: int, delta: float, sign: int) -> np.ndarray:
    """1D DFT (sign -1) or IDFT (+1) along ``axis`` with constant delta / sqrt(2 pi)."""
    g = np.asarray(g, dtype=np.complex128)
    W = dft_kernel(g.shape[axis], sign) * (delta / math.sqrt(2 * math.pi))
    return W @ g if axis == 0 else g @ W.T


def cc1(g, h: float, axis: int, dx: float, dy: float) -> np.ndarray:
    """1D chirp convolution along ``axis``: F_a^-1 CM_a(-h) F_a."""
    g = np.asarray(g, dtype=np.complex128)
    N = g.shape[axis]
    d = dx if axis == 0 else dy
    dw = freq_spacing(N, d)
    X = dft1(g, axis, d, -1)
    k = centered(N).astype(np.float64)
    phi = np.remainder(0.5 * (-h) * dw * dw * (k * k) + math.pi, 2 * math.pi) - math.pi
    ph = np.exp(1j * phi)
    X = X * (ph[:, None] if axis == 0 else ph[None, :])
    return dft1(X, axis, dw, +1)


def forward(p: FastPlan, g, literal: bool = False) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    sgn = 1.0 if literal else -1.0
    if p.kind == "cmccm":
        P1, B, P3 = p.mats
        x = cm(g, P3, p.dx, p.dy)
        x = cc(x, B, p.dx, p.dy)
        return sgn * cm(x, P1, p.dx, p.dy)
    P1, Bp, P3, H = p.mats
    x = cc1(g, p.h, p.axis, p.dx, p.dy)
    x = cm(x, P3, p.dx, p.dy)
    x = cc(x, Bp, p.dx, p.dy)
    return sgn * cm(x, P1, p.dx, p.dy)


def inverse(p: FastPlan, G) -> np.ndarray:
    """Reversed chain with negated stage matrices (as eq. CCCMCCCM30 does for HA)."""
    G = np.asarray(G, dtype=np.complex128)
    if p.kind == "cmccm":
        P1, B, P3 = p.mats
        x = cm(G, -P1, p.dx, p.dy)
        x = cc(x, -B, p.dx, p.dy)
        return -cm(x, -P3, p.dx, p.dy)
    P1, Bp, P3, H = p.mats
    x = cm(G, -P1, p.dx, p.dy)
    x = cc(x, -Bp, p.dx, p.dy)
    x = cm(x, -P3, p.dx, p.dy)
    return -cc1(x, -p.h, p.axis, p.dx, p.dy)
