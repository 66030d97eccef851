"""Basic 2D discrete operations of Sec. 2 (oracle; test infrastructure only).

Conventions (readings where the paper is silent):

* Index ranges: an N-point axis uses the centred signed indices
  m = -floor(N/2), ..., ceil(N/2)-1, so x_m = m*dx and the chirps and the
  Hermite-Gaussian inputs are centred on the origin.
* Grids: a DFT maps spacing dx to the frequency spacing dw = 2*pi/(N*dx)
  (the DFT condition of Sec. 2.2); the CM inside a CC is sampled on that
  frequency grid; the IDFT maps dw back to dx.
* Arrays are [Nx, Ny]: element [m, n] is g(x_m, y_n).

All phases are formed from exact integer products (m*m, m*n) times float64
coefficients and reduced modulo 2*pi before the complex exponential.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def centered(N: int) -> np.ndarray:
    """Centred signed sample indices -floor(N/2) .. ceil(N/2)-1 (int64)."""
    return np.arange(N, dtype=np.int64) - N // 2


def freq_spacing(N: int, delta: float) -> float:
    """Output spacing of an N-point DFT on spacing ``delta`` (Sec. 2.2)."""
    return TWO_PI / (N * delta)


def chirp_phase(P, Nx: int, Ny: int, du: float, dv: float) -> np.ndarray:
    """Phase of the discrete CM kernel of eq. BasicCM12.

    phi[p, q] = 1/2 (c11 p^2 du^2 + 2 c12 p q du dv + c22 q^2 dv^2) with
    P = (c11, c12; c12, c22) symmetric and p, q centred indices.
    """
    P = np.asarray(P, dtype=np.float64)
    p = centered(Nx)[:, None]
    q = centered(Ny)[None, :]
    pp = (p * p).astype(np.float64)          # exact integers
    pq = (p * q).astype(np.float64)
    qq = (q * q).astype(np.float64)
    c12 = 0.5 * (P[0, 1] + P[1, 0])
    return 0.5 * (P[0, 0] * du * du) * pp + (c12 * du * dv) * pq \
        + 0.5 * (P[1, 1] * dv * dv) * qq


def cm(g, P, du: float, dv: float) -> np.ndarray:
    """2D discrete chirp multiplication O_CM^P (Sec. 2.1, eq. BasicCM12)."""
    g = np.asarray(g, dtype=np.complex128)
    phi = chirp_phase(P, g.shape[0], g.shape[1], du, dv)
    phi = np.remainder(phi + math.pi, TWO_PI) - math.pi
    return np.exp(1j * phi) * g


def dft_kernel(N: int, sign: int) -> np.ndarray:
    """Unnormalised N x N kernel exp(sign * j 2 pi k m / N), centred k, m.

    The exponent is taken from the exact integer residue (k*m) mod N, so the
    matrix entries carry no argument-rounding error.
    """
    k = centered(N)
    r = np.mod(np.outer(k, k), N).astype(np.float64)
    return np.exp(sign * 2j * math.pi * r / N)


def dft2(g, dx: float, dy: float) -> np.ndarray:
    """2D DFT F_{x,y} (Sec. 2.2, eq. BasicDFT16).

    G[p,q] = dx dy / (j 2 pi) * sum_{m,n} exp(-j 2 pi (p m / Nx + q n / Ny)) g[m,n],
    written as the two dense matrix products Wx g Wy^T.
    """
    g = np.asarray(g, dtype=np.complex128)
    Wx = dft_kernel(g.shape[0], -1)
    Wy = dft_kernel(g.shape[1], -1)
    return (dx * dy / (2j * math.pi)) * (Wx @ g @ Wy.T)


def idft2(G, dwx: float, dwy: float) -> np.ndarray:
    """2D IDFT F^-1_{x,y} (Sec. 2.2, eq. BasicDFT20), input spacing dwx, dwy.

    Same constant form as the DFT with the opposite exponent sign; its input
    grid is the frequency grid, so the constant is dwx dwy / (j 2 pi).
    """
    G = np.asarray(G, dtype=np.complex128)
    Wx = dft_kernel(G.shape[0], +1)
    Wy = dft_kernel(G.shape[1], +1)
    return (dwx * dwy / (2j * math.pi)) * (Wx @ G @ Wy.T)


def cc(g, B, dx: float, dy: float) -> np.ndarray:
    """2D discrete chirp convolution O_CC^B = F^-1 O_CM^{-B} F (eq. BasicCC20).

    The CM with matrix -B acts on the DFT's output (frequency) grid.
    """
    g = np.asarray(g, dtype=np.complex128)
    Nx, Ny = g.shape
    dwx, dwy = freq_spacing(Nx, dx), freq_spacing(Ny, dy)
    X = dft2(g, dx, dy)
    X = cm(X, -np.asarray(B, dtype=np.float64), dwx, dwy)
    return idft2(X, dwx, dwy)
