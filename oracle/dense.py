"""The HA-NsDLCT as one dense N^2 x N^2 matrix (oracle; test infrastructure only).

Sec. 6.2 (eq. self12) writes the type-1 chain as L = O_CM F^dag O_CM F O_CM
F^dag O_CM F with F the Kronecker product of two 1D DFT matrices and the CMs
diagonal.  Its printed form drops the minus signs of the CC chirps and writes
F^dag for the IDFT; here the signs and constants of eq. HA28 are used, so L
is built from: diagonal CM matrices (eq. BasicCM12), F = dx dy/(j 2 pi)
kron(Wx, Wy) and F^-1 = dwx dwy/(j 2 pi) kron(conj Wx, conj Wy) acting on the
row-major vectorisation g[m, n] -> index m*Ny + n.  The literal Kronecker
products make this an O(N^4) brute force independent of the separable
matrix products in ``ops``.
"""
from __future__ import annotations

import math

import numpy as np

from .plan import Plan


def _w(N, sign):
    k = np.arange(N) - N // 2
    return np.exp(sign * 2j * math.pi * np.mod(np.outer(k, k), N) / N)


def _cm_diag(P, Nx, Ny, du, dv):
    m = (np.arange(Nx) - Nx // 2).astype(np.float64)
    n = (np.arange(Ny) - Ny // 2).astype(np.float64)
    mm, nn = np.meshgrid(m, n, indexing="ij")
    phi = 0.5 * (P[0, 0] * (mm * du) ** 2 + 2 * P[0, 1] * (mm * du) * (nn * dv)
                 + P[1, 1] * (nn * dv) ** 2)
    return np.exp(1j * phi.ravel())


def operator(p: Plan) -> np.ndarray:
    """Dense matrix L with vec(G) = L vec(g) (forward transform of plan p)."""
    Nx, Ny, dx, dy = p.Nx, p.Ny, p.dx, p.dy
    dwx, dwy = p.dwx, p.dwy
    F = (dx * dy / (2j * math.pi)) * np.kron(_w(Nx, -1), _w(Ny, -1))
    Fi = (dwx * dwy / (2j * math.pi)) * np.kron(_w(Nx, +1), _w(Ny, +1))

    def CMs(P):
        return np.diag(_cm_diag(P, Nx, Ny, dx, dy))

    def CMw(P):
        return np.diag(_cm_diag(P, Nx, Ny, dwx, dwy))

    if p.typ == 0:
        return CMs(p.mats[0])
    if p.typ == 1:
        P1, Bp, P3, H = p.mats
        return CMs(P1) @ Fi @ CMw(-Bp) @ F @ CMs(P3) @ Fi @ CMw(-H) @ F
    H1, Q1, B1p, Q3 = p.mats
    return Fi @ CMw(-H1) @ F @ CMs(Q1) @ Fi @ CMw(-B1p) @ F @ CMs(Q3)


def apply_sequential(p: Plan, g) -> np.ndarray:
    """Apply the same dense factors one matrix-vector product at a time.

    Identical arithmetic content to ``operator(p) @ vec(g)`` without forming
    the product, so N = 64 (4096 x 4096 factors) stays affordable.
    """
    Nx, Ny, dx, dy = p.Nx, p.Ny, p.dx, p.dy
    dwx, dwy = p.dwx, p.dwy
    F = (dx * dy / (2j * math.pi)) * np.kron(_w(Nx, -1), _w(Ny, -1))
    Fi = (dwx * dwy / (2j * math.pi)) * np.kron(_w(Nx, +1), _w(Ny, +1))
    v = np.asarray(g, dtype=np.complex128).ravel()

    def cms(P, v):
        return _cm_diag(P, Nx, Ny, dx, dy) * v

    def cmw(P, v):
        return _cm_diag(P, Nx, Ny, dwx, dwy) * v

    if p.typ == 0:
        v = cms(p.mats[0], v)
    elif p.typ == 1:
        P1, Bp, P3, H = p.mats
        v = Fi @ cmw(-H, F @ v)
        v = cms(P3, v)
        v = Fi @ cmw(-Bp, F @ v)
        v = cms(P1, v)
    else:
        H1, Q1, B1p, Q3 = p.mats
        v = cms(Q3, v)
        v = Fi @ cmw(-B1p, F @ v)
        v = cms(Q1, v)
        v = Fi @ cmw(-H1, F @ v)
    return v.reshape(Nx, Ny)
