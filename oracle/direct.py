"""Reference values of the continuous 2D NsLCT (oracle; test infrastructure only).

* ``direct``: the direct method of eq. Intro32, the Riemann sum of the
  defining integral (eq. Intro08) sampled on the input grid,
      G[p,q] = dx dy / (2 pi sqrt(-det B)) sum_{m,n}
               exp(j/2 (r'^T D B^-1 r' - 2 r^T B^-1 r' + r^T B^-1 A r)) g[m,n],
  O(N_in^2 N_out^2), chunked over output points.
* ``gaussian_nslct``: the defining integral eq. Intro08 evaluated in closed
  form for a Gaussian input g(z) = exp(-1/2 z^T S z + beta^T z), S symmetric
  positive definite, beta complex.  With K = B^-1 A (symmetric) the integrand
  is exp(-1/2 z^T (S - jK) z + (beta - j B^-1 z')^T z) times the output chirp,
  and the standard Gaussian integral gives
      G(z') = exp(j/2 z'^T D B^-1 z') exp(1/2 b^T Q^-1 b)
              / (sqrt(-det B) sqrt(det Q)),   Q = S - jK, b = beta - j B^-1 z'.
  sqrt(det Q) is taken continuously from sqrt(det S) along S - j t K, which is
  the product of principal roots of the factors (1 - j lambda_i) with
  lambda_i the eigenvalues of S^-1/2 K S^-1/2.

sqrt(-det B) is real for det B < 0.  For det B > 0 it lies on the branch cut
of the principal root; both ``sign=+1`` and ``sign=-1`` choices of the
branch (+j and -j) are offered, and callers compare with both (the discrete
chain fixes an overall sign that the continuous definition leaves open).
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from .symplectic import blocks


def _sqrt_minus_det(B, sign: int = 1) -> complex:
    d = float(np.linalg.det(B))
    if d < 0:
        return complex(math.sqrt(-d))
    return sign * 1j * math.sqrt(d)


def direct(M, g, dx: float, dy: float, Nout_x: int, Nout_y: int, du: float, dv: float,
           sign: int = 1, chunk: int = 2048) -> np.ndarray:
    """Direct method eq. Intro32 from an input grid onto a centred output grid."""
    A, B, C, D = blocks(M)
    Bi = np.linalg.inv(B)
    DBi = D @ Bi
    BiA = Bi @ A
    g = np.asarray(g, dtype=np.complex128)
    Nx, Ny = g.shape
    xm = (np.arange(Nx) - Nx // 2) * dx
    yn = (np.arange(Ny) - Ny // 2) * dy
    X, Y = np.meshgrid(xm, yn, indexing="ij")
    X = X.ravel()
    Y = Y.ravel()
    gv = g.ravel()
    # Input chirp r^T B^-1 A r (independent of the output point).
    q_in = BiA[0, 0] * X * X + (BiA[0, 1] + BiA[1, 0]) * X * Y + BiA[1, 1] * Y * Y
    up = (np.arange(Nout_x) - Nout_x // 2) * du
    vq = (np.arange(Nout_y) - Nout_y // 2) * dv
    U, V = np.meshgrid(up, vq, indexing="ij")
    U = U.ravel()
    V = V.ravel()
    out = np.empty(U.shape[0], dtype=np.complex128)
    const = dx * dy / (2.0 * math.pi * _sqrt_minus_det(B, sign))
    for s in range(0, U.shape[0], chunk):
        u = U[s:s + chunk, None]
        v = V[s:s + chunk, None]
        q_out = DBi[0, 0] * u * u + (DBi[0, 1] + DBi[1, 0]) * u * v + DBi[1, 1] * v * v
        # r^T B^-1 r' = x (Bi11 u + Bi12 v) + y (Bi21 u + Bi22 v)
        cross = X[None, :] * (Bi[0, 0] * u + Bi[0, 1] * v) + Y[None, :] * (Bi[1, 0] * u + Bi[1, 1] * v)
        ph = 0.5 * (q_out - 2.0 * cross + q_in[None, :])
        out[s:s + chunk] = const * (np.exp(1j * ph) @ gv)
    return out.reshape(Nout_x, Nout_y)


def gaussian(S, beta, Nx: int, Ny: int, dx: float, dy: float) -> np.ndarray:
    """Samples of g(z) = exp(-1/2 z^T S z + beta^T z) on the centred grid."""
    S = np.asarray(S, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.complex128)
    x = (np.arange(Nx) - Nx // 2) * dx
    y = (np.arange(Ny) - Ny // 2) * dy
    X, Y = np.meshgrid(x, y, indexing="ij")
    q = S[0, 0] * X * X + (S[0, 1] + S[1, 0]) * X * Y + S[1, 1] * Y * Y
    return np.exp(-0.5 * q + beta[0] * X + beta[1] * Y)


def gaussian_nslct(M, S, beta, Nx: int, Ny: int, du: float, dv: float,
                   sign: int = 1) -> np.ndarray:
    """Closed-form NsLCT (eq. Intro08) of the Gaussian above, sampled on a grid."""
    A, B, C, D = blocks(M)
    S = np.asarray(S, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.complex128)
    Bi = np.linalg.inv(B)
    K = Bi @ A
    K = 0.5 * (K + K.T)
    Q = S - 1j * K
    Qi = np.linalg.inv(Q)
    # Continuous branch of sqrt(det Q).
    w, V = np.linalg.eigh(S)
    Sm = V @ np.diag(w ** -0.5) @ V.T
    lam = np.linalg.eigvalsh(Sm @ K @ Sm)
    sqrt_det_q = math.sqrt(float(np.prod(w)))
    for l_ in lam:
        sqrt_det_q *= cmath.sqrt(1.0 - 1j * l_)
    DBi = D @ Bi
    u = (np.arange(Nx) - Nx // 2) * du
    v = (np.arange(Ny) - Ny // 2) * dv
    U, V2 = np.meshgrid(u, v, indexing="ij")
    zp = np.stack([U.ravel(), V2.ravel()], axis=0)                 # (2, K)
    b = beta[:, None] - 1j * (Bi @ zp)                             # (2, K)
    quad = np.einsum("ik,ij,jk->k", b, Qi, b)
    out_chirp = np.einsum("ik,ij,jk->k", zp, DBi, zp)
    G = np.exp(0.5j * out_chirp + 0.5 * quad) / (_sqrt_minus_det(B, sign) * sqrt_det_q)
    return G.reshape(Nx, Ny)
