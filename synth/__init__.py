"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input generators only: random images, the Hermite-Gaussian
test signals of the accuracy experiments (Sec. 5.1, eqs. Acc12-Acc20), and
random symplectic ABCD matrices.  It contains none of the transform's own
arithmetic (no chirps, no DFTs, no gauge solving), so both the FP64 oracle and
the GPU path can draw their inputs from here without sharing method code.

Every generator is a pure function of its arguments and a numpy seed.
"""
from __future__ import annotations

import math
from typing import Iterator

import numpy as np

__all__ = [
    "complex_normal",
    "random_phase_field",
    "hermite_gaussian_1d",
    "hg_signal",
    "symplectic_candidates",
    "symplectic_from_params",
    "batch_sizes",
    "PAPER_SIZES",
]

# Image sides of the ragged batched workload: 128..1024, two of them with a
# factor 3.
PAPER_SIZES = (128, 256, 384, 512, 768, 1024)


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Image whose real and imaginary parts are i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(dtype)


def random_phase_field(N: int, delta: float, seed: int, corr_px: float = 8.0,
                       dtype=np.complex128) -> np.ndarray:
    """Smooth Gaussian-windowed random-phase field on a centred N x N grid.

    ``exp(-(x^2+y^2)/(2 s^2)) * exp(j*phi)`` with ``s = N*delta/8`` and ``phi``
    a unit-variance Gaussian random field of correlation length ``corr_px``
    pixels, scaled to 2*pi.  The smoothing is a separable Gaussian blur done by
    circular convolution (input preparation, not part of the transform).
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((N, N))
    k = np.fft.fftfreq(N)
    # Gaussian low-pass with std corr_px pixels in space.
    filt = np.exp(-0.5 * (2 * np.pi * k * corr_px) ** 2)
    w = np.real(np.fft.ifft2(np.fft.fft2(w) * filt[:, None] * filt[None, :]))
    w = (w - w.mean()) / w.std()
    m = (np.arange(N) - N // 2) * delta
    s = N * delta / 8.0
    env = np.exp(-(m[:, None] ** 2 + m[None, :] ** 2) / (2 * s * s))
    return (env * np.exp(2j * np.pi * w)).astype(dtype)


def hermite_gaussian_1d(k: int, x: np.ndarray) -> np.ndarray:
    """Normalised 1D Hermite-Gaussian HG_k(x) of Sec. 5.1 (eq. Acc12).

    HG_k(x) = (2^k k! sqrt(pi))^(-1/2) exp(-x^2/2) H_k(x) with physicists'
    Hermite polynomials, evaluated through the stable three-term recurrence of
    the normalised functions psi_{k+1} = sqrt(2/(k+1)) x psi_k
    - sqrt(k/(k+1)) psi_{k-1}, which never forms the large H_k(x) or k!.
    """
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.zeros_like(x)
    p = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    for j in range(k):
        p_next = math.sqrt(2.0 / (j + 1)) * x * p - math.sqrt(j / (j + 1)) * p_prev
        p_prev, p = p, p_next
    return p


def hg_signal(orders, N: int, delta: float, offset=None) -> np.ndarray:
    """Sum of separable 2D Hermite-Gaussians HG_{k,l}(x, y) (eqs. Acc16, Acc20).

    ``orders`` is a list of (k, l); the grid is centred, x_m = (m - N//2)*delta.
    The first signal of the accuracy experiments is orders [(1,2),(3,1)] on
    100 x 100 at delta 0.25, the second [(2,18),(14,11)] on 165 x 165 at 0.2.
    """
    m = (np.arange(N) - N // 2) * delta
    if offset is not None:
        m = m + offset
    g = np.zeros((N, N), dtype=np.complex128)
    for k, l in orders:
        g += np.outer(hermite_gaussian_1d(k, m), hermite_gaussian_1d(l, m))
    return g


def _rot(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def symplectic_from_params(S1, lam, theta: float, phi: float) -> np.ndarray:
    """ABCD = L(S1) . diag(Lambda, Lambda^-T) . Rot(theta) . Gyr(phi).

    L(S1) = (I, 0; S1, I) with S1 symmetric; Lambda = diag(lam);
    Rot = (R, 0; 0, R) with R the plane rotation; Gyr(phi) =
    (cos(phi) I, sin(phi) S; -sin(phi) S, cos(phi) I) with S = (0,1;1,0).
    Each factor satisfies M J M^T = J, so the product does too.
    """
    I2 = np.eye(2)
    Z = np.zeros((2, 2))
    S1 = np.asarray(S1, dtype=np.float64)
    L = np.block([[I2, Z], [S1, I2]])
    Lam = np.diag(np.asarray(lam, dtype=np.float64))
    Dg = np.block([[Lam, Z], [Z, np.linalg.inv(Lam)]])
    R = _rot(theta)
    Rt = np.block([[R, Z], [Z, R]])
    Sg = np.array([[0.0, 1.0], [1.0, 0.0]])
    c, s = math.cos(phi), math.sin(phi)
    G = np.block([[c * I2, s * Sg], [-s * Sg, c * I2]])
    return L @ Dg @ Rt @ G


def symplectic_candidates(seed: int, s1_std: float = 0.5,
                          lam_range=(0.7, 1.4)) -> Iterator[np.ndarray]:
    """Endless stream of seeded random symplectic ABCD candidates.

    S1 has i.i.d. N(0, s1_std^2) entries (s11, s12, s22), Lambda is uniform on
    ``lam_range``, theta and phi uniform on [0, pi).  Callers apply their own
    acceptance test (invertible B, sampling conditions) and take the first
    candidate that passes; the index of that candidate is part of the recipe.
    """
    rng = np.random.default_rng(seed)
    while True:
        s = rng.normal(0.0, s1_std, size=3)
        S1 = np.array([[s[0], s[1]], [s[1], s[2]]])
        lam = rng.uniform(lam_range[0], lam_range[1], size=2)
        theta, phi = rng.uniform(0.0, np.pi, size=2)
        yield symplectic_from_params(S1, lam, theta, phi)


def batch_sizes(count: int, seed: int, sizes=PAPER_SIZES) -> list:
    """Square image sides drawn uniformly from ``sizes`` (ragged batches)."""
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.choice(np.asarray(sizes), size=count)]
