"""ABCD-matrix helpers (oracle; test infrastructure only).

A valid 2D NsLCT matrix M = (A, B; C, D) satisfies A B^T = B A^T,
C D^T = D C^T, A D^T - B C^T = I (Sec. 1, eq. Intro12), i.e. M J M^T = J with
J = (0, I; -I, 0).  Its inverse is (D^T, -B^T; -C^T, A^T) (Sec. 4.3,
eq. CCCMCCCM20).
"""
from __future__ import annotations

import numpy as np

J4 = np.block([[np.zeros((2, 2)), np.eye(2)], [-np.eye(2), np.zeros((2, 2))]])


def blocks(M):
    """Split a 4x4 ABCD matrix into its 2x2 blocks A, B, C, D."""
    M = np.asarray(M, dtype=np.float64)
    return M[:2, :2], M[:2, 2:], M[2:, :2], M[2:, 2:]


def residual(M) -> float:
    """max |M J M^T - J| (zero for an exactly symplectic matrix)."""
    M = np.asarray(M, dtype=np.float64)
    return float(np.max(np.abs(M @ J4 @ M.T - J4)))


def constraint_residual(M) -> float:
    """Largest violation of the three block constraints of eq. Intro12."""
    A, B, C, D = blocks(M)
    r1 = A @ B.T - B @ A.T
    r2 = C @ D.T - D @ C.T
    r3 = A @ D.T - B @ C.T - np.eye(2)
    return float(max(np.max(np.abs(r1)), np.max(np.abs(r2)), np.max(np.abs(r3))))


def project(M, steps: int = 6):
    """Nearest-symplectic correction of a matrix printed to a few decimals.

    Newton-type step M <- M + 1/2 (M J M^T - J) J M, repeated: with
    E = M J M^T - J small, the corrected matrix has residual O(|E|^2).  The
    matrices printed in Sec. 5 satisfy eq. Intro12 only to their 4 decimals,
    so they are projected before use.
    """
    M = np.array(M, dtype=np.float64)
    for _ in range(steps):
        E = M @ J4 @ M.T - J4
        if np.max(np.abs(E)) < 1e-16:
            break
        M = M + 0.5 * E @ J4 @ M
    return M


def inverse(M):
    """(A, B; C, D)^-1 = (D^T, -B^T; -C^T, A^T) (eq. CCCMCCCM20)."""
    A, B, C, D = blocks(M)
    return np.block([[D.T, -B.T], [-C.T, A.T]])


def compose(*Ms):
    """Matrix product M_1 M_2 ... (the ABCD matrix of applying the last first)."""
    out = np.eye(4)
    for M in Ms:
        out = out @ np.asarray(M, dtype=np.float64)
    return out
