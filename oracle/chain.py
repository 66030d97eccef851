"""The HA-NsDLCT chains, step by step (oracle; test infrastructure only).

Type 1 (CM-CC-CM-CC, Sec. 4.2.1, eq. HA28), rightmost applied first:
    G = CM(P1) F^-1 CM(-B') F CM(P3) F^-1 CM(-H) F g
Type 2 (CC-CM-CC-CM, Sec. 4.3, eq. CCCMCCCM40):
    G = F^-1 CM(-H1) F CM(Q1) F^-1 CM(-B1') F CM(Q3) g
Inverse (eq. CCCMCCCM30): the reversed chain with every stage matrix negated,
    type 1: CC(-H) CM(-P3) CC(-B') CM(-P1),  type 2: CM(-Q3) CC(-B1') CM(-Q1) CC(-H1).

Each CC is evaluated as the paper defines it (eq. BasicCC20) with the paper's
DFT constants dx dy / (j 2 pi) (eqs. BasicDFT16/20); no normalisation is
folded or reordered.
"""
from __future__ import annotations

import numpy as np

from .ops import cc, cm
from .plan import Plan


def forward(p: Plan, g) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    assert g.shape == (p.Nx, p.Ny)
    dx, dy = p.dx, p.dy
    if p.typ == 0:
        return cm(g, p.mats[0], dx, dy)
    if p.typ == 1:
        P1, Bp, P3, H = p.mats
        x = cc(g, H, dx, dy)
        x = cm(x, P3, dx, dy)
        x = cc(x, Bp, dx, dy)
        return cm(x, P1, dx, dy)
    H1, Q1, B1p, Q3 = p.mats
    x = cm(g, Q3, dx, dy)
    x = cc(x, B1p, dx, dy)
    x = cm(x, Q1, dx, dy)
    return cc(x, H1, dx, dy)


def inverse(p: Plan, G) -> np.ndarray:
    G = np.asarray(G, dtype=np.complex128)
    assert G.shape == (p.Nx, p.Ny)
    dx, dy = p.dx, p.dy
    if p.typ == 0:
        return cm(G, -p.mats[0], dx, dy)
    if p.typ == 1:
        P1, Bp, P3, H = p.mats
        x = cm(G, -P1, dx, dy)
        x = cc(x, -Bp, dx, dy)
        x = cm(x, -P3, dx, dy)
        return cc(x, -H, dx, dy)
    H1, Q1, B1p, Q3 = p.mats
    x = cc(G, -H1, dx, dy)
    x = cm(x, -Q1, dx, dy)
    x = cc(x, -B1p, dx, dy)
    return cm(x, -Q3, dx, dy)


def forward_batch(p: Plan, g) -> np.ndarray:
    """forward() over a leading batch axis (one plan for every image)."""
    g = np.asarray(g, dtype=np.complex128)
    return np.stack([forward(p, x) for x in g.reshape(-1, p.Nx, p.Ny)]).reshape(g.shape)


def inverse_batch(p: Plan, G) -> np.ndarray:
    G = np.asarray(G, dtype=np.complex128)
    return np.stack([inverse(p, x) for x in G.reshape(-1, p.Nx, p.Ny)]).reshape(G.shape)


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 (the square is the NMSE of eqs. Acc04, Add16, Rev08)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
