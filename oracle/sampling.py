"""Phase-space growth predicate (oracle; test infrastructure only).

Sec. 4.2.1 explains the HA gauge through the shears each stage applies to a
signal's space / spatial-frequency support: a CM with matrix C adds C z to
the frequencies (eq. HA12), a CC with matrix B adds B omega to the positions
(eq. HA20), and too large a support causes overlap and aliasing.  The paper
gives no numeric sampling condition; the reading used here:

* an N-point axis with spacing d holds positions |x| <= N d / 2 and
  frequencies |omega| <= pi / d;
* the input occupies the central half of both: |x| <= N d / 4,
  |omega| <= pi / (2 d);
* the box is pushed through the four stages in application order with
  per-axis interval arithmetic (the row sums that define gamma, eq. HA16);
* the transform is "well sampled" when the box stays inside the grid after
  every stage.
"""
from __future__ import annotations

import math

import numpy as np

from .plan import Plan


def _cm(box, P):
    X, Y, Wx, Wy = box
    return (X, Y, Wx + abs(P[0, 0]) * X + abs(P[0, 1]) * Y, Wy + abs(P[0, 1]) * X + abs(P[1, 1]) * Y)


def _cc(box, B):
    X, Y, Wx, Wy = box
    return (X + abs(B[0, 0]) * Wx + abs(B[0, 1]) * Wy, Y + abs(B[0, 1]) * Wx + abs(B[1, 1]) * Wy, Wx, Wy)


def stage_boxes(p: Plan):
    """Support box (X, Y, Wx, Wy) after each stage, in application order."""
    box = (p.Nx * p.dx / 4.0, p.Ny * p.dy / 4.0, math.pi / (2 * p.dx), math.pi / (2 * p.dy))
    out = []
    if p.typ == 0:
        return [_cm(box, p.mats[0])]
    if p.typ == 1:
        P1, Bp, P3, H = p.mats
        seq = [(_cc, H), (_cm, P3), (_cc, Bp), (_cm, P1)]
    else:
        H1, Q1, B1p, Q3 = p.mats
        seq = [(_cm, Q3), (_cc, B1p), (_cm, Q1), (_cc, H1)]
    for fn, X in seq:
        box = fn(box, np.asarray(X))
        out.append(box)
    return out


def well_sampled(p: Plan) -> bool:
    lim = (p.Nx * p.dx / 2.0, p.Ny * p.dy / 2.0, math.pi / p.dx, math.pi / p.dy)
    return all(all(b <= l * (1 + 1e-12) for b, l in zip(box, lim)) for box in stage_boxes(p))
