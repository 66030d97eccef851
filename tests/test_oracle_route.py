"""Pins of the oracle's (-B, A; -D, C)(0, -I; I, 0) route (Sec. 4.2.2, the
decomposition for a12 = a21 = 0; ``oracle.route``).

* The Gaussian rule behind the route's constant kappa, factor by factor,
  against the oracle's discrete operators; and, as a finding about the HA
  chain itself, its sign against the continuous definition (eq. Intro08),
  which the same rule predicts.
* Against the oracle's HA chain of the same matrix on a smooth input, for
  matrices with either sign of det B: the same operator (reading: the route
  is the operator of the HA chain).
* kappa is a fourth root of unity; forward then inverse is the identity,
  the route is unitary; it refuses a12 != 0 and a spacing other than
  sqrt(2 pi / N).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import chain, direct, plan as oplan, route

GAUSS_S = np.array([[1.0, 0.2], [0.2, 1.5]])
GAUSS_BETA = np.array([0.3 + 0.4j, -0.2 - 0.1j])


def _blk(A, B, C, D):
    return np.block([[A, B], [C, D]])


def route_matrices(seed, count):
    """(I, 0; P, I) diag(A0, A0^-1) (I, Q; 0, I): a12 = a21 = 0 exactly, B = A0 Q
    not symmetric, C and D general; A0 diagonal with entries of either sign."""
    rng = np.random.default_rng(seed)
    Z, I2 = np.zeros((2, 2)), np.eye(2)
    out = []
    while len(out) < count:
        a = rng.uniform(0.5, 1.5, 2) * rng.choice([-1, 1], 2)
        A0 = np.diag(a)
        Q = rng.normal(0, 0.4, (2, 2))
        P = rng.normal(0, 0.4, (2, 2))
        Q, P = 0.5 * (Q + Q.T), 0.5 * (P + P.T)
        M = _blk(I2, Z, P, I2) @ _blk(A0, Z, Z, np.linalg.inv(A0)) @ _blk(I2, Q, Z, I2)
        if abs(np.linalg.det(M[:2, 2:])) > 0.02:
            out.append(M)
    return out


def _plans(M, N):
    d = math.sqrt(2 * math.pi / N)
    pha = oplan.plan(M, N, N, d, d)
    return d, pha, route.route_plan(M, N, N, d, d, pha)


def _sampled_gaussian(a, S, N, d):
    x = (np.arange(N) - N // 2) * d
    X, Y = np.meshgrid(x, x, indexing="ij")
    q = S[0, 0] * X * X + (S[0, 1] + S[1, 0]) * X * Y + S[1, 1] * Y * Y
    return a * np.exp(-0.5 * q)


def test_gaussian_amplitude_rule_matches_discrete_operators():
    """The closed-form Gaussian propagation behind kappa, factor by factor,
    against the oracle's discrete operators on a well-sampled Gaussian: CM
    (eq. BasicCM12), the unitary CC (two paper CCs, Sec. A3 reading), the
    paper's CC (eq. BasicCC20) and the paper's IDFT (eq. BasicDFT20)."""
    from oracle import ops
    N = 128
    d = math.sqrt(2 * math.pi / N)
    rng = np.random.default_rng(8)
    S0 = np.array([[0.9, 0.2], [0.2, 1.4]])
    g = _sampled_gaussian(1.0, S0, N, d)
    for _ in range(4):
        P = rng.normal(0, 0.5, (2, 2))
        P = 0.5 * (P + P.T)
        B = rng.normal(0, 0.5, (2, 2))
        B = 0.5 * (B + B.T)
        cases = [([("cm", P)], ops.cm(g, P, d, d)),
                 ([("cc_paper", B)], ops.cc(g, B, d, d)),
                 ([("cc", B)], -ops.cc(g, B, d, d)),
                 ([("idft_paper", None)], ops.idft2(g, ops.freq_spacing(N, d), ops.freq_spacing(N, d)))]
        for factors, disc in cases:
            a, S = route.gaussian_amplitude(factors, S0)
            assert chain.rel_l2(disc, _sampled_gaussian(a, S, N, d)) <= 1e-8, factors[0][0]


def test_ha_chain_sign_against_the_definition_is_the_rule():
    """Finding: the HA chain (constant +1, Sec. A3 reading) equals the
    closed-form continuous NsLCT of eq. Intro08 (root of -det B positive for
    det B < 0, +j sqrt(det B) for det B > 0) only up to a sign that depends
    on the matrix and its gauge; the Gaussian rule predicts that sign."""
    N = 128
    seen = set()
    for M in route_matrices(1, 16):
        d = math.sqrt(2 * math.pi / N)
        pha = oplan.plan(M, N, N, d, d)
        g = direct.gaussian(GAUSS_S, GAUSS_BETA, N, N, d, d)
        ref = direct.gaussian_nslct(M, GAUSS_S, GAUSS_BETA, N, N, d, d, sign=1)
        a_ha, _ = route.gaussian_amplitude(route.ha_factors(pha), route.REF_S)
        a_def = direct.gaussian_nslct(M, route.REF_S, np.zeros(2), 1, 1, d, d, sign=1)[0, 0]
        s = a_ha / a_def
        assert abs(abs(s) - 1) <= 1e-9 and min(abs(s - 1), abs(s + 1)) <= 1e-9
        assert chain.rel_l2(chain.forward(pha, g), np.sign(s.real) * ref) <= 1e-6
        seen.add(np.sign(s.real))
    assert seen == {1.0, -1.0}


def test_route_equals_ha_chain_with_either_sign_of_det_b():
    N = 96
    x = (np.arange(N) - N // 2) * math.sqrt(2 * math.pi / N)
    X, Y = np.meshgrid(x, x, indexing="ij")
    g = np.exp(-0.6 * X * X - 0.4 * Y * Y + 0.2j * X * Y + 0.3j * X)
    signs = set()
    for M in route_matrices(2, 24):
        d, pha, pr = _plans(M, N)
        G = route.forward(pr, g)
        H = chain.forward(pha, g)
        assert chain.rel_l2(G, H) <= 1e-3
        assert chain.rel_l2(G, -H) >= 1.9
        assert abs(pr.kappa ** 4 - 1) <= 1e-9
        signs.add((np.sign(np.linalg.det(M[:2, 2:])), pr.kappa.real > 0.5 or pr.kappa.imag > 0.5))
    assert len(signs) >= 3  # both signs of det B and both signs of kappa occur


def test_route_inverse_and_unitarity():
    N = 32
    rng = np.random.default_rng(3)
    g = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    for M in route_matrices(4, 4):
        _, _, pr = _plans(M, N)
        G = route.forward(pr, g)
        assert abs(np.linalg.norm(G) / np.linalg.norm(g) - 1) <= 1e-13
        assert chain.rel_l2(route.inverse(pr, G), g) <= 1e-13


def test_route_refuses():
    M = route_matrices(5, 1)[0]
    N = 32
    d, pha, _ = _plans(M, N)
    with pytest.raises(route.NotApplicable):
        route.route_plan(M, N, N, 1.1 * d, d, pha)
    R = np.array([[math.cos(0.3), -math.sin(0.3)], [math.sin(0.3), math.cos(0.3)]])
    Mr = _blk(R, np.zeros((2, 2)), np.zeros((2, 2)), R) @ M  # a12, a21 != 0
    with pytest.raises(route.NotApplicable):
        route.route_plan(Mr, N, N, d, d, oplan.plan(Mr, N, N, d, d))
