"""Pins of the oracle's reduced decompositions (CM-CC-CM, Sec. 4.1; LC-NsDLCT,
Sec. 4.2.2) against closed forms, the paper's DFT and invariants.

* The FT matrix (B = I symmetric) through CM-CC-CM gives the paper's 2D DFT
  (eq. BasicDFT16) exactly; the expected value is built with numpy.fft.
* CM-CC-CM and LC-NsDLCT of a Gaussian match the closed-form continuous
  NsLCT (eq. Intro08).  The same checks show that the literal one-2D-CC
  chains carry the constant -1 (the reading documented in ``oracle.fast``).
* The 1D CC along an axis is compared with a chirp filter built on
  numpy.fft, and with the identity at h = 0.
* Stage matrices multiply back to M (eqs. Bsym04, LC12 with HA decomposition
  identity); the chains are unitary and the inverse is the adjoint.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import chain, direct, fast

FT = np.block([[np.zeros((2, 2)), np.eye(2)], [-np.eye(2), np.zeros((2, 2))]])
GAUSS_S = np.array([[1.0, 0.2], [0.2, 1.5]])
GAUSS_BETA = np.array([0.3 + 0.4j, -0.2 - 0.1j])
I2, Z2 = np.eye(2), np.zeros((2, 2))


def _cm_mat(P):
    return np.block([[I2, Z2], [P, I2]])


def _cc_mat(B):
    return np.block([[I2, B], [Z2, I2]])


def _sym_draw(rng, s):
    X = rng.normal(size=(2, 2)) * s
    return 0.5 * (X + X.T)


def _cmccm_matrices(seed, count):
    """Symplectic matrices with a symmetric B, built as CM(P1) CC(B) CM(P3)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        P1, B, P3 = _sym_draw(rng, 0.5), _sym_draw(rng, 1.0), _sym_draw(rng, 0.5)
        if abs(np.linalg.det(B)) > 0.05:
            out.append(_cm_mat(P1) @ _cc_mat(B) @ _cm_mat(P3))
    return out


def _cfft(v, axis, inverse=False):
    f = np.fft.ifft if inverse else np.fft.fft
    return np.fft.fftshift(f(np.fft.ifftshift(v, axes=axis), axis=axis, norm="ortho"), axes=axis)


@pytest.mark.parametrize("N", [8, 16, 64])
def test_cmccm_ft_gives_the_paper_dft(N):
    d = math.sqrt(2 * math.pi / N)
    p = fast.cmccm_plan(FT, N, N, d, d)
    g = synth.complex_normal((N, N), seed=N)
    expect = (d * d / (2j * math.pi)) * N * _cfft(_cfft(g, 0), 1)
    got = fast.forward(p, g)
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))
    lit = fast.forward(p, g, literal=True)
    assert np.max(np.abs(lit + expect)) <= 1e-12 * np.max(np.abs(expect))


def test_cmccm_matches_closed_form_gaussian():
    N = 128
    d = math.sqrt(2 * math.pi / N)
    g = direct.gaussian(GAUSS_S, GAUSS_BETA, N, N, d, d)
    seen_pos = False
    for M in _cmccm_matrices(3, 5):
        p = fast.cmccm_plan(M, N, N, d, d)
        G = fast.forward(p, g)
        detB = np.linalg.det(M[:2, 2:])
        if detB < 0:
            ref = direct.gaussian_nslct(M, GAUSS_S, GAUSS_BETA, N, N, d, d)
            assert chain.rel_l2(G, ref) <= 1e-12
            assert chain.rel_l2(fast.forward(p, g, literal=True), -ref) <= 1e-12
        else:  # metaplectic sign ambiguity (det B > 0)
            seen_pos = True
            errs = [chain.rel_l2(G, direct.gaussian_nslct(M, GAUSS_S, GAUSS_BETA, N, N, d, d, sign=s))
                    for s in (1, -1)]
            assert min(errs) <= 1e-12
    assert seen_pos


def test_cmccm_rejects_nonsymmetric_b():
    M = next(synth.symplectic_candidates(7))
    assert np.max(np.abs(M[:2, 2:] - M[2:, 2:].T)) > 0
    with pytest.raises(fast.NotApplicable):
        fast.cmccm_plan(M, 16, 16, 1.0, 1.0)


def test_stage_matrices_multiply_back_to_m():
    for M in _cmccm_matrices(5, 3):
        P1, B, P3 = fast.cmccm_plan(M, 8, 8, 1.0, 1.0).mats
        assert np.max(np.abs(_cm_mat(P1) @ _cc_mat(B) @ _cm_mat(P3) - M)) <= 1e-12
    c = synth.symplectic_candidates(11)
    for _ in range(4):
        M = next(c)
        for axis, h, (P1, Bp, P3, H), f in fast.lc_candidates(M):
            assert H[axis, axis] == h and np.count_nonzero(H) <= 1
            assert np.max(np.abs(Bp - Bp.T)) <= 1e-12
            prod = _cm_mat(P1) @ _cc_mat(Bp) @ _cm_mat(P3) @ _cc_mat(H)
            assert np.max(np.abs(prod - M)) <= 1e-10 * max(1.0, np.max(np.abs(M)))


@pytest.mark.parametrize("axis", [0, 1])
def test_cc1_against_numpy_fft_chirp_filter(axis):
    Nx, Ny, dx, dy, h = 24, 32, 0.4, 0.3, 0.7
    g = synth.complex_normal((Nx, Ny), seed=5)
    N, dd = (Nx, dx) if axis == 0 else (Ny, dy)
    dw = 2 * math.pi / (N * dd)
    k = (np.arange(N) - N // 2) * dw
    tf = np.exp(-0.5j * h * k * k)
    tf = tf[:, None] if axis == 0 else tf[None, :]
    expect = _cfft(tf * _cfft(g, axis), axis, inverse=True)
    assert np.max(np.abs(fast.cc1(g, h, axis, dx, dy) - expect)) <= 1e-13
    assert np.max(np.abs(fast.cc1(g, 0.0, axis, dx, dy) - g)) <= 1e-13


def test_lc_matches_closed_form_gaussian():
    """A draw whose rank-one gauges both give small stage matrices: both LC
    orientations match the closed form; the literal chain is its negative."""
    N = 128
    d = math.sqrt(2 * math.pi / N)
    c = synth.symplectic_candidates(7)
    next(c)
    M = next(c)
    g = direct.gaussian(GAUSS_S, GAUSS_BETA, N, N, d, d)
    ref = direct.gaussian_nslct(M, GAUSS_S, GAUSS_BETA, N, N, d, d)
    for axis in (0, 1):
        p = fast.lc_plan(M, N, N, d, d, axis=axis)
        assert chain.rel_l2(fast.forward(p, g), ref) <= 1e-12
        assert chain.rel_l2(fast.forward(p, g, literal=True), -ref) <= 1e-12
    # The automatic choice takes the smaller eq. HA24 objective.
    cands = fast.lc_candidates(M)
    assert fast.lc_plan(M, N, N, d, d).f == min(cnd[3] for cnd in cands)


def test_lc_not_applicable_without_off_diagonal_a():
    """a12 = a21 = 0 (the FT has A = 0): neither rank-one gauge exists."""
    with pytest.raises(fast.NotApplicable):
        fast.lc_plan(FT, 16, 16, 1.0, 1.0)


@pytest.mark.parametrize("kind", ["cmccm", "lc"])
def test_unitary_and_inverse_is_adjoint(kind):
    Nx, Ny, dx, dy = 16, 24, 0.5, 0.4
    if kind == "cmccm":
        p = fast.cmccm_plan(_cmccm_matrices(9, 1)[0], Nx, Ny, dx, dy)
    else:
        p = fast.lc_plan(next(synth.symplectic_candidates(13)), Nx, Ny, dx, dy)
    x = synth.complex_normal((Nx, Ny), seed=1)
    y = synth.complex_normal((Nx, Ny), seed=2)
    Lx = fast.forward(p, x)
    assert abs(np.linalg.norm(Lx) / np.linalg.norm(x) - 1) <= 1e-13
    assert abs(np.vdot(y, Lx) - np.vdot(fast.inverse(p, y), x)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)
    assert chain.rel_l2(fast.inverse(p, Lx), x) <= 1e-13


def test_planted_mistakes_are_caught(monkeypatch):
    """A wrong h sign (eq. LC08), a transposed P3 / P1 order or a wrong 1D
    DFT constant in the oracle each break one of the pins above."""
    N = 64
    d = math.sqrt(2 * math.pi / N)
    c = synth.symplectic_candidates(7)
    next(c)
    M = next(c)
    g = direct.gaussian(GAUSS_S, GAUSS_BETA, N, N, d, d)
    ref = direct.gaussian_nslct(M, GAUSS_S, GAUSS_BETA, N, N, d, d)

    def lc_err():
        return chain.rel_l2(fast.forward(fast.lc_plan(M, N, N, d, d, axis=1), g), ref)

    assert lc_err() <= 1e-8  # N = 64: the Gaussian's tails alias slightly
    orig_cands = fast.lc_candidates

    def wrong_h(Mx):
        out = []
        for axis, h, mats, f in orig_cands(Mx):
            out.append((axis, -h, mats, f))
        return out

    monkeypatch.setattr(fast, "lc_candidates", wrong_h)
    assert lc_err() > 1e-3
    monkeypatch.setattr(fast, "lc_candidates", orig_cands)

    def swapped(Mx):
        return [(a, h, (m[2], m[1], m[0], m[3]), f) for a, h, m, f in orig_cands(Mx)]

    monkeypatch.setattr(fast, "lc_candidates", swapped)
    assert lc_err() > 1e-3
    monkeypatch.setattr(fast, "lc_candidates", orig_cands)

    orig_dft1 = fast.dft1
    monkeypatch.setattr(fast, "dft1", lambda x, a, dl, s: orig_dft1(x, a, dl, s) * (1j if s < 0 else 1))
    assert lc_err() > 1e-3
