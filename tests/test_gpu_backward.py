"""GPU tests of the adjoint kernel and the differentiable transform.

dLoss/dx and dLoss/dtheta (theta = 10 Lie coordinates of M0 expm(J S(theta)))
for loss = ||NsDLCT_M(theta)(x) - y||^2 are compared with the FP64 oracle:
dLoss/dx = 2 L^H (L x - y) with the oracle's inverse chain, and dLoss/dtheta
with central finite differences (h = 1e-5) of the oracle loss, the oracle
re-planning (its own gauge search) at every M(theta +- h e_i), M built with
scipy's expm.  At the batched 512 x 512 size the dx-gradient is checked
against the oracle on two images, all ten theta components against central
differences (h = 1e-4) of the complex128 loss, and one image's complex128
theta-gradient against the oracle's finite differences.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from scipy.linalg import expm

import synth
from oracle import chain, plan as oplan

pytestmark = pytest.mark.gpu

J4 = np.block([[np.zeros((2, 2)), np.eye(2)], [-np.eye(2), np.zeros((2, 2))]])


def _S(theta):
    S = np.zeros((4, 4))
    k = 0
    for r in range(4):
        for c in range(r, 4):
            S[r, c] = S[c, r] = theta[k]
            k += 1
    return S


def _M(M0, theta):
    return M0 @ expm(J4 @ _S(theta))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def ag(torch):
    from paper_1707_03688_amd import autograd as _ag
    return _ag


def _oracle_loss(M, x, y, dx, dy, typ):
    Nx, Ny = x.shape[-2:]
    p = oplan.plan(M, Nx, Ny, dx, dy, typ=typ)
    return sum(float(np.sum(np.abs(chain.forward(p, xi) - yi) ** 2)) for xi, yi in zip(x, y))


@pytest.mark.parametrize("seed,shape", [(5, (32, 48)), (6, (32, 48)), (6, (30, 45)), (6, (30, 100))])
def test_gradients_match_oracle_finite_differences(torch, ag, seed, shape):
    """(30, 45), (30, 100): both axes without a native line plan (Bluestein
    passes in the forward chain and in the paired backward sweep; 100-long
    lines run on 256-point lines with the alternative split).  The draws have
    their eq. HA24 minimum on a kink set, where both gauge searches land on
    the same gauge to rounding, so the oracle's re-planned central
    differences are clean (at a smooth minimum the two searches' polish,
    ~1e-7 in the stage entries, would dominate a step of 1e-5)."""
    M0 = next(synth.symplectic_candidates(seed))
    (Nx, Ny), dx, dy = shape, 0.45, 0.6
    x = synth.complex_normal((2, Nx, Ny), seed=seed)
    y = synth.complex_normal((2, Nx, Ny), seed=seed + 100)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    yt = torch.from_numpy(y).cuda()
    theta = torch.zeros(10, dtype=torch.float64, requires_grad=True)
    G = ag.nsdlct(xt, theta, M0, dx, dy, precision="c128")
    loss = (G - yt).abs().pow(2).sum()
    loss.backward()
    typ = oplan.plan(M0, Nx, Ny, dx, dy).typ
    # dLoss/dx = 2 L^H (L x - y), with the oracle's chain at the library's
    # stages (the two gauge searches agree to ~1e-7 where the minimum is not
    # on a kink, which moves a 30 x 45 operator by ~1e-6)
    import paper_1707_03688_amd as nl
    st = nl.Plan.lie(M0, np.zeros(10), Nx, Ny, dx, dy, precision="c128").stages()
    p0 = oplan.plan_from_stages(st["type"], st["mats"], Nx, Ny, dx, dy)
    ref_gx = np.stack([2 * chain.inverse(p0, chain.forward(p0, xi) - yi) for xi, yi in zip(x, y)])
    assert chain.rel_l2(xt.grad.cpu().numpy(), ref_gx) <= 1e-9
    # The loss curves strongly in theta: a central difference at h = 1e-5
    # keeps an O(h^2) error of 2e-7 (30 x 45) to 2e-6 (30 x 100) relative, so
    # the reference is the Richardson extrapolation of h and h / 2 (O(h^4)).
    def central(h):
        fd = np.zeros(10)
        for i in range(10):
            e = np.zeros(10)
            e[i] = h
            fd[i] = (_oracle_loss(_M(M0, e), x, y, dx, dy, typ)
                     - _oracle_loss(_M(M0, -e), x, y, dx, dy, typ)) / (2 * h)
        return fd

    fd = (4 * central(5e-6) - central(1e-5)) / 3
    got = theta.grad.numpy()
    assert np.linalg.norm(got - fd) <= 2e-6 * np.linalg.norm(fd), (got, fd)


def test_batch32_512_gradients(torch, ag):
    """32 x 512 x 512 complex64, y the transform under a perturbed matrix
    (theta* ~ N(0, 0.05) in the Lie coordinates).  The library's gradients
    (nslct_backward_theta through the autograd function) against:
      * dLoss/dx of images 0 and 31: the FP64 oracle's 2 L^H (L x - y) at the
        plan's stages;
      * all 10 components of dLoss/dtheta: central differences with h = 1e-4
        and h / 2 (Richardson) of the complex128 loss over the 32 images;
      * the complex128 dLoss/dtheta of image 0 alone: central differences
        (h = 1e-5 and h / 2, Richardson) of the FP64 oracle's loss, the oracle
        planning its own gauge at every M(theta +- h e_i)."""
    import paper_1707_03688_amd as nl
    N = 512
    d = math.sqrt(2 * math.pi / N)
    M0 = next(synth.symplectic_candidates(4))
    rng = np.random.default_rng(4)
    theta_star = rng.normal(0.0, 0.05, size=10)
    x = torch.from_numpy(synth.complex_normal((32, N, N), seed=4)).to(torch.complex64).cuda()
    pstar = nl.Plan.lie(M0, theta_star, N, N, d, d, symplectic_tol=1e-8)
    y = pstar.forward(x)
    xg = x.clone().requires_grad_(True)
    theta = torch.zeros(10, dtype=torch.float64, requires_grad=True)
    G = ag.nsdlct(xg, theta, M0, d, d)
    loss = (G - y).abs().pow(2).sum()
    loss.backward()
    p0 = nl.Plan.lie(M0, np.zeros(10), N, N, d, d, symplectic_tol=1e-8)
    st = p0.stages()
    po = oplan.plan_from_stages(st["type"], st["mats"], N, N, d, d)
    xh = x.cpu().numpy().astype(np.complex128)
    yh = y.cpu().numpy().astype(np.complex128)
    gx = xg.grad.cpu().numpy()
    for i in (0, 31):
        ref = 2 * chain.inverse(po, chain.forward(po, xh[i]) - yh[i])
        assert chain.rel_l2(gx[i], ref) <= 1e-5
    typ = st["type"]
    x64, y64 = x.to(torch.complex128), y.to(torch.complex128)

    def loss64(th):
        p = nl.Plan.lie(M0, th, N, N, d, d, precision="c128", type_override=typ, symplectic_tol=1e-8)
        return (p.forward(x64) - y64).abs().pow(2).sum().item()

    # At 512 x 512 the loss curves strongly in theta: the h = 1e-4 central
    # difference alone is off by ~2e-3 relative (O(h^2)), so it is combined
    # with h / 2 by Richardson extrapolation (error O(h^4)).
    def central(h):
        out = np.zeros(10)
        for i in range(10):
            e = np.zeros(10)
            e[i] = h
            out[i] = (loss64(e) - loss64(-e)) / (2 * h)
        return out

    h = 1e-4
    fd = (4 * central(h / 2) - central(h)) / 3
    got = theta.grad.numpy()
    assert np.linalg.norm(got - fd) <= 1e-4 * np.linalg.norm(fd), (got, fd)
    # One image in complex128 against the oracle's own loss.
    x1 = x64[:1].clone().requires_grad_(True)
    th1 = torch.zeros(10, dtype=torch.float64, requires_grad=True)
    l1 = (ag.nsdlct(x1, th1, M0, d, d, precision="c128") - y64[:1]).abs().pow(2).sum()
    l1.backward()
    def central_oracle(h):
        out = np.zeros(10)
        for i in range(10):
            e = np.zeros(10)
            e[i] = h
            out[i] = (_oracle_loss(_M(M0, e), xh[:1], yh[:1], d, d, typ)
                      - _oracle_loss(_M(M0, -e), xh[:1], yh[:1], d, d, typ)) / (2 * h)
        return out

    h = 1e-5
    fdo = (4 * central_oracle(h / 2) - central_oracle(h)) / 3
    got1 = th1.grad.numpy()
    assert np.linalg.norm(got1 - fdo) <= 2e-6 * np.linalg.norm(fdo), (got1, fdo)


def test_backward_theta_without_theta_and_plan_jacobian(torch, ag):
    """nslct_backward_theta with grad_theta = NULL gives the same grad_x
    bits; the plan's cached Jacobian agrees with nslct_plan_jacobian's
    re-solved central differences (step of its type) to their truncation."""
    import paper_1707_03688_amd as nl
    M0 = next(synth.symplectic_candidates(5))
    Nx, Ny, dx, dy = 64, 48, 0.45, 0.6
    th = np.linspace(-0.02, 0.03, 10)
    p = nl.Plan.lie(M0, th, Nx, Ny, dx, dy, symplectic_tol=1e-8)
    G = torch.from_numpy(synth.complex_normal((3, Nx, Ny), seed=1)).to(torch.complex64).cuda()
    g = torch.from_numpy(synth.complex_normal((3, Nx, Ny), seed=2)).to(torch.complex64).cuda()
    gx1, gt = p.backward_theta(G, g)
    gx2, none = p.backward_theta(G, g, want_theta=False)
    torch.cuda.synchronize()
    assert none is None and torch.equal(gx1, gx2) and np.all(np.isfinite(gt))
    typ = p.stages()["type"]
    ref = ag.plan_jacobian(M0, th, Nx, Ny, dx, dy, type_override=typ, h=1e-5 if typ >= 3 else 1e-4)
    J = p.theta_jacobian()
    assert np.max(np.abs(J - ref)) <= 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("override", [4, 5])
def test_lc_gradients_match_oracle_finite_differences(torch, ag, override):
    """The LC-NsDLCT (rank-one gauge h of eqs. LC08 / LC10, a closed form in
    M): dLoss/dx and dLoss/dtheta against the oracle's LC chain
    (``oracle.fast``), central differences with h = 1e-6."""
    from oracle import fast
    M0 = next(synth.symplectic_candidates(13))
    Nx, Ny, dx, dy = 32, 48, 0.45, 0.6
    axis = override - 4
    x = synth.complex_normal((2, Nx, Ny), seed=3)
    y = synth.complex_normal((2, Nx, Ny), seed=4)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    yt = torch.from_numpy(y).cuda()
    theta = torch.zeros(10, dtype=torch.float64, requires_grad=True)
    G = ag.nsdlct(xt, theta, M0, dx, dy, precision="c128", type_override=override)
    loss = (G - yt).abs().pow(2).sum()
    loss.backward()
    p0 = fast.lc_plan(M0, Nx, Ny, dx, dy, axis=axis)
    ref_gx = np.stack([2 * fast.inverse(p0, fast.forward(p0, xi) - yi) for xi, yi in zip(x, y)])
    assert chain.rel_l2(xt.grad.cpu().numpy(), ref_gx) <= 1e-9

    def oloss(M):
        p = fast.lc_plan(M, Nx, Ny, dx, dy, axis=axis)
        return sum(float(np.sum(np.abs(fast.forward(p, xi) - yi) ** 2)) for xi, yi in zip(x, y))

    # The LC stage matrices of this draw are large, so the loss curves more
    # strongly than in the HA test: h = 1e-6 (FP64 rounding stays ~1e-10).
    h = 1e-6
    fd = np.zeros(10)
    for i in range(10):
        e = np.zeros(10)
        e[i] = h
        fd[i] = (oloss(_M(M0, e)) - oloss(_M(M0, -e))) / (2 * h)
    got = theta.grad.numpy()
    assert np.linalg.norm(got - fd) <= 2e-6 * np.linalg.norm(fd), (got, fd)
