"""GPU tests of the single-launch chain for small square images held in LDS
(32 x 32 at every image count, 64 x 64 from 32 complex64 / 128 complex128
images per call): every image equals the pass-by-pass launches of the same
plan bit for bit where both run line plan 0 (complex128 passes over 64-long
lines take the alternative split, so there the two agree to rounding,
relative L2 <= 1e-13), selected images match the FP64
oracle element by element (relative L2: complex64 <= 1e-5, complex128 <=
1e-11), in place equals out of place, and the inverse reconstructs.  The
reduced schedules (CM-CC-CM, LC, the IDFT route) run through the same
kernel."""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import chain, fast, plan as oplan

pytestmark = pytest.mark.gpu
TOL = {"c64": 1e-5, "c128": 1e-11}
I2, Z2 = np.eye(2), np.zeros((2, 2))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def nl(torch):
    import paper_1707_03688_amd as _nl
    return _nl


def _dtype(torch, precision):
    return torch.complex64 if precision == "c64" else torch.complex128


def _by_passes(p, torch, x, direction=0):
    """One image through launch_pass, pass by pass (the multi-launch path)."""
    z = torch.empty_like(x)
    for k in range(p.passes()):
        p.launch_pass(direction, k, x if k == 0 else z, z)
    return z


@pytest.mark.parametrize("N,count,precision", [(32, 1, "c64"), (32, 1, "c128"), (32, 7, "c64"),
                                               (64, 32, "c64"), (64, 128, "c128")])
def test_resident_chain_matches_passes_and_oracle(torch, nl, N, count, precision):
    c = synth.symplectic_candidates(61 + N)
    M = next(c)
    d = math.sqrt(2 * math.pi / N)
    po = oplan.plan(M, N, N, d, d)
    p = nl.Plan.from_stages(po.typ, po.mats, N, N, d, d, precision)
    g = synth.complex_normal((count, N, N), seed=N + count)
    x = torch.from_numpy(g).to(_dtype(torch, precision)).cuda()
    many = p.forward(x)
    torch.cuda.synchronize()
    same_plan = precision == "c64" or N == 32

    def agree(a, b):
        if same_plan:
            return torch.equal(a, b)
        return chain.rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-13

    for b in sorted({0, count // 2, count - 1}):
        assert agree(_by_passes(p, torch, x[b].contiguous()), many[b]), f"image {b}"
        assert chain.rel_l2(many[b].cpu().numpy(), chain.forward(po, g[b])) <= TOL[precision]
    y = x.clone()
    p.forward(y, out=y)
    assert torch.equal(y, many)
    back = p.inverse(many)
    assert chain.rel_l2(back.cpu().numpy(), g) <= TOL[precision]
    b = count - 1
    assert agree(_by_passes(p, torch, many[b].contiguous(), 1), back[b])


def _cmccm_matrix(seed):
    rng = np.random.default_rng(seed)
    while True:
        P1, B, P3 = [0.5 * (x + x.T) for x in (rng.normal(size=(2, 2)) * s for s in (0.5, 1.0, 0.5))]
        if abs(np.linalg.det(B)) > 0.05:
            return (np.block([[I2, Z2], [P1, I2]]) @ np.block([[I2, B], [Z2, I2]])
                    @ np.block([[I2, Z2], [P3, I2]]))


def _lc_matrix(seed):
    c = synth.symplectic_candidates(seed)
    while True:
        M = next(c)
        if fast.lc_candidates(M):
            return M


@pytest.mark.parametrize("typ", [3, 4, 5])
@pytest.mark.parametrize("N,count,precision", [(32, 2, "c64"), (64, 32, "c64"), (32, 3, "c128")])
def test_resident_reduced_schedules(torch, nl, typ, N, count, precision):
    """CM-CC-CM and LC (three passes, three line DFTs in the middle one)
    against the oracle's reduced chains and against the pass launches."""
    d = math.sqrt(2 * math.pi / N)
    M = _cmccm_matrix(N + typ) if typ == 3 else _lc_matrix(N + typ)
    p = nl.Plan(M, N, N, d, d, precision=precision, type_override=typ)
    assert p.passes() == 3 and p.stages()["type"] == typ
    po = fast.cmccm_plan(M, N, N, d, d) if typ == 3 else fast.lc_plan(M, N, N, d, d, axis=typ - 4)
    g = synth.complex_normal((count, N, N), seed=7 * typ + N)
    x = torch.from_numpy(g).to(_dtype(torch, precision)).cuda()
    many = p.forward(x)
    for b in (0, count - 1):
        assert torch.equal(_by_passes(p, torch, x[b].contiguous()), many[b])
        assert chain.rel_l2(many[b].cpu().numpy(), fast.forward(po, g[b])) <= TOL[precision]
    assert chain.rel_l2(p.inverse(many).cpu().numpy(), g) <= TOL[precision]


@pytest.mark.parametrize("N,count", [(32, 1), (64, 32)])
def test_resident_idft_route(torch, nl, N, count):
    """Type 7 (IDFT, then CM-CC-CM of the rotated matrix; four passes)
    against the oracle's route and the pass launches."""
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from oracle import route
    from test_oracle_route import route_matrices
    d = math.sqrt(2 * math.pi / N)
    M = route_matrices(N, 1)[0]
    p = nl.Plan(M, N, N, d, d, type_override=7)
    assert p.passes() == 4
    pr = route.route_plan(M, N, N, d, d, oplan.plan(M, N, N, d, d))
    g = synth.complex_normal((count, N, N), seed=N + 5)
    x = torch.from_numpy(g).to(torch.complex64).cuda()
    many = p.forward(x)
    for b in (0, count - 1):
        assert torch.equal(_by_passes(p, torch, x[b].contiguous()), many[b])
        assert chain.rel_l2(many[b].cpu().numpy(), route.forward(pr, g[b])) <= TOL["c64"]
    assert chain.rel_l2(p.inverse(many).cpu().numpy(), g) <= TOL["c64"]
