"""GPU parity of the lengths without a native line FFT (Bluestein's chirp-z
form of each line DFT), and the paper's Sec. 5 experiments at the paper's
own grid sizes.

* Rectangular and square shapes with prime, odd and 2 x odd sides, complex64
  (relative L2 <= 1e-5) and complex128 (<= 1e-11) against the FP64 oracle,
  forward and inverse.
* Sec. 5.1 accuracy: g1 = HG1,2 + HG3,1 on 100 x 100 (spacing 0.25) through
  M1: NMSE against the direct method within a factor 3 of the printed 1.7e-6.
* Sec. 5.2 additivity: g2 on 165 x 165 (spacing 0.2), O(M4)O(M2) against
  O(M4 M2): the printed 0.052.
* Zero padding (Sec. 2.2): the same g1 padded to 100 + dN for dN in
  {10, 20, 50}: NMSE falls monotonically below the unpadded value.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import chain, direct, plan as oplan, symplectic
from oracle_fixtures import paper_matrices, printed_values

pytestmark = pytest.mark.gpu


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


def _pair(nl, M, Nx, Ny, dx, dy, precision, typ=0):
    po = oplan.plan(M, Nx, Ny, dx, dy, typ=typ or None)
    pg = nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, dx, dy, precision)
    return po, pg


SHAPES = [(100, 100), (165, 165), (101, 64), (64, 257), (3, 5), (7, 96), (2000, 8), (8, 1025), (1536, 6)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("precision", ["c64", "c128"])
def test_bluestein_lengths_match_oracle(torch, nl, shape, precision):
    Nx, Ny = shape
    M = next(synth.symplectic_candidates(31))
    # Spacing sqrt(2 pi / N) per axis keeps the chirp phases at the size the
    # paper's sampling conditions give; much larger phases (|phi| ~ 1e5 rad)
    # cost the FP64 oracle ~1e-11 of absolute phase rounding by themselves.
    dx, dy = math.sqrt(2 * math.pi / Nx), math.sqrt(2 * math.pi / Ny)
    po, pg = _pair(nl, M, Nx, Ny, dx, dy, precision)
    g = synth.complex_normal(shape, seed=Nx + 3 * Ny)
    dt = torch.complex128 if precision == "c128" else torch.complex64
    x = torch.from_numpy(g).to(dt).cuda()
    tol = 1e-11 if precision == "c128" else 1e-5
    assert chain.rel_l2(pg.forward(x).cpu().numpy(), chain.forward(po, g)) <= tol
    assert chain.rel_l2(pg.inverse(x).cpu().numpy(), chain.inverse(po, g)) <= tol


def _gpu_forward(nl, torch, M, g, d, typ=0):
    N = g.shape[0]
    p = nl.Plan(M, N, N, d, d, precision="c128", type_override=typ)
    return p.forward(torch.from_numpy(np.ascontiguousarray(g)).cuda()).cpu().numpy()


def test_printed_accuracy_g1_m1_at_100(torch, nl):
    pv = printed_values()
    M = symplectic.project(paper_matrices()["M1"])
    N, d = 100, 0.25
    g = synth.hg_signal([(1, 2), (3, 1)], N, d)
    df = pv["truth_spacing"]
    Nf = 2 * int(7.5 / df) + 1
    T = direct.direct(M, synth.hg_signal([(1, 2), (3, 1)], Nf, df), df, df, N, N, d, d)

    def nmse(G, o=0):
        Gc = G[o:o + N, o:o + N]
        return min(chain.rel_l2(Gc, T), chain.rel_l2(Gc, -T)) ** 2

    e0 = nmse(_gpu_forward(nl, torch, M, g, d))
    assert pv["nmse_acc_ha_g1"] / 3 <= e0 <= pv["nmse_acc_ha_g1"] * 3, e0
    prev = e0
    for dN in (10, 20, 50):
        Np = N + dN
        o = Np // 2 - N // 2
        gp = np.zeros((Np, Np), dtype=np.complex128)
        gp[o:o + N, o:o + N] = g
        e = nmse(_gpu_forward(nl, torch, M, gp, d), o)
        assert e < prev, (dN, e, prev)
        prev = e


def test_printed_additivity_g2_at_165(torch, nl):
    pv = printed_values()
    Ms = paper_matrices()
    M2, M4 = symplectic.project(Ms["M2"]), symplectic.project(Ms["M4"])
    N, d = 165, 0.2
    g = synth.hg_signal([(2, 18), (14, 11)], N, d)
    two = _gpu_forward(nl, torch, M4, _gpu_forward(nl, torch, M2, g, d), d)
    one = _gpu_forward(nl, torch, M4 @ M2, g, d)
    assert abs(chain.rel_l2(one, two) ** 2 - pv["nmse_add_ha_g2"]) <= 0.002


@pytest.mark.parametrize("shape", [(100, 75), (128, 64)])
def test_prepared_plan_captures_into_a_graph(torch, nl, shape):
    """After nslct_plan_prepare a transform allocates nothing, so a
    Bluestein-length (and a native) forward + inverse captures into a HIP
    graph; replays with unrelated eager work between them give the eager
    bits every time."""
    Nx, Ny = shape
    M = next(synth.symplectic_candidates(Nx + Ny))
    d = math.sqrt(2 * math.pi / max(Nx, Ny))
    plan = nl.Plan(M, Nx, Ny, d, d).prepare()
    x = torch.from_numpy(synth.complex_normal((2, Nx, Ny), seed=Nx)).to(torch.complex64).cuda()
    ref = plan.forward(x)
    ref_back = plan.inverse(ref)
    y = torch.empty_like(x)
    z = torch.empty_like(x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward(x, out=y)
        plan.inverse(y, out=z)
    for k in range(3):
        y.zero_()
        z.zero_()
        g.replay()
        junk = torch.randn(1 << 18, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(y, ref) and torch.equal(z, ref_back), k
        del junk
