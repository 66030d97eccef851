"""GPU tests of the split-precision path (line DFTs on the matrix cores with
high + low FP16 / BF16 operand parts, FP32 accumulation).

Bars (relative L2): split parts <= 1e-4 against the FP64 oracle at 256 x 256,
256 x 4096 and 4096 x 256, on zero-mean i.i.d. images and on non-negative
images with a large mean (whose 4096-long column DFTs reach values far
beyond FP16's range); at 8 x 4096 x 4096 one image per precision against
the FP64 oracle (complex128 GPU path <= 1e-11, FP32 <= 1e-5, split <= 1e-4)
and every output against the complex128 GPU path.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import synth
from oracle import chain, plan as oplan

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


_ORACLE = {}


def _oracle(po, g, key, direction):
    """Oracle output, computed once per (shape, image, direction) and shared
    by the two split precisions."""
    k = (key, direction)
    if k not in _ORACLE:
        _ORACLE[k] = (chain.forward if direction == "fwd" else chain.inverse)(po, g)
    return _ORACLE[k]


@pytest.mark.parametrize("image", ["normal", "nonneg"])
@pytest.mark.parametrize("precision", ["c64_split_f16", "c64_split_bf16"])
@pytest.mark.parametrize("shape", [(256, 256), (256, 4096), (4096, 256)])
def test_split_matches_oracle(torch, nl, precision, shape, image):
    """Forward and inverse against the FP64 oracle.  'nonneg' is |N(0,1)| + 3
    (mean ~3.8): the DC of a 4096-long column DFT after the row DFT is then
    ~6e7, about a thousand times FP16's largest finite value."""
    Nx, Ny = shape
    M = next(synth.symplectic_candidates(41))
    d = math.sqrt(2 * math.pi / max(Nx, Ny))
    po = oplan.plan(M, Nx, Ny, d, d)
    ps = nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, precision)
    g = synth.complex_normal(shape, seed=9)
    if image == "nonneg":
        g = (np.abs(g) + 3.0).astype(np.complex128)
    x = torch.from_numpy(g).to(torch.complex64).cuda()
    G = ps.forward(x).cpu().numpy()
    assert np.all(np.isfinite(G))
    assert chain.rel_l2(G, _oracle(po, g, (shape, image), "fwd")) <= 1e-4
    Gi = ps.inverse(x).cpu().numpy()
    assert chain.rel_l2(Gi, _oracle(po, g, (shape, image), "inv")) <= 1e-4
    back = ps.inverse(ps.forward(x)).cpu().numpy()
    assert chain.rel_l2(back, g) <= 1e-4


def test_batch8_4096_all_precisions(torch, nl):
    """8 images of 4096 x 4096, one matrix each: split FP16 and BF16 <= 1e-4,
    FP32 <= 1e-5 per output against the complex128 GPU path; image 0 of
    every precision (complex128 GPU <= 1e-11 too) against the FP64 oracle at
    the same stages (one oracle transform, ~30 s of host time)."""
    N = 4096
    d = math.sqrt(2 * math.pi / N)
    cands = synth.symplectic_candidates(3)
    worst = {"c64": 0.0, "c64_split_f16": 0.0, "c64_split_bf16": 0.0}
    for b in range(8):
        M = next(cands)
        p64 = nl.Plan(M, N, N, d, d, precision="c128")
        st = p64.stages()
        g = synth.complex_normal((N, N), seed=100 + b)
        x = torch.from_numpy(g).cuda()
        ref = p64.forward(x)
        xc = x.to(torch.complex64)
        outs = {}
        for prec in worst:
            p = nl.Plan.from_stages(st["type"], st["mats"], N, N, d, d, prec)
            G = p.forward(xc).to(torch.complex128)
            err = (torch.linalg.vector_norm(G - ref) / torch.linalg.vector_norm(ref)).item()
            worst[prec] = max(worst[prec], err)
            if b == 0:
                outs[prec] = G.cpu().numpy()
        if b == 0:
            po = oplan.plan_from_stages(st["type"], st["mats"], N, N, d, d)
            oref = chain.forward(po, g)
            assert chain.rel_l2(ref.cpu().numpy(), oref) <= 1e-11
            assert chain.rel_l2(outs["c64"], oref) <= 1e-5
            assert chain.rel_l2(outs["c64_split_f16"], oref) <= 1e-4
            assert chain.rel_l2(outs["c64_split_bf16"], oref) <= 1e-4
            del outs, oref
        del x, ref, xc
    assert worst["c64"] <= 1e-5, worst
    assert worst["c64_split_f16"] <= 1e-4, worst
    assert worst["c64_split_bf16"] <= 1e-4, worst
