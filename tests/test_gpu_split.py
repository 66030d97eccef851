"""GPU tests of the split-precision path (line DFTs on the matrix cores with
high + low FP16 / BF16 operand parts, FP32 accumulation).

Bars (relative L2): split parts <= 1e-4 against the FP64 oracle at 256 x 256;
at 8 x 4096 x 4096 (beyond the oracle's reach) every output of the split and
FP32 paths against the complex128 GPU path, itself pinned to the oracle at
<= 1e-11 by the parity tests.
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


@pytest.mark.parametrize("precision", ["c64_split_f16", "c64_split_bf16"])
@pytest.mark.parametrize("shape", [(256, 256), (256, 4096), (4096, 256)])
def test_split_matches_oracle(torch, nl, precision, shape):
    Nx, Ny = shape
    M = next(synth.symplectic_candidates(41))
    d = math.sqrt(2 * math.pi / max(Nx, Ny))
    po = oplan.plan(M, Nx, Ny, d, d)
    ps = nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, precision)
    g = synth.complex_normal(shape, seed=9)
    x = torch.from_numpy(g).to(torch.complex64).cuda()
    G = ps.forward(x).cpu().numpy()
    if Nx * Ny <= 256 * 256:
        ref = chain.forward(po, g)
    else:
        p64 = nl.Plan.from_stages(po.typ, po.mats, Nx, Ny, d, d, "c128")
        ref = p64.forward(x.to(torch.complex128)).cpu().numpy()
    assert chain.rel_l2(G, ref) <= 1e-4
    back = ps.inverse(ps.forward(x)).cpu().numpy()
    assert chain.rel_l2(back, g) <= 1e-4


def test_batch8_4096_all_precisions(torch, nl):
    """8 images of 4096 x 4096, one matrix each: split FP16 and BF16 <= 1e-4,
    FP32 <= 1e-5 per output, all against the complex128 GPU path."""
    N = 4096
    d = math.sqrt(2 * math.pi / N)
    cands = synth.symplectic_candidates(3)
    worst = {"c64": 0.0, "c64_split_f16": 0.0, "c64_split_bf16": 0.0}
    for b in range(8):
        M = next(cands)
        p64 = nl.Plan(M, N, N, d, d, precision="c128")
        st = p64.stages()
        x = torch.from_numpy(synth.complex_normal((N, N), seed=100 + b)).cuda()
        ref = p64.forward(x)
        xc = x.to(torch.complex64)
        for prec in worst:
            p = nl.Plan.from_stages(st["type"], st["mats"], N, N, d, d, prec)
            G = p.forward(xc).to(torch.complex128)
            err = (torch.linalg.vector_norm(G - ref) / torch.linalg.vector_norm(ref)).item()
            worst[prec] = max(worst[prec], err)
        del x, ref, xc
    assert worst["c64"] <= 1e-5, worst
    assert worst["c64_split_f16"] <= 1e-4, worst
    assert worst["c64_split_bf16"] <= 1e-4, worst
