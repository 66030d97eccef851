"""GPU test of nslct_backward_theta_noalloc, the allocation-free backward
entry point (static device scratch): its gradients equal those of
nslct_backward_theta on the same inputs, on three workloads in a row (each
smaller than the one before), and after the device's one-time set-up a call takes no
device memory."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _call(nl, fn, plan, G, g, gx):
    gt = np.zeros(10)
    count = G.numel() // (plan.Nx * plan.Ny)
    rc = fn(plan._h, int(count), ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(g.data_ptr()),
            ctypes.c_void_p(gx.data_ptr()), gt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    nl.check(rc)
    return gt


def test_noalloc_backward_matches_allocating_entry_point(torch):
    import paper_1707_03688_amd as nl
    # 40 MiB (3 chunks); 9 images (chunks of 8 and 1: the line plan follows
    # the call's 9 images, not the chunk's); then 1.5 MiB.
    cases = [(512, 512, "c64", 20, 5), (512, 512, "c64", 9, 7), (256, 128, "c128", 3, 6)]
    for Nx, Ny, prec, count, seed in cases:
        print(f"no-alloc backward: {count} x {Nx} x {Ny} {prec}", flush=True)
        dt = torch.complex64 if prec == "c64" else torch.complex128
        d = math.sqrt(2 * math.pi / Nx)
        M0 = next(synth.symplectic_candidates(seed))
        p = nl.Plan.lie(M0, np.linspace(-0.03, 0.02, 10), Nx, Ny, d, d, precision=prec, symplectic_tol=1e-8)
        G = torch.from_numpy(synth.complex_normal((count, Nx, Ny), seed=seed)).to(dt).cuda()
        g = torch.from_numpy(synth.complex_normal((count, Nx, Ny), seed=seed + 1)).to(dt).cuda()
        gx_a = torch.empty_like(G)
        gx_n = torch.full_like(G, float("nan"))
        # The first call on a device may run the library's one-time device
        # set-up (its code objects and their device arrays are loaded then);
        # the call after it takes no device memory (memory released late by
        # earlier stream-ordered frees may show up as more, never less).
        _call(nl, nl.lib.nslct_backward_theta_noalloc, p, G, g, gx_n)
        gx_n.fill_(float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        gt_n = _call(nl, nl.lib.nslct_backward_theta_noalloc, p, G, g, gx_n)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] >= free0
        gt_a = _call(nl, nl.lib.nslct_backward_theta, p, G, g, gx_a)
        torch.cuda.synchronize()
        # Same kernels on the same images: grad_x to the bit; the theta sums
        # are accumulated by atomics in another order (rounding level).
        assert torch.equal(gx_n, gx_a)
        assert np.all(np.isfinite(gt_n))
        assert np.linalg.norm(gt_n - gt_a) <= 1e-12 * np.linalg.norm(gt_a), (gt_n, gt_a)
