"""Differentiable NsDLCT: ``torch.autograd.Function`` over the C ABI.

``nsdlct(x, theta, M0, dx, dy)`` returns the forward transform of x (a
complex tensor [..., Nx, Ny] on the GPU) for the ABCD matrix
M(theta) = M0 expm(J S(theta)), where theta holds the 10 coordinates of the
Lie algebra of the ABCD group (the upper triangle of the symmetric 4x4 S).

Backward (all in the library): ``nslct_backward_theta`` runs the adjoint
chain on the forward output and on the incoming gradient together (the
transform is unitary, so dLoss/dx = L^H grad), collects the derivative with
respect to every stage-matrix entry at the chirp points and chains it with
d(stage entries)/d(theta) of the plan into dLoss/dtheta.  The binding only
marshals arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import Plan, _stream_ptr
from ._lib import check, lib

_D = ctypes.POINTER(ctypes.c_double)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def lie_point(M0, theta) -> np.ndarray:
    """M0 expm(J S(theta)) computed by the library (host)."""
    m = np.ascontiguousarray(np.asarray(M0, dtype=np.float64).reshape(16))
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(10))
    out = np.zeros(16)
    check(lib.nslct_lie_point(_dptr(m), _dptr(th), _dptr(out)))
    return out.reshape(4, 4)


def plan_jacobian(M0, theta, Nx, Ny, dx, dy, precision="c64", type_override=0, h=1e-4) -> np.ndarray:
    """d(stage entries)/d(theta), shape (12, 10)."""
    m = np.ascontiguousarray(np.asarray(M0, dtype=np.float64).reshape(16))
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(10))
    opts = lib.opts()
    opts.precision = {"c64": 0, "c128": 1}[precision]
    opts.type_override = int(type_override)
    jac = np.zeros(120)
    check(lib.nslct_plan_jacobian(_dptr(m), _dptr(th), int(Nx), int(Ny), float(dx), float(dy),
                                  ctypes.byref(opts), float(h), _dptr(jac)))
    return jac.reshape(12, 10)


def backward_sums(plan: Plan, G, grad_out, stream=None):
    """(grad_x, 15 raw sums) of the adjoint sweep (nslct_backward)."""
    count = plan._check_tensor(G)
    plan._check_tensor(grad_out)
    work = torch.empty_like(G)
    grad_x = torch.empty_like(G)
    sums = torch.zeros(15, dtype=torch.float64, device=G.device)
    check(lib.nslct_backward(plan._h, int(count), ctypes.c_void_p(G.data_ptr()),
                             ctypes.c_void_p(grad_out.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                             ctypes.c_void_p(grad_x.data_ptr()), ctypes.c_void_p(sums.data_ptr()),
                             ctypes.c_void_p(_stream_ptr(stream))))
    return grad_x, sums


def stage_gradient(plan: Plan, sums) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(sums, dtype=np.float64).reshape(15))
    g = np.zeros(12)
    check(lib.nslct_plan_stage_gradient(plan._h, _dptr(s), _dptr(g)))
    return g


class NsLCTFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, theta, M0, dx, dy, precision, type_override):
        th = theta.detach().to("cpu", torch.float64).numpy()
        Nx, Ny = int(x.shape[-2]), int(x.shape[-1])
        plan = Plan.lie(M0, th, Nx, Ny, dx, dy, precision=precision, type_override=type_override,
                        symplectic_tol=1e-8)
        G = plan.forward(x.contiguous())
        ctx.plan = plan
        ctx.theta_meta = (theta.dtype, theta.device)
        ctx.save_for_backward(G)
        return G

    @staticmethod
    def backward(ctx, grad_out):
        (G,) = ctx.saved_tensors
        grad_x, gtheta = ctx.plan.backward_theta(G, grad_out.contiguous(), want_theta=ctx.needs_input_grad[1])
        dtype, device = ctx.theta_meta
        gt = torch.as_tensor(gtheta, dtype=dtype, device=device) if gtheta is not None else None
        return grad_x, gt, None, None, None, None, None


def nsdlct(x, theta, M0, dx: float, dy: float, precision: str = "c64", type_override: int = 0):
    """Differentiable forward NsDLCT of x for ABCD = M0 expm(J S(theta))."""
    return NsLCTFunction.apply(x, theta, M0, float(dx), float(dy), precision, int(type_override))
