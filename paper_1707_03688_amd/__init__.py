"""MI355X-native 2D nonseparable discrete LCT (CM-CC-CM-CC decomposition).

Thin Python binding of ``libnslct.so`` (C ABI in ``include/nslct.h``).  The
binding only marshals arguments: every step of the transform runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current HIP
stream.  There is no fallback: if the library is missing or fails to load,
importing this package raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (NSLCT_C64, NSLCT_C128, NslctError, Stages, lib, check)  # noqa: F401

__all__ = ["Plan", "Batch", "NslctError", "lib", "device_copy", "NSLCT_C64", "NSLCT_C128"]

_PRECISION = {"c64": NSLCT_C64, "c128": NSLCT_C128, "c64_split_f16": 2, "c64_split_bf16": 3}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Plan:
    """A planned transform for one ABCD matrix and grid.

    Mirrors ``nslct_plan_ex`` / ``nslct_plan_from_stages``; ``forward`` and
    ``inverse`` run on torch tensors of shape [..., Nx, Ny] (complex64 for
    precision "c64", complex128 for "c128") resident on the current device.
    """

    def __init__(self, abcd=None, Nx: int = 0, Ny: int = 0, dx: float = 1.0, dy: float = 1.0,
                 precision: str = "c64", type_override: int = 0, symplectic_tol: float = 1e-9,
                 _handle=None):
        self.precision = precision
        if _handle is not None:
            self._h = _handle
        else:
            opts = lib.opts()
            opts.precision = _PRECISION[precision]
            opts.type_override = int(type_override)
            opts.symplectic_tol = float(symplectic_tol)
            m = np.ascontiguousarray(np.asarray(abcd, dtype=np.float64).reshape(16))
            h = ctypes.c_void_p()
            check(lib.nslct_plan_ex(m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(Nx), int(Ny),
                                    float(dx), float(dy), ctypes.byref(opts), ctypes.byref(h)))
            self._h = h
        self.Nx, self.Ny = int(Nx), int(Ny)

    @classmethod
    def lie(cls, M0, theta, Nx: int, Ny: int, dx: float = 1.0, dy: float = 1.0, precision: str = "c64",
            type_override: int = 0, symplectic_tol: float = 1e-9) -> "Plan":
        """Plan of M0 expm(J S(theta)) for differentiation (``nslct_plan_lie``)."""
        opts = lib.opts()
        opts.precision = _PRECISION[precision]
        opts.type_override = int(type_override)
        opts.symplectic_tol = float(symplectic_tol)
        m = np.ascontiguousarray(np.asarray(M0, dtype=np.float64).reshape(16))
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(10))
        h = ctypes.c_void_p()
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib.nslct_plan_lie(m.ctypes.data_as(dp), th.ctypes.data_as(dp), int(Nx), int(Ny), float(dx),
                                 float(dy), ctypes.byref(opts), ctypes.byref(h)))
        p = cls.__new__(cls)
        p.precision = precision
        p._h = h
        p.Nx, p.Ny = int(Nx), int(Ny)
        return p

    @classmethod
    def from_stages(cls, typ: int, mats, Nx: int, Ny: int, dx: float, dy: float,
                    precision: str = "c64", phase_q: int = 0) -> "Plan":
        st = Stages()
        st.type = int(typ)
        st.phase_q = int(phase_q)
        for i, X in enumerate(mats):
            X = np.asarray(X, dtype=np.float64)
            st.mats[i][0] = X[0, 0]
            st.mats[i][1] = 0.5 * (X[0, 1] + X[1, 0])
            st.mats[i][2] = X[1, 1]
        st.dx, st.dy = float(dx), float(dy)
        opts = lib.opts()
        opts.precision = _PRECISION[precision]
        h = ctypes.c_void_p()
        check(lib.nslct_plan_from_stages(ctypes.byref(st), int(Nx), int(Ny), ctypes.byref(opts),
                                         ctypes.byref(h)))
        p = cls.__new__(cls)
        p.precision = precision
        p._h = h
        p.Nx, p.Ny = int(Nx), int(Ny)
        return p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.nslct_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------------ info
    def stages(self) -> dict:
        st = Stages()
        check(lib.nslct_plan_get_stages(self._h, ctypes.byref(st)))
        mats = []
        for i in range(4):
            a, b, c = st.mats[i][0], st.mats[i][1], st.mats[i][2]
            mats.append(np.array([[a, b], [b, c]]))
        return {"type": st.type, "mats": mats, "h": np.array(list(st.h)),
                "f": st.gauge_objective, "residual": st.symplectic_residual,
                "dx": st.dx, "dy": st.dy, "dwx": st.dwx, "dwy": st.dwy, "phase_q": st.phase_q,
                "Nx": getattr(self, "Nx", None), "Ny": getattr(self, "Ny", None)}

    def prepare(self):
        """Device tables of the plan on the current device (``nslct_plan_prepare``):
        afterwards its transforms allocate nothing and can be graph-captured."""
        check(lib.nslct_plan_prepare(self._h))
        return self

    def passes(self) -> int:
        """Passes of the single-image path (3 for the reduced chains, else 5)."""
        n = ctypes.c_int()
        check(lib.nslct_plan_passes(self._h, ctypes.byref(n)))
        return n.value

    def box_check(self, frac: float = 0.5) -> bool:
        ok = ctypes.c_int()
        check(lib.nslct_plan_box_check(self._h, float(frac), ctypes.byref(ok)))
        return bool(ok.value)

    # ------------------------------------------------------------- transforms
    def _check_tensor(self, x):
        torch = _torch()
        want = torch.complex128 if self.precision == "c128" else torch.complex64
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_cuda:
            raise TypeError("tensor must be on the GPU")
        if tuple(x.shape[-2:]) != (self.Nx, self.Ny):
            raise ValueError(f"expected [..., {self.Nx}, {self.Ny}], got {tuple(x.shape)}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.numel() // (self.Nx * self.Ny)

    def _run(self, fn, x, out, stream):
        count = self._check_tensor(x)
        if out is None:
            out = _torch().empty_like(x)
        else:
            self._check_tensor(out)
            if out.shape != x.shape:
                raise ValueError("out must have the shape of x")
        check(fn(self._h, count, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                 ctypes.c_void_p(_stream_ptr(stream))))
        return out

    def forward(self, x, out=None, stream=None):
        return self._run(lib.nslct_forward_many, x, out, stream)

    def inverse(self, x, out=None, stream=None):
        return self._run(lib.nslct_inverse_many, x, out, stream)

    def backward_theta(self, G, grad_out, grad_x=None, want_theta: bool = True, stream=None):
        """(grad_x, grad_theta) of ``nslct_backward_theta``: grad_x on the
        device, grad_theta a numpy array of 10 doubles (None if not asked)."""
        count = self._check_tensor(G)
        self._check_tensor(grad_out)
        if grad_x is None:
            grad_x = _torch().empty_like(G)
        self._check_tensor(grad_x)
        gt = np.zeros(10) if want_theta else None
        check(lib.nslct_backward_theta(self._h, int(count), ctypes.c_void_p(G.data_ptr()),
                                       ctypes.c_void_p(grad_out.data_ptr()), ctypes.c_void_p(grad_x.data_ptr()),
                                       gt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if want_theta else None,
                                       ctypes.c_void_p(_stream_ptr(stream))))
        return grad_x, gt

    def theta_jacobian(self) -> np.ndarray:
        """d(stage entries)/d(theta), shape (12, 10) (``nslct_plan_theta_jacobian``)."""
        jac = np.zeros(120)
        check(lib.nslct_plan_theta_jacobian(self._h, jac.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return jac.reshape(12, 10)

    def launch_pass(self, direction: int, pass_: int, x, out, stream=None):
        count = self._check_tensor(x)
        check(lib.nslct_launch_pass(self._h, int(direction), int(pass_), int(count),
                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(_stream_ptr(stream))))
        return out


def device_copy(src, dst, stream=None):
    """Plain copy kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    check(lib.nslct_device_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                ctypes.c_size_t(nbytes), ctypes.c_void_p(_stream_ptr(stream))))
    return dst


class Batch:
    """A ragged batch of plans over one packed buffer (``nslct_batch_create``).

    Image i occupies samples [offsets[i], offsets[i] + Nx_i * Ny_i) of a flat
    complex tensor of ``total`` samples.  ``forward`` / ``inverse`` replay a
    captured HIP graph of the batched passes; ``run(mode=2)`` is the per-image
    reference loop.
    """

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        check(lib.nslct_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        total = ctypes.c_size_t()
        mult = ctypes.c_int()
        tuned = ctypes.c_double()
        check(lib.nslct_batch_info(h, ctypes.byref(total), ctypes.byref(mult), ctypes.byref(tuned)))
        self.total = int(total.value)
        self.mult = int(mult.value)
        self.tuned_us = float(tuned.value)
        self.precision = self.plans[0].precision
        self.offsets = []
        off = 0
        for p in self.plans:
            self.offsets.append(off)
            off += p.Nx * p.Ny

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.nslct_batch_destroy(h)
            self._h = None

    def _check(self, x):
        torch = _torch()
        want = torch.complex128 if self.precision == "c128" else torch.complex64
        if x.dtype != want or not x.is_cuda or not x.is_contiguous() or x.numel() != self.total:
            raise ValueError(f"expected a contiguous {want} GPU tensor of {self.total} samples")

    def run(self, x, out=None, direction: int = 0, mode: int = 0, stream=None):
        self._check(x)
        if out is None:
            out = _torch().empty_like(x)
        self._check(out)
        check(lib.nslct_batch_run(self._h, int(direction), int(mode), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))))
        return out

    def forward(self, x, out=None, stream=None):
        return self.run(x, out, 0, 0, stream)

    def inverse(self, x, out=None, stream=None):
        return self.run(x, out, 1, 0, stream)

    def set_grid(self, mult: int):
        """Override the autotuned grid (``nslct_batch_set_grid``): mult
        workgroups per CU, or 0 for one workgroup per work item."""
        check(lib.nslct_batch_set_grid(self._h, int(mult)))
        self.mult = int(mult)

    def group(self, col: int, N: int) -> dict:
        """Schedule of one group (``nslct_batch_group``): line plan, lines per
        work item, grid (workgroups per CU, 0 = one per item), cached."""
        plan, lines, mult, cached = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib.nslct_batch_group(self._h, int(col), int(N), ctypes.byref(plan), ctypes.byref(lines),
                                    ctypes.byref(mult), ctypes.byref(cached)))
        return {"plan": plan.value, "lines": lines.value, "mult": mult.value, "cached": bool(cached.value)}

    def schedules(self) -> dict:
        """Schedules of every group: {(col, N): {...}}."""
        out = {}
        for col in (0, 1):
            for N in sorted({p.Nx if col else p.Ny for p in self.plans}):
                out[(col, N)] = self.group(col, N)
        return out

    def set_group(self, col: int, N: int, lines: int, mult: int, plan: int = 0):
        """Set one group's line plan, tile width and grid (``nslct_batch_set_group``)."""
        check(lib.nslct_batch_set_group(self._h, int(col), int(N), int(plan), int(lines), int(mult)))

    def views(self, flat):
        """Per-image [Nx, Ny] views of a packed tensor."""
        return [flat[o:o + p.Nx * p.Ny].view(p.Nx, p.Ny) for o, p in zip(self.offsets, self.plans)]
