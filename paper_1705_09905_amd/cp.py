"""CP decomposition drivers over the library: CP-ALS (Algorithm 1; one sweep
per fcoo_cp_als_iter call, everything on the device, the fit read back once
per sweep) and gradient-based sparse CP through torch.autograd Functions
whose backward passes are the library's SpMTTKRP kernels."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from . import _lib as L
from .tensor import Tensor, _dtype_code, _stream


def _torch():
    import torch
    return torch


def cp_als(t: Tensor, R: int, sweeps: int, init: Sequence, dtype: str = "f32", tol: float = 0.0,
           threadlen: int = 0, tile_nnz: int = 0, build: bool = True):
    """CP-ALS of `t` at rank R.  `init`: one dims[m] x R array per mode
    (numpy or torch; A_0's values are never read, Algorithm 1 overwrites
    them first).  dtype 'f32' or 'bf16' is the factor storage.  Stops after
    `sweeps` sweeps, or when tol > 0 and |fit change| < tol.
    Returns dict(factors=[torch], lam=torch (R,), fits=[float], used_pinv=[int bitmask])."""
    torch = _torch()
    if dtype not in ("f32", "bf16"):
        raise ValueError(f"dtype must be 'f32' or 'bf16' (got {dtype!r})")
    if len(init) != t.order:
        raise ValueError(f"need {t.order} initial factors")
    for m, a in enumerate(init):
        if tuple(a.shape) != (t.dims[m], R):
            raise ValueError(f"initial factor {m} must be {t.dims[m]} x {R} (got {tuple(a.shape)})")
    if build:
        for m in range(t.order):
            inf = None
            try:
                inf = t.info(m, "mttkrp")
            except L.FcooError:
                pass
            if inf is None or not inf["on_device"]:
                t.build(m, "mttkrp", threadlen=threadlen, tile_nnz=tile_nnz)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    factors = []
    for m, a in enumerate(init):
        x = torch.as_tensor(np.asarray(a, dtype=np.float32) if not isinstance(a, torch.Tensor) else a)
        # a private copy: the sweeps overwrite the factors in place, and for a
        # contiguous CUDA float32 input the conversions below return the
        # caller's own tensor
        f = torch.empty((t.dims[m], R), dtype=tdt, device="cuda")
        f.copy_(x.to(device="cuda", dtype=torch.float32))
        factors.append(f)
    code = _dtype_code(factors[0])
    lam = torch.zeros(R, dtype=torch.float64, device="cuda")
    grams = torch.zeros((t.order, R, R), dtype=torch.float64, device="cuda")
    fp = L.ptr_array([f.data_ptr() for f in factors])
    fits, pinv = [], []
    fit = C.c_double()
    used = C.c_int()
    for s in range(sweeps):
        L.check(L.fcoo_cp_als_iter(t.handle, fp, code, R, lam.data_ptr(), grams.data_ptr(),
                                   1 if s > 0 else 0, C.byref(fit), C.byref(used), _stream()))
        fits.append(float(fit.value))
        pinv.append(int(used.value))
        if tol > 0 and s > 0 and abs(fits[-1] - fits[-2]) < tol:
            break
    return dict(factors=factors, lam=lam, fits=fits, used_pinv=pinv, grams=grams)


class CPAtNonzeros:
    """xhat = CPAtNonzeros.apply(t, *factors): the CP model at the nonzeros of
    `t` (input order).  Backward: grad A_m = SpMTTKRP_m with the incoming
    gradient as the values (fcoo_spmttkrp_values), so no Khatri-Rao row is
    stored.  Needs the MTTKRP build of every mode whose gradient is wanted.
    Factors may be float32 or bfloat16; gradients come back in the factor's
    dtype."""

    @staticmethod
    def apply(t: Tensor, *factors):
        return _cp_at_nnz_fn().apply(t, *factors)


class CPMSELoss:
    """loss = CPMSELoss.apply(t, dtype, *master_factors): L = (1/2Z) sum_e
    (xhat_e - x_e)^2 over the nonzeros, as a float64 scalar.  `master_factors`
    are float32; with dtype 'bf16' the kernels read bfloat16 copies of them
    (refreshed on every call) and the gradient flows to the float32 masters.
    The forward pass is the fused residual SpMTTKRP of mode 0 (it yields the
    loss and grad A_0 together); the backward pass runs it for modes 1..N-1."""

    @staticmethod
    def apply(t: Tensor, dtype: str, *factors):
        return _cp_mse_fn().apply(t, dtype, *factors)


_FNS = {}


def _cp_at_nnz_fn():
    if "at" in _FNS:
        return _FNS["at"]
    torch = _torch()

    class _CPAt(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t, *factors):
            ctx.t = t
            ctx.save_for_backward(*factors)
            return t.model_at_nnz(list(factors))

        @staticmethod
        def backward(ctx, g):
            factors = ctx.saved_tensors
            t = ctx.t
            g = g.contiguous().to(torch.float32)
            out = [None]
            for m in range(t.order):
                if ctx.needs_input_grad[m + 1]:
                    fs = [f if k != m else None for k, f in enumerate(factors)]
                    out.append(t.spmttkrp_values(m, g, fs).to(factors[m].dtype))
                else:
                    out.append(None)
            return tuple(out)

    _FNS["at"] = _CPAt
    return _CPAt


def _cp_mse_fn():
    if "mse" in _FNS:
        return _FNS["mse"]
    torch = _torch()

    class _CPMSE(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t, dtype, *masters):
            shadows = [m if dtype == "f32" else m.detach().to(torch.bfloat16).contiguous() for m in masters]
            loss = torch.zeros((), dtype=torch.float64, device="cuda")
            g0 = t.resid_spmttkrp(0, shadows, loss=loss)
            ctx.t = t
            ctx.shadows = shadows
            ctx.g0 = g0
            return loss

        @staticmethod
        def backward(ctx, go):
            t = ctx.t
            scale = go.to(torch.float32)
            grads = [ctx.g0 * scale]
            for m in range(1, t.order):
                grads.append(t.resid_spmttkrp(m, ctx.shadows) * scale)
            ctx.shadows = None
            ctx.g0 = None
            return (None, None) + tuple(grads)

    _FNS["mse"] = _CPMSE
    return _CPMSE
