"""torch.autograd.Function over the hand-written SPH adjoint kernels.

``acceleration(x, v, m, ...)`` returns the force loop's accelerations a(x, v, m)
(float64) with the density computed inside; its backward calls the HIP adjoint
kernels (force adjoint, which recomputes the density, then density adjoint)
through the C-ABI.  h, u, the viscosity switch alpha~ and alpha_d are
constants.  All arithmetic runs in the
library's kernels; this module only allocates tensors and marshals pointers.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import sph


class _Ctx:
    def __init__(self, plan: sph.Plan, h, u, atilde, alpha_d, params=None):
        self.plan = plan
        self.h = h.contiguous()
        self.u = u.contiguous()
        self.atilde = atilde.contiguous()
        self.alpha_d = alpha_d.contiguous()
        self.params = params if params is not None else sph.default_params()
        b = C.c_size_t()
        sph._check(sph.lib().sph_adjoint_ws_bytes(plan.ptr, C.byref(b)), "sph_adjoint_ws_bytes")
        self.ws = torch.empty(b.value, dtype=torch.uint8, device=h.device)


def _p(t):
    return t.data_ptr()


def adjoint_forward(ctx: _Ctx, x, v, m):
    n = x.shape[0]
    dev = x.device
    rho = torch.empty(n, dtype=torch.float64, device=dev)
    rdh = torch.empty(n, dtype=torch.float64, device=dev)
    a = torch.empty(n, 3, dtype=torch.float64, device=dev)
    udt = torch.empty(n, dtype=torch.float64, device=dev)
    L = sph.lib()
    sph._check(L.sph_adjoint_forward(ctx.plan.ptr, _p(x), _p(v), _p(m), _p(ctx.h), _p(ctx.u), _p(ctx.atilde),
                                     _p(ctx.alpha_d), C.byref(ctx.params), _p(rho), _p(rdh), _p(a), _p(udt),
                                     _p(ctx.ws), ctx.ws.numel(), sph._stream(None)), "sph_adjoint_forward")
    return a, rho, rdh, udt


def adjoint_backward(ctx: _Ctx, x, v, m, a_bar):
    n = x.shape[0]
    dev = x.device
    xb = torch.empty(n, 3, dtype=torch.float64, device=dev)
    vb = torch.empty(n, 3, dtype=torch.float64, device=dev)
    mb = torch.empty(n, dtype=torch.float64, device=dev)
    rb = torch.empty(n, dtype=torch.float64, device=dev)
    db = torch.empty(n, dtype=torch.float64, device=dev)
    a_bar = a_bar.contiguous().to(torch.float64)
    L = sph.lib()
    sph._check(L.sph_force_adjoint(ctx.plan.ptr, _p(x), _p(v), _p(m), _p(ctx.h), _p(ctx.u), _p(ctx.atilde),
                                   _p(ctx.alpha_d), C.byref(ctx.params), _p(a_bar), _p(xb), _p(vb), _p(mb),
                                   _p(rb), _p(db), _p(ctx.ws), ctx.ws.numel(), sph._stream(None)),
               "sph_force_adjoint")
    sph._check(L.sph_density_adjoint(ctx.plan.ptr, _p(x), _p(m), _p(ctx.h), _p(rb), _p(db), _p(xb), _p(mb),
                                     _p(ctx.ws), ctx.ws.numel(), sph._stream(None)), "sph_density_adjoint")
    return xb, vb, mb


class SphAcceleration(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, v, m, ctx: _Ctx):
        x = x.contiguous()
        v = v.contiguous()
        m = m.contiguous()
        a, _, _, _ = adjoint_forward(ctx, x, v, m)
        fctx.save_for_backward(x, v, m)
        fctx.sph = ctx
        return a

    @staticmethod
    def backward(fctx, a_bar):
        x, v, m = fctx.saved_tensors
        xb, vb, mb = adjoint_backward(fctx.sph, x, v, m, a_bar)
        return xb.to(x.dtype), vb.to(v.dtype), mb.to(m.dtype), None


def make_context(plan: sph.Plan, h, u, atilde, alpha_d, params=None) -> _Ctx:
    return _Ctx(plan, h, u, atilde, alpha_d, params)


def acceleration(x, v, m, ctx: _Ctx):
    """a(x, v, m): x float64 [n,3], v float32 [n,3], m float32 [n] on the GPU."""
    return SphAcceleration.apply(x, v, m, ctx)
