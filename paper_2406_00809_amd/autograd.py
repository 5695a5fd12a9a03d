"""torch.autograd binding of the hand-written network backward.

GNPFunction.apply(b, theta, model, prec) returns z = M_theta(b) computed by
gnp_forward_save; its backward calls gnp_backward, which recomputes
A-hat X per layer and returns d<dz, z>/dtheta.  No gradient flows to b.
All arithmetic runs in libgnp; this module only passes pointers.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .api import PREC, Model, _dev_ptr, _stream
from ._lib import check


class GNPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b: torch.Tensor, theta: torch.Tensor, model: Model, prec: str = "f64"):
        p = PREC[prec]
        if p not in (_lib.GNP_F32, _lib.GNP_F64):
            raise ValueError("training precision must be f32 or f64")
        dt = torch.float64 if p == _lib.GNP_F64 else torch.float32
        L = _lib.load()
        st = _stream()
        theta = theta.detach().contiguous()
        check(L.gnp_params_set_device(model.handle, _dev_ptr(theta, torch.float64,
                                                             model.nparams, "theta"),
                                      model.nparams, st))
        nrhs = 1 if b.dim() == 1 else b.shape[1]
        bb = b.detach().to(dt).contiguous()
        z = torch.empty_like(bb)
        check(L.gnp_forward_save(model.handle, _dev_ptr(bb, dt, None, "b"),
                                 _dev_ptr(z, dt, None, "z"), nrhs, p, st))
        ctx.model = model
        ctx.dt = dt
        return z

    @staticmethod
    def backward(ctx, dz: torch.Tensor):
        model = ctx.model
        dzc = dz.detach().to(ctx.dt).contiguous()
        g = torch.empty(model.nparams, dtype=torch.float64, device=dz.device)
        check(_lib.load().gnp_backward(model.handle, _dev_ptr(dzc, ctx.dt, None, "dz"),
                                       _dev_ptr(g, torch.float64, model.nparams, "grad"),
                                       _stream()))
        return None, g, None, None


def gnp(b: torch.Tensor, theta: torch.Tensor, model: Model, prec: str = "f64") -> torch.Tensor:
    return GNPFunction.apply(b, theta, model, prec)
