"""``torch.autograd.Function`` around the multidirect loop and its adjoint.

Forward: ``ib_multidirect_force`` (keeping F^1..F^ns).  Backward:
``ib_multidirect_backward``, the hand-written reverse sweep that recomputes
the intermediate fields from u0 and F^m.  Differentiable inputs: the velocity
field u0 (box layout, plan precision), the particles' U_r and W_r (FP64
[np][3]) and the marker positions X (FP64 [nl][3]).  The buckets must have
been built from the same X (bucketing is integer and carries no gradient).
"""
from __future__ import annotations

import torch

from . import ibx


class MultidirectFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, up, om, X, plan, level, xc, d, pid, dv, offs, buckets, ns, dt):
        X = X.detach().contiguous()
        m = ibx.Markers(offs, X[:, 0].contiguous(), X[:, 1].contiguous(),
                        X[:, 2].contiguous(), pid, dv)
        parts = ibx.Particles(xc, d, up.detach().contiguous(), om.detach().contiguous())
        Fhist = torch.empty((max(ns, 1), m.nl, 3), dtype=u0.dtype, device=u0.device)
        ustar, f, F = plan.multidirect_force(level, parts, m, buckets, ns, dt,
                                             u0.detach().contiguous(), Fhist=Fhist)
        ctx.save_for_backward(u0.detach(), Fhist)
        ctx.state = (plan, level, parts, m, buckets, ns, dt)
        return ustar, f, F

    @staticmethod
    def backward(ctx, g_ustar, g_f, g_F):
        u0, Fhist = ctx.saved_tensors
        plan, level, parts, m, buckets, ns, dt = ctx.state
        c = lambda t: None if t is None else t.contiguous()
        g_u0, g_up, g_om, g_X = plan.backward(level, parts, m, buckets, ns, dt, u0, Fhist,
                                              g_ustar=c(g_ustar), g_f=c(g_f), g_F=c(g_F))
        return (g_u0, g_up, g_om, g_X) + (None,) * 10


def multidirect(plan, level, parts, markers, buckets, ns, dt, u0, up=None, om=None, X=None):
    """Differentiable multidirect forcing: returns (ustar, f, F)."""
    up = parts.up if up is None else up
    om = parts.om if om is None else om
    X = markers.xyz() if X is None else X
    return MultidirectFunction.apply(u0, up, om, X, plan, level, parts.xc, parts.d,
                                     markers.pid, markers.dv, markers.offs, buckets, ns, dt)
