"""Differentiable probed modelling: m -> d_pred with a hand-written backward.

forward:  rtm_forward_probe (traces d_pred, compressed u_tt history Ubar)
backward: rtm_adjoint_probe driven by the incoming trace gradient, then the
          probed imaging condition with scale -1/r (Eq. 3), i.e. the
          randomized-trace estimate of the vector-Jacobian product
          -sum_n u_tt^n lam^n of Eq. 2.  With BF16 probe paths the imaging
          is folded into the adjoint probe blocks (Vbar never stored).

With orthogonal probes and r = nt (Z Z^T = r I) the backward is the exact
vector-Jacobian product of the discrete forward map, which is what
torch.autograd.gradcheck checks.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import (Plan, _check, _dev, _pos, _stream, _work, _z, rtm_adjoint_probe,
                  rtm_forward_probe, rtm_image)


def _adjoint_image_fused(plan: Plan, m, rec_pos, res, Z, Ubar, work=None) -> torch.Tensor:
    """Adjoint sweep with the imaging condition folded into its probe blocks."""
    s = plan.spec
    dev = m.device
    g = torch.empty(plan.N, dtype=plan.dtype, device=dev)
    work = _work(plan, work, dev)
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    zp, zt = _z(plan, Z)
    _check(_lib.load().rtm_adjoint_image(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), rpp,
        _dev(res, plan.dtype, s.nt * s.nrec, "res"), zp, zt,
        _dev(Ubar, plan.dtype, s.r * plan.Npad, "Ubar"), -1.0 / s.r,
        _dev(g, plan.dtype, plan.N, "image"), ctypes.c_void_p(work.data_ptr()), work.numel(),
        _stream(dev)), "rtm_adjoint_image")
    return g


class ProbedModeling(torch.autograd.Function):
    """d_pred = F(m); grad_m = probed adjoint-state gradient of <grad_d, F(m)>."""

    @staticmethod
    def forward(ctx, m, plan: Plan, src_pos, q, rec_pos, Z, work=None):
        out = rtm_forward_probe(plan, m.detach(), src_pos, q, rec_pos, Z=Z, what="utt",
                                work=work)
        ctx.save_for_backward(m.detach(), out["Ubar"], Z)
        ctx.plan, ctx.rec_pos, ctx.work = plan, rec_pos, work
        return out["d"]

    @staticmethod
    def backward(ctx, grad_d):
        m, Ubar, Z = ctx.saved_tensors
        plan = ctx.plan
        res = grad_d.detach().to(plan.dtype).contiguous()
        if plan.spec.probe in ("bf16", "bf16x2", "f16s"):
            g = _adjoint_image_fused(plan, m, ctx.rec_pos, res, Z, Ubar, ctx.work)
        else:
            V = rtm_adjoint_probe(plan, m, ctx.rec_pos, res, Z=Z, work=ctx.work)["Vbar"]
            g = rtm_image(plan, Ubar, V, scale=-1.0 / plan.spec.r)
        return g, None, None, None, None, None, None


def probed_modeling(plan: Plan, m, src_pos, q, rec_pos, Z, work=None) -> torch.Tensor:
    """Differentiable forward modelling; see ProbedModeling."""
    return ProbedModeling.apply(m, plan, src_pos, q, rec_pos, Z, work)
