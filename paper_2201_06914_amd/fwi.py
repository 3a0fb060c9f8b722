"""Multi-shot FWI on one GPU with stacked probed gradients.

The paper's images and gradients are sums over sources, and the probing noise
of each source's estimate (Eq. 3) is independent when every source draws its
own probes, so it averages out in the stack as the fold grows (Section
"Approximate gradient calculations", the remark after Eq. 4; Section
"Discussion and conclusions" on FWI).  This module drives that loop:

  for each iteration:
    - every shot draws a fresh Rademacher probe matrix Z_i (nt x r, +-1);
    - one batched call computes all shots' probed gradients and adds them into
      one stacked gradient (fwi_gradient_batched with a shared buffer), with
      each shot's misfit;
    - a backtracking line search along the negative stacked gradient, scaled
      so that the first trial changes the model by `step` times its largest
      value, keeps the first trial model whose total misfit (forward sweeps
      and rtm_residual) is below the current one, inside [m_min, m_max].

Every wave-equation evaluation runs in the library's kernels; this loop only
updates the model and draws the probes.  With exact=True the stacked gradient
is the exact one (fwi_gradient_exact per shot, summed), for comparison.
"""
from __future__ import annotations

import dataclasses

import torch

from . import api


@dataclasses.dataclass
class Shot:
    src_pos: object      # host [nsrc][3]
    q: torch.Tensor      # device [nt][nsrc]
    rec_pos: object      # host [nrec][3]
    d_obs: torch.Tensor  # device [nt][nrec]


def _misfit(plan: api.Plan, m, shots, work) -> float:
    J = 0.0
    for sh in shots:
        d = api.rtm_forward_probe(plan, m, sh.src_pos, sh.q, sh.rec_pos, work=work)["d"]
        _, Jd = api.rtm_residual(plan, d, sh.d_obs, resid=d, work=work)
        J += float(Jd.item())
    return J


def probes(nt: int, r: int, gen: torch.Generator, device) -> torch.Tensor:
    """A Rademacher probe matrix [nt][r] of int8 +-1 from a torch generator."""
    return (torch.randint(0, 2, (nt, r), generator=gen, device=device, dtype=torch.int8) * 2
            - 1).to(torch.int8)


def fwi(spec: api.PlanSpec, m0: torch.Tensor, shots: list, iters: int, seed: int = 0,
        step: float = 0.05, m_min: float | None = None, m_max: float | None = None,
        exact: bool = False, max_halvings: int = 4, m_true: torch.Tensor | None = None,
        log=None) -> dict:
    """Runs `iters` iterations from m0 (device [N], slowness squared).  spec
    describes every shot's grid (the shots share it).  Returns the final model
    and per-iteration records: misfit before the update, accepted step, trial
    count, and (with m_true) the relative model error."""
    dev = m0.device
    m = m0.clone()
    plan = api.Plan(spec)
    work = plan.workspace(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    if exact:
        ework = torch.empty(api.exact_workspace_bytes(plan), dtype=torch.uint8, device=dev)
    else:
        batch = api.Batch([spec] * len(shots))
        outs = batch.outputs(dev, stack=True)
        bwork = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device=dev)
        Jv = torch.empty(len(shots), dtype=torch.float64, device=dev)
    hist = []

    def model_err():
        if m_true is None:
            return None
        return float(torch.linalg.vector_norm((m - m_true).double())
                     / torch.linalg.vector_norm((m0 - m_true).double()))
    for it in range(iters):
        if exact:
            g = torch.zeros_like(m)
            J0 = 0.0
            for sh in shots:
                o = api.fwi_gradient_exact(plan, m, sh.src_pos, sh.q, sh.rec_pos, sh.d_obs,
                                           work=ework)
                g += o["grad"]
                J0 += float(o["misfit"].item())
        else:
            inputs = [dict(m=m, src_pos=sh.src_pos, q=sh.q, rec_pos=sh.rec_pos, d_obs=sh.d_obs,
                           Z=probes(spec.nt, spec.r, gen, dev)) for sh in shots]
            batch.fwi_gradient(inputs, outs=outs, misfit=Jv, work=bwork)
            g = outs[0]["grad"]
            J0 = float(Jv.sum().item())
        gmax = float(g.abs().max().item())
        if not gmax > 0.0:
            hist.append({"iter": it, "misfit": J0, "alpha": 0.0, "trials": 0,
                         "model_err": model_err()})
            break
        d = -g * (step * float(m.abs().max().item()) / gmax)
        alpha, trials, accepted = 1.0, 0, False
        while trials <= max_halvings:
            trials += 1
            m_try = m + alpha * d
            if m_min is not None or m_max is not None:
                m_try = m_try.clamp(min=m_min, max=m_max)
            J1 = _misfit(plan, m_try, shots, work)
            if J1 < J0:
                m = m_try
                accepted = True
                break
            alpha *= 0.5
        rec = {"iter": it, "misfit": J0, "alpha": alpha if accepted else 0.0, "trials": trials,
               "model_err": model_err()}
        hist.append(rec)
        if log:
            log(rec)
        if not accepted:
            break
    final = _misfit(plan, m, shots, work)
    return {"m": m, "history": hist, "final_misfit": final, "final_model_err": model_err()}
