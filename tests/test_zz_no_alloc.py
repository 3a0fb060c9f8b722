"""fwi_gradient_noalloc, the gradient entry point for callers that cannot
allocate device memory (its workspace is a static device array of the
library), against fwi_gradient with a caller-owned workspace on the same
seeded inputs: two calls in a row, the second on a smaller grid, so the
second runs on an array that still holds the first call's levels.  Both use
the same kernels and launch shapes, so the outputs agree bit for bit."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, require_gpu, say

pytestmark = pytest.mark.gpu

# (shape, nt, r, fused imaging, Z seed): the first call is the larger
CALLS = [((40, 36, 70), 120, 16, True, 11), ((24, 20, 30), 60, 8, False, 23)]


def _case(shape, nt, r, seed):
    import paper_2201_06914_amd as P
    wl = synth.workload_small_3d(shape=shape, nt=nt, r=r, seed=seed)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    # observed data from a 2 % slower model, so that the residual is not d_pred
    d_obs = P.rtm_forward_probe(plan, dev(wl.m * 1.02, torch.float32), wl.src_pos,
                                dev(wl.q, torch.float32), wl.rec_pos)["d"]
    ins = dict(m=dev(wl.m, torch.float32), src_pos=wl.src_pos, q=dev(wl.q, torch.float32),
               rec_pos=wl.rec_pos, d_obs=d_obs, Z=dev(wl.Z, torch.int8))
    return plan, ins


def test_noalloc_equals_fwi_gradient_on_two_calls():
    require_gpu()
    import paper_2201_06914_amd as P
    cases, refs = [], []
    for shape, nt, r, fused, seed in CALLS:
        plan, ins = _case(shape, nt, r, seed)
        refs.append(P.fwi_gradient(plan, ins["m"], ins["src_pos"], ins["q"], ins["rec_pos"],
                                   ins["d_obs"], ins["Z"], fused=fused))
        cases.append((plan, ins, fused))
    torch.cuda.synchronize()
    outs = []
    for (plan, ins, fused), (shape, nt, r, _, _) in zip(cases, CALLS):
        say(f"fwi_gradient_noalloc: grid {shape}, nt={nt}, r={r}, fused={fused}")
        s = plan.spec
        U = torch.full((plan.Npad // 32, s.r, 32), float("nan"), device="cuda")
        V = None if fused else torch.full_like(U, float("nan"))
        res = torch.full((s.nt, s.nrec), float("nan"), device="cuda")
        g = torch.full((plan.N,), float("nan"), device="cuda")
        J = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        P.fwi_gradient_noalloc(plan, ins["m"], ins["src_pos"], ins["q"], ins["rec_pos"],
                               ins["d_obs"], ins["Z"], (U, V), res, g, J)
        outs.append(dict(grad=g, misfit=J, Ubar=U, Vbar=V, resid=res))
    torch.cuda.synchronize()
    for o, ref, (plan, _, fused) in zip(outs, refs, cases):
        assert torch.isfinite(o["grad"]).all()
        assert float(ref["misfit"].item()) > 0.0
        for key in ("grad", "misfit", "Ubar", "resid") + (() if fused else ("Vbar",)):
            assert torch.equal(o[key], ref[key]), key
    # the static array keeps nothing a later call reads: the larger grid again
    # after the smaller one gives the same result as its first call
    plan, ins, fused = cases[0]
    s = plan.spec
    U = torch.empty((plan.Npad // 32, s.r, 32), device="cuda")
    res = torch.empty((s.nt, s.nrec), device="cuda")
    g = torch.empty((plan.N,), device="cuda")
    J = torch.empty((1,), dtype=torch.float64, device="cuda")
    P.fwi_gradient_noalloc(plan, ins["m"], ins["src_pos"], ins["q"], ins["rec_pos"],
                           ins["d_obs"], ins["Z"], (U, None), res, g, J)
    torch.cuda.synchronize()
    assert torch.equal(g, outs[0]["grad"]) and torch.equal(J, outs[0]["misfit"])
