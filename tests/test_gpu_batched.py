"""Batched shots on uneven windows (one stencil launch per step for all
shots) and HIP-graph replay, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say
from oracle import Grid

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402

SHAPES = [(24, 22, 40), (30, 26, 35), (20, 34, 47), (28, 19, 64)]


@pytest.fixture(scope="module")
def case():
    require_gpu()
    wls = synth.workload_batched(nt=70, r=32, k_block=16, shapes=SHAPES)
    shots, specs = [], []
    for wl in wls:
        wl.nb = 5
        rec = wl.rec_pos[::5]
        wl.rec_pos = rec
        d_obs = np.zeros((wl.nt, rec.shape[0]), dtype=np.float32)
        specs.append(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, 4725.0,
                                "f32", "bf16x2", wl.r, wl.k_block, 1, rec.shape[0]))
        shots.append(dict(m=dev(wl.m, torch.float32), src_pos=wl.src_pos,
                          q=dev(wl.q, torch.float32), rec_pos=rec,
                          d_obs=dev(d_obs, torch.float32), Z=dev(wl.Z, torch.int8), wl=wl,
                          d_obs_np=d_obs))
    return wls, shots, specs


def test_batched_equals_single_shots_bitwise(case):
    wls, shots, specs = case
    B = P.Batch(specs)
    outs, J = B.fwi_gradient(shots)
    torch.cuda.synchronize()
    for i, (sp, sh) in enumerate(zip(specs, shots)):
        plan = P.Plan(sp)
        one = P.fwi_gradient(plan, sh["m"], sh["src_pos"], sh["q"], sh["rec_pos"], sh["d_obs"],
                             sh["Z"], fused=True)
        torch.cuda.synchronize()
        for k in ("grad", "resid", "Ubar"):
            assert torch.equal(outs[i][k], one[k]), (i, k)
        assert float(J[i].item()) == float(one["misfit"].item()), i
    say(f"  batched == single for {len(specs)} shots")


def test_batched_matches_oracle(case):
    wls, shots, specs = case
    B = P.Batch(specs)
    outs, J = B.fwi_gradient(shots)
    torch.cuda.synchronize()
    for i, (wl, sh) in enumerate(zip(wls, shots)):
        g = Grid.of(wl)
        Jo, go, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, sh["rec_pos"],
                                              sh["d_obs_np"], wl.Z)
        e, eJ = rel(host(outs[i]["grad"]), go), abs(float(J[i].item()) - Jo) / Jo
        say(f"  shot {i} {wl.shape}: grad {e:.2e} misfit {eJ:.2e}")
        assert e < 1e-3 and eJ < 1e-5


def test_graph_replays_equal_eager(case):
    """Capture once, replay three times with eager work and synchronisations
    in between; every replay equals the eager result bit for bit."""
    wls, shots, specs = case
    B = P.Batch(specs)
    ref, Jref = B.fwi_gradient(shots)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in o.items()} for o in ref]
    Jref = Jref.clone()
    outs = B.outputs()
    J = torch.empty(len(shots), dtype=torch.float64, device="cuda")
    work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device="cuda")
    for rep in range(3):
        for o in outs:
            for v in o.values():
                v.fill_(float("nan"))
        J.fill_(float("nan"))
        B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=True, work=work)
        torch.cuda.synchronize()
        for i in range(len(shots)):
            for k in ("grad", "resid", "Ubar"):
                assert torch.equal(outs[i][k], ref[i][k]), (rep, i, k)
        assert torch.equal(J, Jref), rep
        # eager work between replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    say("  3 graph replays == eager")


def test_batch_rejects_mismatched_shots():
    sp = P.PlanSpec(3, (20, 20, 20), 12.5, 1e-3, 10, 3, 3000.0, 1e-3, 3000.0, "f32", "bf16x2",
                    8, 8, 1, 1)
    sp2 = P.PlanSpec(3, (20, 20, 20), 12.5, 1e-3, 11, 3, 3000.0, 1e-3, 3000.0, "f32", "bf16x2",
                     8, 8, 1, 1)
    with pytest.raises(P.RtmError):
        P.Batch([sp, sp2])


def test_batched_long_blocks_work_queue_equal_single_shots_and_oracle():
    """64-step blocks: the forward probe launches of the batch and of the
    single-shot sweeps take their tiles from a work queue (in-place update,
    blocks longer than 32 steps).  The batch equals the single shots bit for
    bit and matches the oracle (Eq. 3 per shot)."""
    require_gpu()
    wls = synth.workload_batched(nt=70, r=32, k_block=64, shapes=SHAPES[:2])
    specs, shots = [], []
    for wl in wls:
        wl.nb = 5
        rec = wl.rec_pos[::5]
        d_obs = (0.02 * np.random.default_rng(4).standard_normal((wl.nt, rec.shape[0]))
                 ).astype(np.float32)
        specs.append(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, 4725.0,
                                "f32", "bf16x2", wl.r, wl.k_block, 1, rec.shape[0]))
        shots.append(dict(m=dev(wl.m, torch.float32), src_pos=wl.src_pos,
                          q=dev(wl.q, torch.float32), rec_pos=rec,
                          d_obs=dev(d_obs, torch.float32), Z=dev(wl.Z, torch.int8),
                          d_obs_np=d_obs))
    say(f"case: batched, k = 64, {len(specs)} shots")
    B = P.Batch(specs)
    outs, J = B.fwi_gradient(shots)
    torch.cuda.synchronize()
    for i, (wl, sp, sh) in enumerate(zip(wls, specs, shots)):
        one = P.fwi_gradient(P.Plan(sp), sh["m"], sh["src_pos"], sh["q"], sh["rec_pos"],
                             sh["d_obs"], sh["Z"], fused=True)
        torch.cuda.synchronize()
        for k in ("grad", "resid", "Ubar"):
            assert torch.equal(outs[i][k], one[k]), (i, k)
        g = Grid.of(wl)
        Jo, go, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, sh["rec_pos"],
                                              sh["d_obs_np"], wl.Z)
        e, eJ = rel(host(outs[i]["grad"]), go), abs(float(J[i].item()) - Jo) / Jo
        say(f"  shot {i} {wl.shape}: batched == single, grad vs oracle {e:.2e}, misfit {eJ:.2e}")
        assert e < 1e-3 and eJ < 1e-5
