"""The non-finite watch words (rtm_stream_status, rtm_batch_stream_status) on
the GPU: clean sweeps report OK; a NaN in the model, an infinity in the
observed data or a NaN in the anisotropy reaches the checked values and is
reported; the next clean call on the same workspace clears it."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, require_gpu, say

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def test_forward_nan_model_flagged_then_cleared():
    wl = synth.workload_small_2d(shape=(30, 34), nt=64, r=16)
    plan = P.Plan.for_workload(wl, field="f64", probe="f64")
    work = plan.workspace("cuda")
    q, Z = dev(wl.q, torch.float64), dev(wl.Z, torch.int8)
    m = dev(wl.m, torch.float64)
    P.rtm_forward_probe(plan, m, wl.src_pos, q, wl.rec_pos, Z=Z, work=work)
    ok_clean = P.stream_status(plan, work)
    bad = wl.m.copy()
    bad[15 * 34 + 17] = np.nan
    P.rtm_forward_probe(plan, dev(bad, torch.float64), wl.src_pos, q, wl.rec_pos, Z=Z, work=work)
    ok_nan = P.stream_status(plan, work)
    P.rtm_forward_probe(plan, m, wl.src_pos, q, wl.rec_pos, Z=Z, work=work)
    ok_again = P.stream_status(plan, work)
    say(f"  forward: clean {ok_clean}, NaN model {ok_nan}, clean again {ok_again}")
    assert ok_clean and not ok_nan and ok_again


def test_gradient_inf_data_flagged():
    wl = synth.workload_small_3d(shape=(20, 18, 40), nt=60, nb=4)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    work = plan.workspace("cuda")
    d_obs = np.zeros((wl.nt, wl.rec_pos.shape[0]), dtype=np.float32)
    args = (plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos)
    Z = dev(wl.Z, torch.int8)
    P.fwi_gradient(*args, dev(d_obs, torch.float32), Z, work=work, fused=True)
    ok_clean = P.stream_status(plan, work)
    d_obs[10, 1] = np.inf
    P.fwi_gradient(*args, dev(d_obs, torch.float32), Z, work=work, fused=True)
    ok_inf = P.stream_status(plan, work)
    say(f"  gradient: clean {ok_clean}, Inf in d_obs {ok_inf}")
    assert ok_clean and not ok_inf


def test_tti_nan_anisotropy_flagged():
    wl, an = synth.workload_tti(shape=(18, 16, 20), nt=40, r=8, sigma=2.0, nb=4, f0=15.0,
                                rec_stride=7, dtype=np.float32)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=wl.c_ref)
    from paper_2201_06914_amd.api import tti_workspace
    work = tti_workspace(plan, "cuda")
    m, q, Z = dev(wl.m, torch.float32), dev(wl.q, torch.float32), dev(wl.Z, torch.int8)
    P.rtm_tti_forward_probe(plan, m, dev(an, torch.float32), wl.src_pos, q, wl.rec_pos, Z=Z,
                            work=work)
    ok_clean = P.stream_status(plan, work)
    bad = an.copy()
    bad.reshape(bad.shape[0], -1)[0, 100] = np.nan
    P.rtm_tti_forward_probe(plan, m, dev(bad, torch.float32), wl.src_pos, q, wl.rec_pos, Z=Z,
                            work=work)
    ok_nan = P.stream_status(plan, work)
    say(f"  TTI: clean {ok_clean}, NaN anisotropy {ok_nan}")
    assert ok_clean and not ok_nan


def test_unstable_run_is_flagged():
    """A plan that under-declares c_max by 3x (with a 3x longer dt) passes the
    host CFL check (it sees the same dt c_max / h) but steps the real model
    at three times the stable Courant number (0.77 against the 0.55 bound; the
    Nyquist mode grows ~5x per step): the field overflows FP32 within the 128
    steps and the status word reports it; the honest plan does not."""
    wl = synth.workload_small_2d(shape=(30, 34), nt=128, r=16)

    def plan_of(dt, c_max):
        return P.Plan(P.PlanSpec(2, wl.shape, wl.h, dt, wl.nt, wl.nb, wl.c_ref, wl.R, c_max,
                                 "f32", "f32", 16, 16, int(np.shape(wl.src_pos)[0]),
                                 int(np.shape(wl.rec_pos)[0])))
    res = {}
    for tag, pl in (("honest", plan_of(wl.dt, wl.c_ref)),
                    ("c_max / 3", plan_of(3 * wl.dt, wl.c_ref / 3))):
        work = pl.workspace("cuda")
        P.rtm_forward_probe(pl, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                            wl.rec_pos, work=work)
        res[tag] = P.stream_status(pl, work)
    say(f"  finite: {res}")
    assert res["honest"] and not res["c_max / 3"]


def test_batched_nan_in_one_shot_flagged_then_cleared():
    """The batched gradient's own watch word (rtm_batch_stream_status): clean
    shots leave it clear; a NaN in one shot's model reaches that shot's
    gradient and misfit and sets it; the next clean call on the same
    workspace clears it again (with and without graph replay)."""
    shapes = [(20, 18, 40), (24, 22, 33)]
    wls = synth.workload_batched(nt=48, r=16, k_block=16, shapes=shapes)
    shots, specs = [], []
    for wl in wls:
        wl.nb = 4
        rec = wl.rec_pos[::7]
        d_obs = np.zeros((wl.nt, rec.shape[0]), dtype=np.float32)
        specs.append(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, 4725.0,
                                "f32", "bf16x2", wl.r, wl.k_block, 1, rec.shape[0]))
        shots.append(dict(m=dev(wl.m, torch.float32), src_pos=wl.src_pos,
                          q=dev(wl.q, torch.float32), rec_pos=rec,
                          d_obs=dev(d_obs, torch.float32), Z=dev(wl.Z, torch.int8)))
    B = P.Batch(specs)
    work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device="cuda")
    res = {}
    for graph in (False, True):
        outs = B.outputs("cuda")
        B.fwi_gradient(shots, outs=outs, work=work, use_graph=graph)
        res[("clean", graph)] = B.stream_status(work)
        good = shots[1]["m"].clone()
        nz, ny, nx = shapes[1]
        shots[1]["m"].view(nz, ny, nx)[nz // 2, ny // 2, nx // 2] = float("nan")
        B.fwi_gradient(shots, outs=outs, work=work, use_graph=graph)
        res[("nan", graph)] = B.stream_status(work)
        shots[1]["m"].copy_(good)
        B.fwi_gradient(shots, outs=outs, work=work, use_graph=graph)
        res[("again", graph)] = B.stream_status(work)
    say("  batched watch word: " + ", ".join(f"{k[0]}{'/graph' if k[1] else ''} {v}"
                                              for k, v in res.items()))
    for graph in (False, True):
        assert res[("clean", graph)] and not res[("nan", graph)] and res[("again", graph)]
