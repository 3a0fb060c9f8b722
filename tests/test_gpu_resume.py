"""Checkpoint / resume of the forward sweep through rtm_forward_probe_range:
a sweep split into ranges at probe-block boundaries, each resumed from the
previous range's state and partial Ubar, equals the uninterrupted sweep bit
for bit (data, compressed field, final state)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, host, require_gpu, say

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _case(kind):
    if kind == "3d-f32-bf16x2":
        wl = synth.workload_small_3d(shape=(22, 20, 44), nt=90, nb=4)
        plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=16)
        t = torch.float32
    else:
        wl = synth.workload_small_2d(shape=(30, 34), nt=70, r=16)
        plan = P.Plan.for_workload(wl, field="f64", probe="f64", k_block=8)
        t = torch.float64
    return wl, plan, t


@pytest.mark.parametrize("kind,cuts", [("3d-f32-bf16x2", [48]), ("3d-f32-bf16x2", [16, 64]),
                                       ("2d-f64", [24, 40, 64])])
def test_split_sweep_equals_whole_sweep_bitwise(kind, cuts):
    wl, plan, t = _case(kind)
    m, q, Z = dev(wl.m, t), dev(wl.q, t), dev(wl.Z, torch.int8)
    work = plan.workspace("cuda")
    whole = P.rtm_forward_probe(plan, m, wl.src_pos, q, wl.rec_pos, Z=Z, final=True, work=work)
    bounds = [0] + cuts + [wl.nt]
    out = None
    for a, b in zip(bounds[:-1], bounds[1:]):
        out = P.rtm_forward_probe_range(
            plan, m, wl.src_pos, q, wl.rec_pos, Z, a, b,
            state_in=None if out is None else out["state"],
            Ubar=None if out is None else out["Ubar"], d=None if out is None else out["d"],
            work=work)
    torch.cuda.synchronize()
    same = {k: np.array_equal(host(whole[k]), host(out[k2]))
            for k, k2 in (("d", "d"), ("Ubar", "Ubar"), ("final", "state"))}
    say(f"  resume {kind} cuts {cuts}: {same}")
    assert all(same.values())
