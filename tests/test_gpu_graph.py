"""HIP-graph replay of single-shot gradients (rtm_set_graph): the captured
launch sequence replayed several times, with eager work and synchronisations
between the replays, equals the eager result bit for bit each time; new data
in the same buffers is picked up by a replay, a new buffer starts a new
capture."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["3d-f32-bf16x2-fused", "3d-f32-bf16x2-k64", "2d-f64"])
def test_graph_replays_equal_eager(case):
    """k64: 64-step blocks, whose forward probe launches take their tiles from a
    work queue (a counter reset by a kernel before each launch)."""
    require_gpu()
    import paper_2201_06914_amd as P
    if case.startswith("3d"):
        k64 = case.endswith("k64")
        wl = synth.workload_small_3d(shape=(30, 26, 44), nt=140 if k64 else 70,
                                     r=32 if k64 else 16)
        plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=64 if k64 else None)
        dt, fused = torch.float32, True
    else:
        wl = synth.workload_small_2d(shape=(40, 52), nt=90, r=8)
        plan = P.Plan.for_workload(wl, field="f64", probe="f64")
        dt, fused = torch.float64, False
    say(f"case: graph replay {case}")
    m, q, Z = dev(wl.m, dt), dev(wl.q, dt), dev(wl.Z, torch.int8)
    d_obs = dev(0.01 * np.random.default_rng(3).standard_normal((wl.nt, wl.rec_pos.shape[0])), dt)
    work = plan.workspace()
    bars = (plan.empty_bar(), None if fused else plan.empty_bar())

    def run():
        o = P.fwi_gradient(plan, m, wl.src_pos, q, wl.rec_pos, d_obs, Z, work=work, bars=bars,
                           fused=fused)
        torch.cuda.synchronize()
        return o["grad"].clone(), o["misfit"].clone()
    P.set_graph(False)
    g0, J0 = run()
    try:
        P.set_graph(True)
        for i in range(3):
            g, J = run()                      # capture on the first call, replays after
            assert torch.equal(g, g0) and torch.equal(J, J0), i
            x = torch.randn(1 << 20, device="cuda", dtype=dt)   # eager work between replays
            (x * 2).sum().item()
        # new values in the same buffer: the replay reads them
        d_obs.mul_(1.5)
        P.set_graph(False)
        g1, J1 = run()
        P.set_graph(True)
        g, J = run()
        assert torch.equal(g, g1) and torch.equal(J, J1)
        assert not torch.equal(g1, g0)
        # a new buffer: a new capture, still equal to eager
        d_obs = d_obs.clone()
        g, J = run()
        assert torch.equal(g, g1) and torch.equal(J, J1)
    finally:
        P.set_graph(False)
