"""Grid caps of the probe-GEMM launches (rtm_set_probe_grid): every tile's
arithmetic is the same whether a wave strides over many tiles, each
workgroup takes four tiles and exits, or the waves take tiles from a work
queue, so the compressed fields, the image and the gradient are equal bit
for bit across caps."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import dev, require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fused,probe,k", [(True, "bf16x2", 32), (False, "bf16x2", 32),
                                           (True, "bf16x2", 64), (False, "bf16x2", 64),
                                           (False, "f16s", 64), (True, "f16s", 32)])
def test_probe_grid_caps_give_identical_results(fused, probe, k):
    require_gpu()
    import paper_2201_06914_amd as P
    # 2880 full 32-cell tiles plus none ragged; r = 64 (two row-tile pairs);
    # k = 64: the automatic launches of the forward blocks use the work queue
    wl = synth.workload_small_3d(shape=(40, 36, 64), nt=140 if k == 64 else 70, r=64)
    plan = P.Plan.for_workload(wl, field="f32", probe=probe, k_block=k)
    m, q, Z = dev(wl.m, torch.float32), dev(wl.q, torch.float32), dev(wl.Z, torch.int8)
    d_obs = dev(0.01 * np.random.default_rng(5).standard_normal((wl.nt, wl.rec_pos.shape[0])),
                torch.float32)
    say(f"case: probe grid caps, {wl.shape}, r={wl.r}, k={k}, {probe}, fused={fused}")
    out = {}
    try:
        # 8: every wave strides over ~90 tiles; 0: no stride; then the defaults
        for caps in ((8, 8), (0, 0), (-1, -1), (2048, 2048), (-2, -2)):
            P.set_probe_grid(*caps)
            o = P.fwi_gradient(plan, m, wl.src_pos, q, wl.rec_pos, d_obs, Z, fused=fused)
            torch.cuda.synchronize()
            out[caps] = o
    finally:
        P.set_probe_grid(-1, -1)  # the defaults (automatic)
    ref = out[(8, 8)]
    for caps, o in out.items():
        assert torch.equal(o["grad"], ref["grad"]), caps
        assert torch.equal(o["misfit"], ref["misfit"]), caps
        if not fused:
            assert torch.equal(o["Vbar"], ref["Vbar"]), caps
        assert torch.equal(o["Ubar"], ref["Ubar"]), caps
    say("  probe grid caps (8, 8), (0, 0), automatic, (2048, 2048), work queue: equal bit for bit")
