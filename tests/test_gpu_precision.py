"""The probe-GEMM operand forms against the FP64 oracle on a z-slab of the
384 x 512 x 512 layered model (24 x 512 x 512 cells, nt = 80, r = 128
Rademacher probes, k = 32, a source mid-slab and the full 512 x 512
receiver plane), the case the benchmark's precision section reports:

- bf16 (one MFMA): within the 1e-3 stated for a BF16-probed image;
- bf16 hi + lo (two MFMAs, the default) and the FP32 vector path: at the
  FP32 propagator's level (5e-5, the bar of the compressed FP32 fields);
- float16 after a power-of-two scale per 16-step chunk (one MFMA): 5e-4.

Eq. 3 with the same probes on both sides; the misfit to 1e-5 in every form."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say

pytestmark = pytest.mark.gpu


def test_precision_forms_against_fp64_oracle_on_a_full_extent_slab():
    require_gpu()
    import paper_2201_06914_amd as P
    planes, nt, r, k = 24, 80, 128, 32
    wl = synth.workload_c2(nt=nt, r=r, shape=(planes, 512, 512))
    g = oracle.Grid(3, wl.shape, wl.h, wl.dt, nt, min(wl.nb, (planes - 1) // 2), wl.c_ref, wl.R)
    src = np.array([[planes // 2, 256.0, 256.0]])
    rec = synth.plane_receivers(planes // 2 + 1, 512, 512)
    d_obs = np.zeros((nt, rec.shape[0]))
    say(f"oracle: {wl.shape} nt={nt} r={r} probed gradient")
    J, gref, _, _ = oracle.probed_gradient(g, wl.m, src, wl.q, rec, d_obs, wl.Z)
    m, q = dev(wl.m, torch.float32), dev(wl.q, torch.float32)
    Z, do = dev(wl.Z, torch.int8), dev(d_obs, torch.float32)
    bars = {"bf16": 1e-3, "bf16x2": 5e-5, "f16s": 5e-4, "f32": 5e-5}
    for probe, bar in bars.items():
        plan = P.Plan(P.PlanSpec(3, g.shape, g.h, g.dt, g.nt, g.nb, g.c_ref, g.R, wl.c_ref,
                                 "f32", probe, r, k, 1, rec.shape[0]))
        o = P.fwi_gradient(plan, m, src, q, rec, do, Z, fused=probe != "f32")
        torch.cuda.synchronize()
        e = rel(host(o["grad"]).astype(np.float64), gref)
        eJ = abs(float(o["misfit"].item()) - J) / J
        say(f"  {probe}: gradient vs FP64 oracle {e:.2e} (bar {bar:.0e}), misfit {eJ:.2e}")
        assert e < bar and eJ < 1e-5, (probe, e, eJ)
