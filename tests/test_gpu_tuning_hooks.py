"""Tuning hooks that change launch geometry or memory hints only: the z split
of the tiled acoustic stencil (rtm_set_stencil_blocks), the direction of its
z-march (rtm_set_stencil_alternate), the z split of the tiled TTI steps
(rtm_set_tti_blocks), non-temporal probe traffic (rtm_set_probe_nt) and
per-kernel profiling (rtm_profile_enable).  Each cell's arithmetic is the
same however z is cut into chunks, whichever way a chunk is marched and
whatever the cache hints, so the data, Ubar and the gradient are equal bit
for bit across every setting."""
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


def test_stencil_z_split_and_march_direction_bitwise():
    """(70, 30, 90): 1, 2 and 4 z-chunks (at least 16 planes each), ragged
    tiles in x and y, marched upwards only or alternately."""
    wl = synth.workload_small_3d(shape=(70, 30, 90), nt=60, r=16, nb=5)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=16)
    rng = np.random.default_rng(3)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    args = (plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32), dev(wl.Z, torch.int8))
    out = {}
    try:
        P.set_stencil_variant(13)
        for blocks in (1, 8, 100000):
            for alt in (True, False):
                P.set_stencil_blocks(blocks)
                P.set_stencil_alternate(alt)
                out[(blocks, alt)] = P.fwi_gradient(*args, fused=True)
                torch.cuda.synchronize()
    finally:
        P.set_stencil_variant(-1)
        P.set_stencil_blocks(0)
        P.set_stencil_alternate(True)
    ref = out[(1, False)]
    for key, o in out.items():
        for k in ("resid", "Ubar", "grad"):
            assert torch.equal(o[k], ref[k]), (key, k)
        assert float(o["misfit"].item()) == float(ref["misfit"].item()), key
    say(f"  stencil: {len(out)} z-split / march settings equal bit for bit")


def test_tti_z_split_bitwise():
    """(70, 27, 75): the tiled TTI steps with 1, 2 and 4 z-chunks each
    (warm-up planes re-marched per chunk) and the default targets."""
    wl, an = synth.workload_tti(shape=(70, 27, 75), nt=40, r=16, sigma=3.0, nb=5, f0=12.0,
                                rec_stride=4)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=wl.c_ref)
    rng = np.random.default_rng(4)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    args = (plan, dev(wl.m, torch.float32), dev(an, torch.float32), wl.src_pos,
            dev(wl.q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
            dev(wl.Z, torch.int8))
    out = {}
    try:
        for tf, ta in ((1, 1), (28, 16), (100000, 100000), (0, 0), (1, 100000)):
            P.set_tti_blocks(tf, ta)
            out[(tf, ta)] = P.fwi_gradient_tti(*args, fused=True)
            torch.cuda.synchronize()
    finally:
        P.set_tti_blocks(0, 0)
    ref = out[(1, 1)]
    for key, o in out.items():
        for k in ("resid", "Ubar", "grad"):
            assert torch.equal(o[k], ref[k]), (key, k)
    say(f"  TTI: {len(out)} z-split settings equal bit for bit")


def test_probe_nt_and_profiling_bitwise():
    """Non-temporal compressed-field traffic in the probe kernels on or off
    (rtm_set_probe_nt) and per-kernel HIP-event profiling on or off
    (rtm_profile_enable) leave the results unchanged bit for bit."""
    wl = synth.workload_small_3d(shape=(40, 36, 70), nt=60, r=16, nb=5)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=16)
    rng = np.random.default_rng(5)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    args = (plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32), dev(wl.Z, torch.int8))
    out = {}
    try:
        for nt_on in (True, False):
            for prof in (0, 1):
                P.set_probe_nt(nt_on)
                P.profile_enable(prof)
                out[(nt_on, prof)] = P.fwi_gradient(*args, fused=True)
                torch.cuda.synchronize()
                if prof:
                    ms, n = P.profile_read("stencil")
                    assert n > 0 and ms > 0.0
    finally:
        P.set_probe_nt(True)
        P.profile_enable(0)
    ref = out[(True, 0)]
    for key, o in out.items():
        for k in ("resid", "Ubar", "grad"):
            assert torch.equal(o[k], ref[k]), (key, k)
    say(f"  probe non-temporal / profiling: {len(out)} settings equal bit for bit")
