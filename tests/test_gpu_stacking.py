"""Stacking over sources and the FWI loop on the GPU.

- fwi_gradient_batched with one gradient buffer shared by all shots returns
  the stack (sum over shots, each shot with its own probes), equal to the sum
  of the shots' separate gradients and to the oracle's stack on the same
  probes (Eq. 3 per shot, summed).
- The batched call's non-finite watch word reports a NaN in one shot's model.
- rtm_residual equals the oracle's misfit.
- The FWI loop with stacked probed gradients lowers the misfit every
  iteration, and so does the same loop with exact gradients.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, rel, require_gpu, say

pytestmark = pytest.mark.gpu

SHAPE, NT, R = (30, 28, 44), 90, 8
XS = (10.0, 22.0, 34.0)


def _shots(wl, m_obs_host):
    """Three sources along x on one grid; observed data from m_obs."""
    import paper_2201_06914_amd as P
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    shots = []
    for i, x in enumerate(XS):
        src = np.array([[wl.nb + 2.0, SHAPE[1] // 2, x]])
        d_obs = P.rtm_forward_probe(plan, dev(m_obs_host, torch.float32), src,
                                    dev(wl.q, torch.float32), wl.rec_pos)["d"]
        shots.append(dict(m=dev(wl.m, torch.float32), src_pos=src, q=dev(wl.q, torch.float32),
                          rec_pos=wl.rec_pos, d_obs=d_obs,
                          Z=dev(synth.rademacher(NT, R, 40 + i), torch.int8)))
    return plan, shots


def test_stacked_batched_gradient_is_the_sum_of_shots_and_matches_oracle():
    require_gpu()
    import paper_2201_06914_amd as P
    wl = synth.workload_small_3d(shape=SHAPE, nt=NT, r=R, seed=31)
    plan, shots = _shots(wl, wl.m * 0.97)
    spec = plan.spec
    say(f"stacking: {len(shots)} shots on {SHAPE}, nt={NT}, r={R}")
    B = P.Batch([spec] * len(shots))
    sep, Jsep = B.fwi_gradient(shots, outs=B.outputs())
    stk_outs = B.outputs(stack=True)
    assert all(o["grad"] is stk_outs[0]["grad"] for o in stk_outs)
    stk, Jstk = B.fwi_gradient(shots, outs=stk_outs)
    torch.cuda.synchronize()
    gsum = sum(o["grad"].double() for o in sep)
    gstk = stk[0]["grad"].double()
    assert torch.equal(Jsep, Jstk)
    assert rel(gstk.cpu().numpy(), gsum.cpu().numpy()) < 1e-5
    # the oracle's stack on the same probes (FP64)
    g = oracle.Grid.of(wl)
    oshots = [(sh["src_pos"], wl.q.astype(np.float64), wl.rec_pos,
               sh["d_obs"].double().cpu().numpy()) for sh in shots]
    Zs = [sh["Z"].cpu().numpy() for sh in shots]
    J, G = oracle.stacked_probed_gradient(g, wl.m.astype(np.float64), oshots, Zs)
    e = rel(gstk.cpu().numpy(), G)
    say(f"stacked gradient vs oracle: {e:.2e}; misfit {float(Jstk.sum()):.6e} vs {J:.6e}")
    assert e < 1e-3
    # the misfit is 1/2 |d_pred - d_obs|^2: an error of relative size 1e-5 in
    # the FP32 traces (the propagator's bar) moves it by at most about
    # 2e-5 |d_pred| / |resid| relative
    res = torch.cat([o["resid"].reshape(-1) for o in stk]).double()
    dp = res + torch.cat([sh["d_obs"].reshape(-1) for sh in shots]).double()
    amp = float(torch.linalg.vector_norm(dp) / torch.linalg.vector_norm(res))
    say(f"misfit: rel diff {abs(float(Jstk.sum()) / J - 1):.2e}, |d_pred| / |resid| = {amp:.1f}")
    assert float(Jstk.sum()) == pytest.approx(J, rel=2e-5 * amp)


def test_batched_watch_word_reports_nan_model():
    require_gpu()
    import paper_2201_06914_amd as P
    wl = synth.workload_small_3d(shape=SHAPE, nt=NT, r=R, seed=31)
    plan, shots = _shots(wl, wl.m * 0.97)
    B = P.Batch([plan.spec] * len(shots))
    work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device="cuda")
    outs = B.outputs(stack=True)
    B.fwi_gradient(shots, outs=outs, work=work)
    assert B.stream_status(work)
    bad = shots[1]["m"].clone()
    bad[1234] = float("nan")
    shots[1] = dict(shots[1], m=bad)
    B.fwi_gradient(shots, outs=outs, work=work)
    assert not B.stream_status(work)
    shots[1] = dict(shots[1], m=shots[0]["m"])
    B.fwi_gradient(shots, outs=outs, work=work)
    assert B.stream_status(work)


def test_rtm_residual_matches_oracle_misfit():
    require_gpu()
    import paper_2201_06914_amd as P
    wl = synth.workload_small_2d(shape=(40, 50), nt=120, r=4)
    plan = P.Plan.for_workload(wl, field="f64", probe="f64")
    rng = np.random.default_rng(5)
    d = rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))
    d_obs = rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))
    res, J = P.rtm_residual(plan, dev(d, torch.float64), dev(d_obs, torch.float64))
    Jo, reso = oracle.misfit(d, d_obs)
    assert float(J.item()) == pytest.approx(Jo, rel=1e-13)
    np.testing.assert_array_equal(res.cpu().numpy(), reso)


@pytest.mark.parametrize("exact", [False, True], ids=["probed", "exact"])
def test_fwi_loop_lowers_the_misfit(exact):
    require_gpu()
    import paper_2201_06914_amd as P
    from paper_2201_06914_amd import fwi
    wl = synth.workload_small_3d(shape=SHAPE, nt=NT, r=16, seed=31)
    v = 1.0 / np.sqrt(wl.m.astype(np.float64)).reshape(SHAPE)
    z, y, x = np.ogrid[:SHAPE[0], :SHAPE[1], :SHAPE[2]]
    blob = ((z - 18) / 5.0) ** 2 + ((y - 14) / 6.0) ** 2 + ((x - 22) / 8.0) ** 2 <= 1.0
    v_true = np.where(blob, v * 1.15, v)
    m_true = (1.0 / v_true ** 2).astype(np.float32).ravel()
    plan, shots = _shots(wl, m_true)
    m_min, m_max = float(m_true.min()) * 0.8, float(m_true.max()) * 1.2
    # the CFL check covers every model the loop may reach (m >= m_min)
    spec = dataclasses.replace(plan.spec, r=16, c_max=1.0 / np.sqrt(m_min))
    fs = [fwi.Shot(sh["src_pos"], sh["q"], sh["rec_pos"], sh["d_obs"]) for sh in shots]
    m0 = dev(wl.m, torch.float32)
    out = fwi.fwi(spec, m0, fs, iters=3, seed=7, step=0.03, exact=exact, m_min=m_min,
                  m_max=m_max, m_true=dev(m_true, torch.float32))
    h = out["history"]
    say(f"fwi ({'exact' if exact else 'probed'}): " +
        ", ".join(f"{r['misfit']:.4e}/a={r['alpha']}" for r in h) +
        f", final {out['final_misfit']:.4e}, model err {out['final_model_err']:.4f}")
    assert len(h) == 3 and all(r["alpha"] > 0 for r in h)
    js = [r["misfit"] for r in h] + [out["final_misfit"]]
    assert all(b < a for a, b in zip(js, js[1:])), js
    assert js[-1] < 0.6 * js[0], js
    # three short steps: the model moves little, and not away from the truth
    assert out["final_model_err"] < 1.01
