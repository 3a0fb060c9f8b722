"""TTI stability checks on the GPU: the screen every TTI call runs before it
writes anything (delta <= eps, plan c_max >= max v sqrt(max(1, 1 + 2 eps))),
and the power-iteration spectral radius of the discrete operator against the
eigenvalues of the oracle's operator assembled as a dense matrix."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, require_gpu, say

pytestmark = pytest.mark.gpu


def _small():
    return synth.workload_tti(shape=(18, 16, 20), nt=40, r=8, sigma=2.0, nb=4, f0=15.0)


def test_screen_rejects_delta_above_eps_and_low_c_max():
    require_gpu()
    import paper_2201_06914_amd as P
    wl, an = _small()
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=wl.c_ref)
    m, q, Z = dev(wl.m, torch.float32), dev(wl.q, torch.float32), dev(wl.Z, torch.int8)
    out = P.rtm_tti_forward_probe(plan, m, dev(an, torch.float32), wl.src_pos, q, wl.rec_pos, Z=Z)
    assert torch.isfinite(out["d"]).all()
    bad = an.copy()
    i = int(np.argmax(bad[0]))            # a cell with eps > 0: delta = eps + 0.01 there
    bad[1].reshape(-1)[i] = bad[0].reshape(-1)[i] + 0.01
    with pytest.raises(P.RtmError) as e:
        P.rtm_tti_forward_probe(plan, m, dev(bad, torch.float32), wl.src_pos, q, wl.rec_pos, Z=Z)
    assert e.value.code == 1 and "delta" in str(e.value)
    # c_max from the velocity alone misses the sqrt(1 + 2 eps) of the fastest
    # direction: give the fastest (salt) cells eps = 0.2 and plan with max v
    v = np.sqrt(1.0 / wl.m.astype(np.float64))
    vmax = float(v.max())
    fast = an.copy()
    fast[0].reshape(-1)[v >= vmax * (1 - 1e-6)] = 0.2
    low = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=vmax)
    with pytest.raises(P.RtmError) as e:
        P.fwi_gradient_tti(low, m, dev(fast, torch.float32), wl.src_pos, q, wl.rec_pos,
                           torch.zeros((wl.nt, wl.rec_pos.shape[0]), device="cuda"), Z, fused=True)
    assert e.value.code == 4
    # the same plan passes where the fastest cells are isotropic (c_max = max v)
    out = P.rtm_tti_forward_probe(low, m, dev(an, torch.float32), wl.src_pos, q, wl.rec_pos, Z=Z)
    assert torch.isfinite(out["d"]).all()
    say(f"screen: delta > eps -> code 1; c_max {vmax:.1f} below {vmax * np.sqrt(1.4):.1f} "
        f"-> code 4")


def test_power_iteration_spectral_radius_matches_dense_oracle_operator():
    require_gpu()
    import paper_2201_06914_amd as P
    sh, h = (6, 7, 8), 12.5
    wl, an = synth.workload_tti(shape=sh, nt=8, r=4, sigma=1.5, nb=1, f0=15.0)
    an = an.astype(np.float64)
    m = wl.m.astype(np.float64)
    N = int(np.prod(sh))
    M = np.zeros((2 * N, 2 * N))
    for j in range(2 * N):
        e = np.zeros(2 * N)
        e[j] = 1.0
        op, oq = oracle.tti_apply(*(a.reshape(sh) for a in an), e[:N].reshape(sh),
                                  e[N:].reshape(sh), h)
        M[:N, j] = op.ravel() / m
        M[N:, j] = oq.ravel() / m
    rho = np.abs(np.linalg.eigvals(M)).max()
    plan = P.Plan.for_workload(wl, field="f64", probe="f64", c_max=wl.c_ref)
    est = P.tti_spectral_radius(plan, dev(m, torch.float64), dev(an, torch.float64), iters=400,
                                seed=3)
    say(f"spectral radius: power iteration {est:.6e}, dense eigenvalues {rho:.6e}")
    assert 0.95 * rho <= est <= 1.02 * rho
    # the leapfrog bound dt <= 2 / sqrt(rho) is at least the plan's dt here
    assert 2.0 / np.sqrt(est) >= wl.dt
