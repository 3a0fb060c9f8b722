"""Exact checkpointed gradient (Eq. 2), the autograd wrapper and finite
differences, on the GPU through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say
from oracle import Grid

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402
from paper_2201_06914_amd.autograd import probed_modeling  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _fwi_2d():
    wl = synth.workload_small_2d(shape=(40, 44), nt=150, r=8)
    g = Grid.of(wl)
    m_true = wl.m
    m0 = synth.smooth(m_true.reshape(40, 44), 3.0).ravel()
    d_obs = oracle.forward(g, m_true, wl.src_pos, wl.q, wl.rec_pos)["d"]
    return wl, g, m0, d_obs


@pytest.mark.parametrize("c", [0, 1, 7, 150])
def test_exact_gradient_matches_oracle_f64(c):
    wl, g, m0, d_obs = _fwi_2d()
    J, ge = oracle.exact_gradient(g, m0, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    plan = P.Plan.for_workload(wl, field="f64", probe="f64")
    out = P.fwi_gradient_exact(plan, dev(m0, torch.float64), wl.src_pos,
                               dev(wl.q, torch.float64), wl.rec_pos,
                               dev(d_obs, torch.float64), checkpoint_every=c)
    torch.cuda.synchronize()
    e = rel(host(out["grad"]), ge)
    eJ = abs(float(out["misfit"].item()) - J) / J
    say(f"  exact f64 c={c}: grad {e:.2e} misfit {eJ:.2e}")
    assert e < 1e-10 and eJ < 1e-12


def test_exact_gradient_f32_3d():
    """FP32: u_tt from FP32 levels carries ~1e-5 relative rounding (second
    difference amplification), so the bar is 1e-4."""
    wl = synth.workload_small_3d(shape=(30, 26, 44), nt=100, nb=5)
    g = Grid.of(wl)
    d_obs = np.zeros((wl.nt, wl.rec_pos.shape[0]), dtype=np.float32)
    J, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    out = P.fwi_gradient_exact(plan, dev(wl.m, torch.float32), wl.src_pos,
                               dev(wl.q, torch.float32), wl.rec_pos,
                               dev(d_obs, torch.float32))
    torch.cuda.synchronize()
    e = rel(host(out["grad"]), ge)
    say(f"  exact f32 3D: grad {e:.2e}")
    assert e < 1e-4


@pytest.mark.parametrize("variant", [1, 7])
def test_exact_fused_epilogue_equals_separate_passes(variant):
    """The u_tt store and the correlation folded into the tiled stencil (with
    the injected increments corrected at source and receiver cells) agree with
    the separate second-difference and correlation passes to FP32 rounding,
    and with the oracle."""
    wl = synth.workload_small_3d(shape=(30, 26, 44), nt=90, nb=5)
    g = Grid.of(wl)
    rng = np.random.default_rng(3)
    d_obs = (0.1 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    args = (plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32))
    P.set_stencil_variant(variant)
    try:
        P.set_exact_fused(False)
        sep = P.fwi_gradient_exact(*args, checkpoint_every=11)
        P.set_exact_fused(True)
        fus = P.fwi_gradient_exact(*args, checkpoint_every=11)
        torch.cuda.synchronize()
    finally:
        P.set_exact_fused(True)
        P.set_stencil_variant(-1)
    e = rel(host(fus["grad"]), host(sep["grad"]))
    J, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    eo = rel(host(fus["grad"]), ge)
    say(f"  exact fused vs separate (variant {variant}): {e:.2e}, vs oracle {eo:.2e}")
    assert e < 2e-6 and eo < 1e-4
    assert torch.equal(fus["resid"], sep["resid"])


def test_probed_with_orthogonal_probes_equals_exact_on_gpu():
    """Both GPU gradients, Hadamard probes with r = nt: identical up to FP32 /
    BF16X2 rounding."""
    nt = 64
    wl = synth.workload_small_3d(shape=(24, 22, 30), nt=nt, nb=4)
    d_obs = np.zeros((nt, wl.rec_pos.shape[0]), dtype=np.float32)
    plan = P.Plan(P.PlanSpec(3, wl.shape, wl.h, wl.dt, nt, wl.nb, wl.c_ref, wl.R, wl.c_ref,
                             "f32", "bf16x2", nt, 32, 1, wl.rec_pos.shape[0]))
    args = (plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32))
    gp = P.fwi_gradient(*args, dev(synth.sylvester_hadamard(nt), torch.int8), fused=True)
    ge = P.fwi_gradient_exact(*args, checkpoint_every=9)
    torch.cuda.synchronize()
    e = rel(host(gp["grad"]), host(ge["grad"]))
    say(f"  hadamard probed vs exact (GPU): {e:.2e}")
    assert e < 2e-4


def test_autograd_gradcheck_f64_orthogonal_probes():
    """torch.autograd.gradcheck of m -> d_pred (FP64, tiny grid).  With
    Z Z^T = r I and r = nt the probed backward is the exact vector-Jacobian
    product; m = m0 (1 + x) makes the finite-difference step relative."""
    nt = 32
    wl = synth.workload_small_2d(shape=(9, 10), nt=nt, nb=2)
    src = np.array([[3.0, 0.0, 4.0]])
    rec = np.array([[3.0, 0.0, 2.0], [4.0, 0.0, 7.0], [6.0, 0.0, 5.0]])
    plan = P.Plan(P.PlanSpec(2, wl.shape, wl.h, wl.dt, nt, 2, wl.c_ref, wl.R, wl.c_ref, "f64",
                             "f64", nt, 8, 1, 3))
    m0 = dev(wl.m, torch.float64)
    q = dev(wl.q, torch.float64)
    Z = dev(synth.sylvester_hadamard(nt), torch.int8)

    def f(x):
        return probed_modeling(plan, m0 * (1.0 + x), src, q, rec, Z)

    x = torch.zeros(plan.N, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-9, rtol=1e-5)


def test_autograd_backward_equals_fwi_gradient():
    wl = synth.workload_small_3d(shape=(26, 24, 34), nt=80, r=32, nb=4)
    g = Grid.of(wl)
    d_obs = oracle.forward(g, wl.m * 1.02, wl.src_pos, wl.q, wl.rec_pos)["d"].astype(np.float32)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=16)
    m = dev(wl.m, torch.float32).requires_grad_(True)
    q, Z, dobs = dev(wl.q, torch.float32), dev(wl.Z, torch.int8), dev(d_obs, torch.float32)
    d = probed_modeling(plan, m, wl.src_pos, q, wl.rec_pos, Z)
    loss = 0.5 * ((d.double() - dobs.double()) ** 2).sum()
    loss.backward()
    ref = P.fwi_gradient(plan, m.detach(), wl.src_pos, q, wl.rec_pos, dobs, Z)
    torch.cuda.synchronize()
    e = rel(host(m.grad), host(ref["grad"]))
    eJ = abs(loss.item() - ref["misfit"].item()) / loss.item()
    say(f"  autograd vs fwi_gradient: grad {e:.2e} misfit {eJ:.2e}")
    assert e < 1e-5 and eJ < 1e-6


def test_exact_gradient_matches_finite_differences_f32():
    """Central differences of the FP64-reduced misfit along a smooth random
    direction against <g_exact, dm> (GPU, FP32 fields)."""
    wl = synth.workload_small_3d(shape=(30, 28, 36), nt=120, nb=5)
    g = Grid.of(wl)
    d_obs = oracle.forward(g, wl.m * 1.03, wl.src_pos, wl.q, wl.rec_pos)["d"].astype(np.float32)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    rng = np.random.default_rng(12)
    dm = synth.smooth(rng.standard_normal(wl.shape), 3.0).ravel()
    dm = (dm / np.abs(dm).max() * 0.01 * wl.m).astype(np.float32)
    q, dobs = dev(wl.q, torch.float32), dev(d_obs, torch.float32)
    ex = P.fwi_gradient_exact(plan, dev(wl.m, torch.float32), wl.src_pos, q, wl.rec_pos, dobs)
    lin = float(np.dot(host(ex["grad"]), dm.astype(np.float64)))
    Zd = dev(wl.Z, torch.int8)
    Js = []
    for sgn in (1.0, -1.0):
        mp = (wl.m + sgn * dm).astype(np.float32)
        Js.append(P.fwi_gradient(plan, dev(mp, torch.float32), wl.src_pos, q, wl.rec_pos, dobs,
                                 Zd)["misfit"].item())
    fd = (Js[0] - Js[1]) / 2.0
    say(f"  FD {fd:.6e} vs <g,dm> {lin:.6e} rel {abs(fd - lin) / abs(lin):.2e}")
    assert abs(fd - lin) < 2e-3 * abs(lin)


def test_probed_error_decreases_with_r():
    """Eq. 1: the probed estimate's error against the exact gradient shrinks
    with r (mean squared error ~ 1/r); averaged over four probe draws."""
    wl = synth.workload_small_3d(shape=(28, 24, 36), nt=100, nb=5)
    d_obs = np.zeros((wl.nt, wl.rec_pos.shape[0]), dtype=np.float32)
    base = dict(m=dev(wl.m, torch.float32), q=dev(wl.q, torch.float32),
                dobs=dev(d_obs, torch.float32))
    errs = {}
    ge = None
    for r in (16, 64):
        plan = P.Plan(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R,
                                 wl.c_ref, "f32", "bf16x2", r, 32, 1, wl.rec_pos.shape[0]))
        if ge is None:
            ge = host(P.fwi_gradient_exact(plan, base["m"], wl.src_pos, base["q"], wl.rec_pos,
                                           base["dobs"])["grad"])
        e2 = []
        for seed in range(4):
            Z = dev(synth.rademacher(wl.nt, r, 50 + seed), torch.int8)
            gp = host(P.fwi_gradient(plan, base["m"], wl.src_pos, base["q"], wl.rec_pos,
                                     base["dobs"], Z, fused=True)["grad"])
            e2.append(rel(gp, ge) ** 2)
        errs[r] = float(np.sqrt(np.mean(e2)))
    say(f"  probed vs exact rms rel error: r=16 {errs[16]:.3f}  r=64 {errs[64]:.3f}")
    assert errs[64] < 0.8 * errs[16]
