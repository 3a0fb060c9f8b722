"""Range-finder probes on the GPU (space sketch, orthonormal columns, the
projected gradient) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say
from oracle import Grid

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _plan(wl, field, probe, r, k):
    return P.Plan(P.PlanSpec(wl.ndim, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R,
                             wl.c_ref, field, probe, r, k, int(np.shape(wl.src_pos)[0]),
                             int(np.shape(wl.rec_pos)[0])))


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_sketch_f64_matches_oracle(case):
    if case == "2d":
        wl = synth.workload_small_2d(shape=(30, 34), nt=90, r=8)
        r, k = 12, 16
    else:
        wl = synth.workload_small_3d(shape=(21, 19, 37), nt=70, nb=4, dtype=np.float64)
        r, k = 40, 16
    g = Grid.of(wl)
    say(f"case: sketch F64 {wl.shape} nt={wl.nt} r={r} k={k}")
    Y0 = oracle.sketch(g, wl.m, wl.src_pos, wl.q, 77, r)
    plan = _plan(wl, "f64", "f64", r, k)
    Y = P.rtm_sketch(plan, dev(wl.m, torch.float64), wl.src_pos, dev(wl.q, torch.float64), 77)
    torch.cuda.synchronize()
    e = rel(host(Y), Y0)
    say(f"  sketch F64: {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("r,k", [(48, 32), (32, 64), (100, 16)])
def test_sketch_f32_mfma_matches_oracle(r, k):
    """FP32 levels, u_tt split into bf16 hi + lo on MFMA, FP32 partial sums:
    the norm-wise error is set by u_tt's FP32 rounding (second difference of
    FP32 levels, ~1e-5) and the 16-bit operand mantissa."""
    wl = synth.workload_small_3d(shape=(26, 23, 45), nt=96, nb=5)
    g = Grid.of(wl)
    say(f"case: sketch F32/MFMA {wl.shape} nt={wl.nt} r={r} k={k}")
    Y0 = oracle.sketch(g, wl.m, wl.src_pos, wl.q, 5, r)
    plan = _plan(wl, "f32", "f32", r, k)
    Y = P.rtm_sketch(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), 5)
    torch.cuda.synchronize()
    e = rel(host(Y), Y0)
    say(f"  sketch F32: {e:.2e}")
    assert e < 2e-4


@pytest.mark.parametrize("field", ["f64", "f32"])
def test_orthonormalize_spans_the_columns(field):
    wl = synth.workload_small_2d(shape=(20, 22), nt=150, r=8)
    r = 24
    plan = _plan(wl, field, field, r, 16)
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((wl.nt, r)) @ np.diag(0.7 ** np.arange(r))
    Y[:, 7] = 2.0 * Y[:, 3]                        # a dependent column
    Q = host(P.rtm_orthonormalize(plan, dev(Y, torch.float64)))
    torch.cuda.synchronize()
    tol = 1e-12 if field == "f64" else 2e-6
    assert np.abs(Q[:, 7]).max() == 0.0
    keep = [j for j in range(r) if j != 7]
    Qk = Q[:, keep]
    assert np.abs(Qk.T @ Qk - np.eye(r - 1)).max() < tol
    Pg = Q @ Q.T
    Q0 = oracle.range_finder(Y[:, keep])
    e = np.abs(Pg - Q0 @ Q0.T).max()
    say(f"  orthonormalize {field}: projector diff {e:.2e}")
    assert e < 10 * tol


def test_fwi_gradient_rf_f64_matches_oracle():
    wl = synth.workload_small_2d(shape=(28, 30), nt=100, r=8)
    g = Grid.of(wl)
    r, seed = 16, 9
    d_obs = oracle.forward(g, wl.m * 1.03, wl.src_pos, wl.q, wl.rec_pos)["d"]
    J, g0, Q0, _ = oracle.rf_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, seed, r)
    plan = _plan(wl, "f64", "f64", r, 16)
    out = P.fwi_gradient_rf(plan, dev(wl.m, torch.float64), wl.src_pos,
                            dev(wl.q, torch.float64), wl.rec_pos, dev(d_obs, torch.float64), seed)
    torch.cuda.synchronize()
    e, eJ = rel(host(out["grad"]), g0), abs(float(out["misfit"].item()) - J) / J
    Q = host(out["Q"])
    eP = np.abs(Q @ Q.T - Q0 @ Q0.T).max()
    say(f"  rf gradient F64: grad {e:.2e} misfit {eJ:.2e} projector {eP:.2e}")
    assert e < 1e-9 and eJ < 1e-12 and eP < 1e-9


def test_fwi_gradient_rf_f32_3d_given_its_probes():
    """FP32: the probes Q come from an FP32 sketch, so they are compared through
    the oracle run with the same Q (FP64 probing, scale -1)."""
    wl = synth.workload_small_3d(shape=(24, 22, 38), nt=80, nb=5)
    g = Grid.of(wl)
    r, seed = 32, 4
    rng = np.random.default_rng(6)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    plan = _plan(wl, "f32", "f32", r, 32)
    out = P.fwi_gradient_rf(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                            wl.rec_pos, dev(d_obs, torch.float32), seed)
    torch.cuda.synchronize()
    Q = host(out["Q"]).astype(np.float64)
    assert np.abs(Q.T @ Q - np.eye(r)).max() < 1e-5
    _, g0, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, Q)
    g0 = g0 * r      # probed_gradient scales by -1/r; the range finder uses -1
    e = rel(host(out["grad"]), g0)
    say(f"  rf gradient F32 given Q: {e:.2e}")
    assert e < 1e-4


def test_rf_gradient_bf16x2_fused_given_its_probes():
    """BF16X2 plan: the real probes are split into bf16 hi + lo on MFMA (three
    products per step chunk) and the imaging is fused; compared through the
    oracle run with the GPU's own Q (FP64, scale -1)."""
    wl = synth.workload_small_3d(shape=(24, 22, 38), nt=80, nb=5)
    g = Grid.of(wl)
    r, seed = 32, 4
    rng = np.random.default_rng(6)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    plan = _plan(wl, "f32", "bf16x2", r, 32)
    out = P.fwi_gradient_rf(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                            wl.rec_pos, dev(d_obs, torch.float32), seed)
    torch.cuda.synchronize()
    assert out["Vbar"] is None
    Q = host(out["Q"]).astype(np.float64)
    _, g0, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, Q)
    e = rel(host(out["grad"]), g0 * r)
    say(f"  rf gradient BF16X2 fused given Q: {e:.2e}")
    assert e < 1e-3


@pytest.mark.parametrize("k", [16, 32, 20])
def test_real_probes_on_mfma_equal_fma_path(k):
    """Gaussian probes through fwi_gradient: BF16X2 (MFMA, hi + lo on both
    operands; k = 20 takes the edge kernel) against the FP32 FMA path."""
    wl = synth.workload_small_3d(shape=(20, 18, 40), nt=60, nb=4)
    r = 32
    rng = np.random.default_rng(12)
    Zf = rng.standard_normal((wl.nt, r)).astype(np.float32)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    args = (dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32), dev(Zf, torch.float32))
    gm = P.fwi_gradient(_plan(wl, "f32", "bf16x2", r, k), *args, fused=True)
    gv = P.fwi_gradient(_plan(wl, "f32", "f32", r, k), *args)
    torch.cuda.synchronize()
    e = rel(host(gm["grad"]), host(gv["grad"]))
    say(f"  real probes MFMA vs FMA (k = {k}): {e:.2e}")
    assert e < 2e-4


def test_rf_gradient_equals_exact_when_rank_at_most_r():
    """N = 30 cells <= r = 30 < nt = 80 on the GPU (F64): the projected gradient
    equals the exact checkpointed gradient."""
    wl = synth.workload_small_2d(shape=(6, 5), nt=80, r=8, nb=1)
    wl.src_pos = np.array([[2.0, 0.0, 2.0]])
    wl.rec_pos = np.array([[1.0, 0.0, 1.0], [4.0, 0.0, 3.0]])
    plan = _plan(wl, "f64", "f64", 30, 16)
    d_obs = np.zeros((wl.nt, 2))
    args = (plan, dev(wl.m, torch.float64), wl.src_pos, dev(wl.q, torch.float64), wl.rec_pos,
            dev(d_obs, torch.float64))
    rf = P.fwi_gradient_rf(*args, 5)
    ex = P.fwi_gradient_exact(*args)
    torch.cuda.synchronize()
    e = rel(host(rf["grad"]), host(ex["grad"]))
    say(f"  rf (r = N) vs exact on GPU: {e:.2e}")
    assert e < 1e-9


def test_rf_beats_rademacher_on_gpu():
    wl = synth.workload_small_3d(shape=(30, 26, 44), nt=120, nb=5)
    r = 16
    plan_rf = _plan(wl, "f32", "f32", r, 16)
    plan_z = _plan(wl, "f32", "bf16x2", r, 16)
    rng = np.random.default_rng(8)
    d_obs = (0.1 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    args = (dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32), wl.rec_pos,
            dev(d_obs, torch.float32))
    ex = host(P.fwi_gradient_exact(plan_rf, *args)["grad"])
    gz = host(P.fwi_gradient(plan_z, *args, dev(synth.rademacher(wl.nt, r, 3), torch.int8),
                             fused=True)["grad"])
    gq = host(P.fwi_gradient_rf(plan_rf, *args, 3)["grad"])
    torch.cuda.synchronize()
    ez, eq = rel(gz, ex), rel(gq, ex)
    say(f"  r = {r}: Rademacher {ez:.3f}, range finder {eq:.3f}")
    assert eq < 0.5 * ez


@pytest.mark.parametrize("probe", ["f32", "bf16x2"])
def test_rf_gradient_r_equals_nt_is_the_oracle_exact_gradient(probe):
    """End to end against the oracle without the GPU's Q: with r = nt the
    sketch Y = H Omega has full column rank, Q spans every time direction and
    Q Q^T = I, so the range-finder gradient is the exact gradient of Eq. 2,
    which the oracle computes from stored histories (no probes at all)."""
    wl = synth.workload_small_3d(shape=(22, 20, 34), nt=64, nb=5)
    g = Grid.of(wl)
    r, seed = 64, 12
    rng = np.random.default_rng(8)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    J0, g0 = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    plan = _plan(wl, "f32", probe, r, 32)
    out = P.fwi_gradient_rf(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                            wl.rec_pos, dev(d_obs, torch.float32), seed)
    torch.cuda.synchronize()
    Q = host(out["Q"]).astype(np.float64)
    eI = np.abs(Q @ Q.T - np.eye(wl.nt)).max()
    e = rel(host(out["grad"]), g0)
    eJ = abs(float(out["misfit"].item()) - J0) / J0
    say(f"  rf {probe} r = nt: |Q Q^T - I| {eI:.2e}, grad vs exact {e:.2e}, misfit {eJ:.2e}")
    assert eI < 1e-5 and e < 1e-4 and eJ < 1e-5
