"""Pseudo-acoustic TTI on the GPU (through the C ABI) against the FP64 oracle."""
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


def _plan(wl, field, probe, nrec=None, k_block=16):
    return P.Plan(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, wl.c_ref,
                             field, probe, wl.r, k_block, 1,
                             wl.rec_pos.shape[0] if nrec is None else nrec))


def _rows(plan, bar2):
    return np.stack([host(P.rtm_bar_to_rows(plan, bar2[f])) for f in range(2)])


@pytest.fixture
def variant(request):
    """(stencil variant, TTI tile shape) for the test's duration: variant -1
    lets the library pick (the tiled TTI kernels, in the given tile shape), 0
    forces the one-thread-per-cell kernels."""
    v, sh = request.param
    P.set_stencil_variant(v)
    P.set_tti_shape(sh)
    yield request.param
    P.set_stencil_variant(-1)
    P.set_tti_shape(21)  # the default


@pytest.mark.parametrize("variant,shape", [((-1, 1), (18, 16, 20)), ((0, 1), (18, 16, 20)),
                                           ((-1, 1), (40, 21, 70)), ((-1, 2), (40, 21, 70)),
                                           ((-1, 3), (40, 21, 70)), ((-1, 4), (40, 21, 70)),
                                           ((-1, 5), (40, 21, 70)), ((-1, 6), (40, 21, 70)),
                                           ((-1, 6), (18, 16, 20)), ((-1, 7), (40, 21, 70)),
                                           ((-1, 8), (40, 21, 70)), ((-1, 9), (40, 21, 70)),
                                           ((-1, 9), (18, 16, 20)), ((-1, 10), (40, 21, 70)),
                                           ((-1, 11), (40, 21, 70)), ((-1, 11), (18, 16, 20)),
                                           ((-1, 12), (40, 21, 70)), ((-1, 13), (37, 21, 70)),
                                           ((-1, 14), (37, 21, 70)), ((-1, 15), (37, 21, 70)),
                                           ((-1, 15), (18, 16, 20)), ((-1, 16), (37, 21, 70)),
                                           ((-1, 16), (18, 16, 20)), ((-1, 17), (37, 21, 70)),
                                           ((-1, 17), (18, 16, 20)), ((-1, 18), (37, 21, 70)),
                                           ((-1, 19), (37, 21, 70)), ((-1, 19), (18, 16, 20)),
                                           ((-1, 20), (37, 21, 70)), ((-1, 21), (37, 21, 70))],
                         indirect=["variant"])
def test_tti_f64_forward_adjoint_gradient_match_oracle(variant, shape):
    """(40, 21, 70): two z-chunks, ragged tiles in x and y for the tiled kernels
    (tile shapes 1..3: 64 x 8 and 64 x 4 columns; 4, 5: fused forward step; 6:
    both steps fused; 7, 8: both fused, the transpose step on 64 x 8 tiles).
    (37, 21, 70): z-chunks of 27 and 26 planes with the warm-up, so the
    transpose kernels carrying 2 or 3 planes per loop trip (shapes 14, 15) run
    their remainder loop in one chunk or both."""
    wl, an = synth.workload_tti(shape=shape, nt=50, r=8, sigma=2.0, nb=4, f0=15.0,
                                rec_stride=7, dtype=np.float64)
    g = Grid.of(wl)
    say(f"case: TTI F64 {wl.shape} nt={wl.nt} r={wl.r} variant {variant}")
    f = oracle.tti_forward(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z)
    plan = _plan(wl, "f64", "f64")
    m, a, q, Z = (dev(wl.m, torch.float64), dev(an, torch.float64), dev(wl.q, torch.float64),
                  dev(wl.Z, torch.int8))
    out = P.rtm_tti_forward_probe(plan, m, a, wl.src_pos, q, wl.rec_pos, Z=Z)
    torch.cuda.synchronize()
    e_d, e_u = rel(host(out["d"]), f["d"]), rel(_rows(plan, out["Ubar"]), f["bar"])
    rng = np.random.default_rng(3)
    res = rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))
    ad = oracle.tti_adjoint(g, wl.m, an, wl.rec_pos, res, src_pos=wl.src_pos, Z=wl.Z)
    adj = P.rtm_tti_adjoint_probe(plan, m, a, wl.rec_pos, dev(res, torch.float64), Z=Z,
                                  src_pos=wl.src_pos, want_qadj=True)
    torch.cuda.synchronize()
    e_v, e_qa = rel(_rows(plan, adj["Vbar"]), ad["bar"]), rel(host(adj["qadj"]), ad["qadj"])
    d_obs = oracle.tti_forward(g, wl.m * 1.03, an, wl.src_pos, wl.q, wl.rec_pos)["d"]
    J, gp, _, _ = oracle.tti_probed_gradient(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos, d_obs,
                                             wl.Z)
    gr = P.fwi_gradient_tti(plan, m, a, wl.src_pos, q, wl.rec_pos, dev(d_obs, torch.float64), Z)
    torch.cuda.synchronize()
    e_g = rel(host(gr["grad"]), gp)
    e_J = abs(float(gr["misfit"].item()) - J) / J
    say(f"  d {e_d:.2e} Ubar {e_u:.2e} Vbar {e_v:.2e} qadj {e_qa:.2e} grad {e_g:.2e} J {e_J:.2e}")
    assert max(e_d, e_u, e_v, e_qa, e_g) < 1e-10 and e_J < 1e-12


def test_tti_gpu_dot_test_and_isotropic_limit():
    wl, an = synth.workload_tti(shape=(20, 18, 22), nt=60, r=4, sigma=2.0, nb=4, f0=15.0,
                                rec_stride=9, dtype=np.float64)
    plan = _plan(wl, "f64", "f64")
    rng = np.random.default_rng(4)
    m, a = dev(wl.m, torch.float64), dev(an, torch.float64)
    qx = dev(rng.standard_normal((wl.nt, 1)), torch.float64)
    y = dev(rng.standard_normal((wl.nt, wl.rec_pos.shape[0])), torch.float64)
    d = P.rtm_tti_forward_probe(plan, m, a, wl.src_pos, qx, wl.rec_pos)["d"]
    qa = P.rtm_tti_adjoint_probe(plan, m, a, wl.rec_pos, y, src_pos=wl.src_pos,
                                 want_qadj=True)["qadj"]
    l, r_ = P.rtm_dot(plan, d.reshape(-1), y.reshape(-1)).item(), \
        P.rtm_dot(plan, qx.reshape(-1), qa.reshape(-1)).item()
    say(f"  TTI dot test: rel {abs(l - r_) / abs(l):.2e}")
    assert abs(l - r_) <= 1e-12 * abs(l)
    iso = an.copy()
    iso[0] = 0.0
    iso[1] = 0.0
    d_tti = P.rtm_tti_forward_probe(plan, m, dev(iso, torch.float64), wl.src_pos, qx,
                                    wl.rec_pos)["d"]
    d_ac = P.rtm_forward_probe(plan, m, wl.src_pos, qx, wl.rec_pos)["d"]
    torch.cuda.synchronize()
    e = rel(host(d_tti), host(d_ac))
    say(f"  isotropic TTI vs acoustic: {e:.2e}")
    assert e < 1e-12


@pytest.mark.parametrize("k", [16, 64])
def test_tti_f32_bf16x2_fused_gradient(k):
    """k = 64: one 64-step block and a 16-step one; the probe launches of the
    64-step block stride over a fixed number of tiles per wave (the TTI sweeps
    have no work-queue counter)."""
    wl, an = synth.workload_tti(shape=(30, 26, 36), nt=80, r=16, sigma=3.0, nb=5, f0=12.0,
                                rec_stride=3)
    g = Grid.of(wl)
    d_obs = np.zeros((wl.nt, wl.rec_pos.shape[0]), dtype=np.float32)
    J, gp, _, _ = oracle.tti_probed_gradient(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos, d_obs,
                                             wl.Z)
    plan = _plan(wl, "f32", "bf16x2", k_block=k)
    args = (plan, dev(wl.m, torch.float32), dev(an, torch.float32), wl.src_pos,
            dev(wl.q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
            dev(wl.Z, torch.int8))
    fu = P.fwi_gradient_tti(*args, fused=True)
    un = P.fwi_gradient_tti(*args)
    torch.cuda.synchronize()
    e_f, e_u = rel(host(fu["grad"]), gp), rel(host(fu["grad"]), host(un["grad"]))
    e_J = abs(float(fu["misfit"].item()) - J) / J
    say(f"  TTI f32/bf16x2 fused: vs oracle {e_f:.2e}, vs unfused {e_u:.2e}, misfit {e_J:.2e}")
    assert e_f < 1e-3 and e_u < 1e-5 and e_J < 1e-5


@pytest.mark.parametrize("shape", [3, 4, 6, 7, 8, 9, 10, 11, 12, 13, 15, 16, 17, 18, 19, 20, 21])
def test_tti_f32_tiled_equals_simple_kernels(shape):
    """The tiled TTI step (mixed terms once per unordered pair, intermediates
    staged per plane) against the one-thread-per-cell step on the same FP32
    inputs: equal to FP32 rounding for the data, the compressed fields and the
    gradient.  The fields themselves agree to ~1e-8; u_tt is a second time
    difference of FP32 levels (about three digits cancel), so Ubar and the
    gradient carry ~2e-5 and the bar is 5e-5, as for the acoustic FP32 Ubar."""
    wl, an = synth.workload_tti(shape=(44, 27, 75), nt=70, r=32, sigma=3.0, nb=5, f0=12.0,
                                rec_stride=4)
    rng = np.random.default_rng(9)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    plan = _plan(wl, "f32", "bf16x2", k_block=32)
    args = (plan, dev(wl.m, torch.float32), dev(an, torch.float32), wl.src_pos,
            dev(wl.q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
            dev(wl.Z, torch.int8))
    out = {}
    for v in (0, -1):
        P.set_stencil_variant(v)
        P.set_tti_shape(shape)
        try:
            out[v] = P.fwi_gradient_tti(*args, fused=False)
            torch.cuda.synchronize()
        finally:
            P.set_stencil_variant(-1)
            P.set_tti_shape(21)  # the default
    e = {k: rel(host(out[-1][k]), host(out[0][k])) for k in ("resid", "Ubar", "Vbar", "grad")}
    say(f"  TTI tiled (shape {shape}) vs simple (f32): " +
        " ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["resid"] < 1e-6 and max(e.values()) < 5e-5


def test_tti_f32_lds_queue_kernels_equal_shape_11():
    """Shapes 13-15 keep the transpose's halo queues in LDS and carry 1-3
    planes per loop trip, 16 and 17 also carry two or three planes per trip in
    the forward step, 18 takes one workgroup barrier per plane in the
    transpose: the same arithmetic in the same order as shape 11, so
    the FP32 results are equal bit for bit.  (37, 27, 75):
    z-chunks of 27 and 26 planes with the warm-up, so the loops carrying 2 or 3
    planes per trip run their remainder in one chunk or both."""
    wl, an = synth.workload_tti(shape=(37, 27, 75), nt=70, r=32, sigma=3.0, nb=5, f0=12.0,
                                rec_stride=4)
    rng = np.random.default_rng(9)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    plan = _plan(wl, "f32", "bf16x2", k_block=32)
    args = (plan, dev(wl.m, torch.float32), dev(an, torch.float32), wl.src_pos,
            dev(wl.q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
            dev(wl.Z, torch.int8))
    out = {}
    try:
        for shape in (11, 13, 14, 15, 16, 17, 18):
            P.set_tti_shape(shape)
            out[shape] = P.fwi_gradient_tti(*args, fused=True)
            torch.cuda.synchronize()
    finally:
        P.set_tti_shape(21)  # the default
    for shape in (13, 14, 15, 16, 17, 18):
        for k in ("resid", "Ubar", "grad"):
            assert torch.equal(out[shape][k], out[11][k]), (shape, k)
    say("  TTI shapes 13-18 equal shape 11 bit for bit (resid, Ubar, grad)")


def test_tti_f32_merged_transpose_forms_agree():
    """Shapes 19-21 sum the transpose's p equation as one second difference
    per axis of (1 - n_a^2) w1 and carry 3, 4 or 6 planes per loop trip: equal
    to each other bit for bit.  Against shape 18 (the same step with the
    Laplacian and the H_z sum formed apart and subtracted) they differ by
    rounding only, so both are held to the FP64 oracle's probed gradient on
    the same probes, at the bar of the FP32 fused TTI gradient (1e-3; here
    about 2.1e-4 merged and 1.3e-4 unmerged).  The forward step is shared, so
    the data and Ubar agree exactly.  (37, 27, 75): z-chunks of 27 and 26
    planes with the warm-up, so each loop runs a remainder."""
    wl, an = synth.workload_tti(shape=(37, 27, 75), nt=70, r=32, sigma=3.0, nb=5, f0=12.0,
                                rec_stride=4)
    rng = np.random.default_rng(9)
    d_obs = (0.05 * rng.standard_normal((wl.nt, wl.rec_pos.shape[0]))).astype(np.float32)
    g = Grid.of(wl)
    _, gp, _, _ = oracle.tti_probed_gradient(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos,
                                             d_obs.astype(np.float64), wl.Z)
    plan = _plan(wl, "f32", "bf16x2", k_block=32)
    args = (plan, dev(wl.m, torch.float32), dev(an, torch.float32), wl.src_pos,
            dev(wl.q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
            dev(wl.Z, torch.int8))
    out = {}
    try:
        for shape in (18, 19, 20, 21):
            P.set_tti_shape(shape)
            out[shape] = P.fwi_gradient_tti(*args, fused=True)
            torch.cuda.synchronize()
    finally:
        P.set_tti_shape(21)  # the default
    for shape in (20, 21):
        for k in ("resid", "Ubar", "grad"):
            assert torch.equal(out[shape][k], out[19][k]), (shape, k)
    assert torch.equal(out[19]["resid"], out[18]["resid"])
    assert torch.equal(out[19]["Ubar"], out[18]["Ubar"])
    e18, e19 = rel(host(out[18]["grad"]), gp), rel(host(out[19]["grad"]), gp)
    e = rel(host(out[19]["grad"]), host(out[18]["grad"]))
    say(f"  TTI shapes 19-21 equal bit for bit; vs the FP64 oracle: merged {e19:.2e}, "
        f"unmerged {e18:.2e} (apart {e:.2e})")
    assert e19 < 1e-3 and e18 < 1e-3
