"""Full-size parity.  The 384 x 512 x 512 layered 3D grid (r = 128 probes,
k = 32, BF16X2 MFMA probing, FP32 fields) through fwi_gradient - the launch
configuration the benchmark times - truncated to nt = 64 steps so the FP64
oracle can follow it: traces (the whole 512 x 512 receiver plane) and the
misfit in full, the compressed fields and the gradient on a sample of cells
(near the source, in the sponge, at grid corners, random), with the image
taken separately and fused into the adjoint probe blocks.  The anisotropic
TTI gradient on a 48-plane slab of the full 400 x 400 extent against the
oracle; the whole 300 x 400 x 400 TTI grid through properties that hold at
any size (dot test, isotropic limit), and its 81-offset image volume on
sampled rows against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say
from oracle import Grid

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402


def _sample_cells(shape, src, seed=0, n_rand=1500):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    z0, y0, x0 = (int(v) for v in src)
    near = np.stack([rng.integers(max(z0 - 14, 0), z0 + 15, 600),
                     rng.integers(y0 - 14, y0 + 15, 600),
                     rng.integers(x0 - 14, x0 + 15, 600)], 1)
    anywhere = np.stack([rng.integers(0, nz, n_rand), rng.integers(0, ny, n_rand),
                         rng.integers(0, nx, n_rand)], 1)
    corners = np.array([[0, 0, 0], [nz - 1, ny - 1, nx - 1], [0, ny - 1, 0], [5, 3, nx - 2],
                        [z0, y0, x0], [z0 + 1, y0, x0], [z0, y0 - 1, x0 + 2]])
    c = np.vstack([near, anywhere, corners])
    idx = np.unique((c[:, 0] * ny + c[:, 1]) * nx + c[:, 2])
    return idx.astype(np.int64)


@pytest.fixture(scope="module")
def c2_truncated():
    """The bench workload truncated to nt = 64, its sampled cells, and the
    oracle's probed gradient on them (computed once for both legs)."""
    require_gpu()
    nt = 64
    wl = synth.workload_c2(nt=nt)
    idx = _sample_cells(wl.shape, wl.src_pos[0])
    d_obs = np.zeros((nt, wl.rec_pos.shape[0]), dtype=np.float32)
    say(f"oracle: full-size {wl.shape} nt={nt} r={wl.r} probed gradient on {idx.size} cells")
    Jo, go, f, a = oracle.probed_gradient(Grid.of(wl), wl.m, wl.src_pos, wl.q, wl.rec_pos,
                                          d_obs, wl.Z, sample_idx=idx)
    return wl, idx, d_obs, Jo, go, f, a


@pytest.mark.parametrize("fused,k", [(False, 32), (True, 32), (True, 64)],
                         ids=["separate-image", "fused-image", "fused-image-k64"])
def test_fullsize_layered_3d_gradient_truncated(c2_truncated, fused, k):
    """fused=True is the benchmark's adjoint kernel (imaging folded into the
    probe blocks, Vbar never stored) at a size where each wave's grid-stride
    loop visits many 32-cell tiles.  k = 64: one 64-step block, whose forward
    probe launch takes its tiles from the work queue (the oracle's probed
    gradient does not depend on the block length)."""
    wl, idx, d_obs, Jo, go, f, a = c2_truncated
    nt = wl.nt
    say(f"case: full-size {wl.shape} nt={nt} r={wl.r} k={k} bf16x2 fwi_gradient "
        f"fused={fused}")
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=k)
    out = P.fwi_gradient(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                         wl.rec_pos, dev(d_obs, torch.float32), dev(wl.Z, torch.int8),
                         fused=fused)
    torch.cuda.synchronize()
    res = host(out["resid"])
    J = float(out["misfit"].item())
    ii = torch.from_numpy(idx).cuda()
    bi = torch.from_numpy(P.bar_index(plan, idx)).cuda()
    U = host(out["Ubar"].reshape(-1)[bi])
    V = None if fused else host(out["Vbar"].reshape(-1)[bi])
    gr = host(out["grad"][ii])
    del out
    torch.cuda.empty_cache()
    e = dict(d=rel(res, f["d"]), J=abs(J - Jo) / Jo, U=rel(U, f["Ubar"]), g=rel(gr, go))
    if V is not None:
        e["V"] = rel(V, a["Vbar"])
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["d"] < 1e-5 and e["J"] < 2e-5
    assert e["U"] < 1e-4 and e.get("V", 0.0) < 1e-4 and e["g"] < 1e-3


def test_fullsize_tti_anisotropic_slab_against_oracle():
    """The anisotropic TTI gradient on a 48-plane slab of the full 400 x 400
    x/y extent (r = 64 on p and q, k = 32, BF16X2, fused imaging: the
    benchmark's kernels, default tile shape and z split) against the oracle.
    nt = 36 is one full probe block and a short one.  So that every tile
    carries signal from the first step, 1875 sources on a 16-cell lattice at
    three depths inject seeded noise.  Checked: the whole receiver plane, the
    misfit, both compressed fields and the gradient on sampled cells."""
    require_gpu()
    nt = 36
    wl, an = synth.workload_tti(shape=(48, 400, 400), nt=nt, r=64)
    nz, ny, nx = wl.shape
    zz, yy, xx = np.meshgrid([8.0, 24.0, 40.0], np.arange(8.0, ny, 16.0),
                             np.arange(8.0, nx, 16.0), indexing="ij")
    src = np.column_stack([zz.ravel(), yy.ravel(), xx.ravel()])
    q = (np.random.default_rng(31).standard_normal((nt, src.shape[0])) / wl.h ** 3).astype(
        np.float32)
    rng = np.random.default_rng(32)
    idx = np.unique(np.concatenate([
        rng.integers(0, wl.N, 3000),
        (np.array([0, nz - 1, 12, 24])[:, None] * ny * nx
         + np.array([0, ny * nx - 1, 200 * nx + 200, 399 * nx])[None, :]).ravel()]))
    d_obs = np.zeros((nt, wl.rec_pos.shape[0]), dtype=np.float32)
    say(f"case: TTI slab {wl.shape} nt={nt} r={wl.r} nsrc={src.shape[0]} "
        f"nrec={wl.rec_pos.shape[0]} fused bf16x2")
    plan = P.Plan(P.PlanSpec(3, wl.shape, wl.h, wl.dt, nt, wl.nb, wl.c_ref, wl.R, wl.c_ref,
                             "f32", "bf16x2", wl.r, 32, src.shape[0], wl.rec_pos.shape[0]))
    out = P.fwi_gradient_tti(plan, dev(wl.m, torch.float32), dev(an, torch.float32), src,
                             dev(q, torch.float32), wl.rec_pos, dev(d_obs, torch.float32),
                             dev(wl.Z, torch.int8), fused=True)
    torch.cuda.synchronize()
    res = host(out["resid"])
    J = float(out["misfit"].item())
    bi = torch.from_numpy(P.bar_index(plan, idx)).cuda()
    fs = wl.r * plan.Npad
    U = np.stack([host(out["Ubar"].reshape(-1)[f * fs + bi]) for f in range(2)])
    gr = host(out["grad"][torch.from_numpy(idx).cuda()])
    del out
    torch.cuda.empty_cache()
    say("  gpu done; oracle TTI forward + adjoint on the slab ...")
    Jo, go, f, a = oracle.tti_probed_gradient(Grid.of(wl), wl.m, an, src, q, wl.rec_pos, d_obs,
                                              wl.Z, sample_idx=idx)
    e = dict(d=rel(res, f["d"]), J=abs(J - Jo) / Jo, U=rel(U, f["bar"]), g=rel(gr, go))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["d"] < 1e-5 and e["J"] < 2e-5
    assert e["U"] < 1e-4 and e["g"] < 1e-3


def test_fullsize_tti_dot_test_and_isotropic_limit():
    """TTI at its full size (300 x 400 x 400, full receiver plane) in the
    launch configuration the benchmark times (FP32, tiled fused step kernels),
    truncated to 48 steps: the forward map and its transpose pass the dot
    test, and with eps = delta = 0 the forward traces equal the acoustic ones
    (to FP32 rounding: the TTI step forms H0 = L - Hz, the acoustic one L)."""
    require_gpu()
    nt = 48
    wl, an = synth.workload_tti(nt=nt)
    say(f"case: full-size TTI {wl.shape} nt={nt} nrec={wl.rec_pos.shape[0]}")
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=wl.c_ref)
    rng = np.random.default_rng(21)
    m, a = dev(wl.m, torch.float32), dev(an, torch.float32)
    qx = dev(rng.standard_normal((nt, 1)).astype(np.float32), torch.float32)
    y = dev(rng.standard_normal((nt, wl.rec_pos.shape[0])).astype(np.float32), torch.float32)
    d = P.rtm_tti_forward_probe(plan, m, a, wl.src_pos, qx, wl.rec_pos)["d"]
    qa = P.rtm_tti_adjoint_probe(plan, m, a, wl.rec_pos, y, src_pos=wl.src_pos,
                                 want_qadj=True)["qadj"]
    lhs = P.rtm_dot(plan, d.reshape(-1), y.reshape(-1)).item()
    rhs = P.rtm_dot(plan, qx.reshape(-1), qa.reshape(-1)).item()
    say(f"  full-size TTI dot test: {lhs:.9e} {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    iso = an.copy()
    iso[0] = 0.0
    iso[1] = 0.0
    d_tti = host(P.rtm_tti_forward_probe(plan, m, dev(iso, torch.float32), wl.src_pos, qx,
                                         wl.rec_pos)["d"])
    d_ac = host(P.rtm_forward_probe(plan, m, wl.src_pos, qx, wl.rec_pos)["d"])
    e = rel(d_tti, d_ac)
    say(f"  full-size isotropic TTI vs acoustic: {e:.2e}")
    assert e < 1e-5


def test_fullsize_offset_gathers_sampled_rows():
    """The 81-offset image volume at 300 x 400 x 400 from two r = 64 compressed
    fields (the benchmark's launch): whole x rows, all offsets, compared with
    the oracle evaluated on those rows' probe values."""
    require_gpu()
    shape, r, nh = (300, 400, 400), 64, 40
    plan = P.Plan(P.PlanSpec(3, shape, 12.5, 1e-3, 64, 10, 4500.0, 1e-3, 4500.0, "f32",
                             "bf16x2", r, 32, 1, 1))
    gen = torch.Generator(device="cuda").manual_seed(5)
    nb = 2 * r * plan.Npad
    U = torch.randn(nb, generator=gen, device="cuda")
    V = torch.randn(nb, generator=gen, device="cuda")
    G = P.rtm_offset_gathers(plan, U, V, nh, nfield=2)
    torch.cuda.synchronize()
    nz, ny, nx = shape
    rng = np.random.default_rng(3)
    rows = [(0, 0), (nz - 1, ny - 1)] + [tuple(v) for v in
                                         np.stack([rng.integers(0, nz, 30),
                                                   rng.integers(0, ny, 30)], 1)]
    worst = 0.0
    for z, yy in rows:
        cells = (z * ny + yy) * nx + np.arange(nx)
        bi = torch.from_numpy(P.bar_index(plan, cells)).cuda()   # [r][nx] offsets in a field
        fs = r * plan.Npad
        Ur = [host(U[f * fs + bi]) for f in range(2)]
        Vr = [host(V[f * fs + bi]) for f in range(2)]
        G0 = sum(oracle.offset_gathers(Ur[f].astype(np.float64), Vr[f].astype(np.float64),
                                       (1, 1, nx), nh, 1.0 / r) for f in range(2))
        Gr = host(G[:, torch.from_numpy(cells).cuda()]).astype(np.float64)
        worst = max(worst, rel(Gr, G0))
    say(f"  full-size gathers, {len(rows)} rows: worst rel {worst:.2e}")
    assert worst < 1e-5


def test_fullsize_batched_equals_single_shots_bitwise():
    """The 16-window batched case at its full size (181 M cells, full receiver
    planes, r = 64, k = 32, BF16X2, fused imaging), truncated to 64 steps: one
    stencil launch per step over every window gives the same gradient,
    residuals and compressed fields as each shot alone, bit for bit (the
    single shots are pinned against the oracle by the full-size acoustic test
    and the small batched test)."""
    require_gpu()
    nt = 64
    wls = synth.workload_batched(nt=nt)
    say(f"case: full-size batched {len(wls)} windows, {sum(int(np.prod(w.shape)) for w in wls)} "
        f"cells, nt={nt}")
    specs, shots = [], []
    for wl in wls:
        specs.append(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, 4725.0,
                                "f32", "bf16x2", wl.r, wl.k_block, 1, wl.rec_pos.shape[0]))
        shots.append(dict(m=dev(wl.m, torch.float32), src_pos=wl.src_pos,
                          q=dev(wl.q, torch.float32), rec_pos=wl.rec_pos,
                          d_obs=torch.zeros((nt, wl.rec_pos.shape[0]), device="cuda"),
                          Z=dev(wl.Z, torch.int8)))
    B = P.Batch(specs)
    outs, J = B.fwi_gradient(shots)
    torch.cuda.synchronize()
    del B
    same = 0
    for i, (sp, sh) in enumerate(zip(specs, shots)):
        plan = P.Plan(sp)
        one = P.fwi_gradient(plan, sh["m"], sh["src_pos"], sh["q"], sh["rec_pos"], sh["d_obs"],
                             sh["Z"], fused=True)
        torch.cuda.synchronize()
        ok = all(torch.equal(outs[i][k], one[k]) for k in ("grad", "resid", "Ubar")) and \
            float(J[i].item()) == float(one["misfit"].item())
        same += ok
        del one, plan
        torch.cuda.empty_cache()
    say(f"  full-size batched == single for {same} of {len(specs)} shots")
    assert same == len(specs)
