"""Throughput of the probed FWI gradient on one MI355X.

One step = one whole pass of the hot path over the 3D layered workload:
forward sweep (FP32 8th-order stencil, source injection, receiver sampling,
BF16X2 MFMA probing of u_tt every k steps), residual + FP64 misfit, adjoint
sweep (receiver injection, probing of the adjoint field), probed imaging
condition.  Workload: 384 x 512 x 512 cells (z, y, x) incl. 10 damping cells
per face, h = 12.5 m, nt = 3000, dt = 1 ms, 12 layers 1.5-4.5 km/s with +-5 %
perturbation, one shot, 512 x 512 receiver plane, r = 128 Rademacher probes,
k = 32 (synthetic inputs, seeded).

value = 2 N nt / wall time (Gcell-updates/s, forward + adjoint, inputs resident
in HBM).  The roofline object covers the dominant kernel, timed with HIP events
on the sweep's own stream during the timed steps (every --prof-stride-th
stencil launch, every probe-GEMM launch).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector-ALU issue ceiling: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 FP32 VALU
# instruction per SIMD every 4 cycles (16 lanes; the packed-FP32 forms that
# double the vendor's FP32 vector figure are not used)
VALU_PEAK_GINSTS = 256 * 4 * 2.4 / 4
PMC_SOURCE = ("stored rocprofv3 --pmc record profiles/pmc_traffic.json, taken on these kernel "
              "sources (hash match), not measured in this run")


def _pmc_kernels(part: str, grid, **params):
    """Per-dispatch counters of one workload ("acoustic", "tti" or "gathers")
    from the stored rocprofv3 --pmc record, keyed by kernel, if the kernel
    sources are unchanged since the counters were taken and the workload (grid
    and params) matches; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for name in ("stencil.hip", "probe.hip", "misc.hip", "tti.hip", "tti_tiled.hip",
                 "gathers.hip"):
        with open(os.path.join(ROOT, "paper_2201_06914_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    w = rec.get(part)
    if rec.get("source_hash") != h.hexdigest()[:16] or not w or w.get("grid") != list(grid) \
            or any(w.get(k) != v for k, v in params.items()):
        return None
    return w["kernels"]


def measured_traffic(part: str, grid, **params):
    """HBM bytes per dispatch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy
    of known size) from the stored PMC record, keyed by kernel, or None."""
    ks = _pmc_kernels(part, grid, **params)
    if ks is None:
        return None
    return {key: v["read_bytes"] + v["write_bytes"] for key, v in ks.items()}


def valu_entry(part: str, grid, key: str, avg_launch_us: float, cells: int, **params):
    """The kernel's vector-ALU issue rate: SQ_INSTS_VALU per dispatch (wave64
    instructions, stored PMC record) over the launch time measured in this
    run, against VALU_PEAK_GINSTS; None without a matching record."""
    ks = _pmc_kernels(part, grid, **params)
    if not ks or key not in ks or "valu_insts" not in ks[key] or not avg_launch_us:
        return None
    n = ks[key]["valu_insts"]
    ach = n / (avg_launch_us * 1e-6) / 1e9
    return {"bound": "alu", "achieved": round(ach, 1), "peak": VALU_PEAK_GINSTS,
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / VALU_PEAK_GINSTS, 4),
            "insts_per_launch": n, "lane_insts_per_cell": round(n * 64 / cells, 1),
            "source": PMC_SOURCE}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=3000)
    ap.add_argument("--k-block", type=int, default=32)
    ap.add_argument("--probe", default="bf16x2", choices=["bf16x2", "bf16", "f32"])
    ap.add_argument("--prof-stride", type=int, default=50)
    ap.add_argument("--stencil-variant", type=int, default=None,
                    help="fix the stencil kernel variant instead of autotuning it")
    ap.add_argument("--stencil-blocks", type=int, default=None,
                    help="with --stencil-variant: the z-split target (default 2048)")
    ap.add_argument("--unfused", action="store_true",
                    help="store Vbar and run the separate imaging kernel (default: fused imaging)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the one step with the other imaging variant (fused / separate)")
    ap.add_argument("--no-exact", action="store_true",
                    help="skip the exact (checkpointed FP32) comparator run")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (PMC calibration)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 16-shot batched workload section")
    ap.add_argument("--batched-nt", type=int, default=2000)
    ap.add_argument("--no-rsweep", action="store_true",
                    help="skip the 300^3 four-shot probe-count sweep against the exact gradient")
    ap.add_argument("--rsweep-n", type=int, default=300)
    ap.add_argument("--rsweep-nt", type=int, default=2000)
    ap.add_argument("--no-fwi", action="store_true",
                    help="skip the FWI iterations (stacked probed vs exact) on the 300^3 case")
    ap.add_argument("--fwi-iters", type=int, default=3)
    ap.add_argument("--no-tti", action="store_true",
                    help="skip the 300x400x400 TTI gradient section")
    ap.add_argument("--tti-nt", type=int, default=2500)
    ap.add_argument("--no-gathers", action="store_true",
                    help="skip the 81-offset image volume at the TTI grid")
    ap.add_argument("--no-ksweep", action="store_true",
                    help="skip the k = 64 / 128 runs of the headline gradient")
    ap.add_argument("--cpu-planes", type=int, default=24)
    ap.add_argument("--cpu-nt", type=int, default=80)
    return ap.parse_args()


def cpu_baseline(planes: int, nt: int, r: int):
    """The FP64 oracle, as it stands, on a z-slab of the same model: `planes`
    x 512 x 512 cells, `nt` steps, forward + adjoint with r-probe compression
    and the probed image (Gcell-updates/s).  Two more legs time the oracle on
    the 2D two-layer case in full and on a slab of the TTI model."""
    import numpy as np

    import oracle
    import synth
    wl = synth.workload_c2(nt=nt, r=r, shape=(planes, 512, 512))
    g = oracle.Grid(3, wl.shape, wl.h, wl.dt, nt, min(wl.nb, (planes - 1) // 2), wl.c_ref, wl.R)
    src = np.array([[planes // 2, 256.0, 256.0]])
    rec = synth.plane_receivers(planes // 2 + 1, 512, 512)
    d_obs = np.zeros((nt, rec.shape[0]))
    t0 = time.perf_counter()
    J, gref, f, _ = oracle.probed_gradient(g, wl.m, src, wl.q, rec, d_obs, wl.Z)
    dt = time.perf_counter() - t0
    # kept for the precision comparison (the same slab on the GPU)
    slab = dict(grid=g, m=wl.m, src=src, q=wl.q, rec=rec, d_obs=d_obs, Z=wl.Z, J=J, grad=gref,
                d=f["d"], c_ref=wl.c_ref)
    del wl, f
    out = {"value": 2.0 * g.N * nt / dt / 1e9, "unit": "Gcell-updates/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"FP64 oracle, {planes}x512x512 z-slab of the same model, nt={nt}, "
                     f"r={r}, forward+adjoint with probing + image, {dt:.1f} s"}
    print("cpu baseline: 3D slab done", file=sys.stderr, flush=True)
    # 2D two-layer case (221 x 221, nt = 1000, r = 32, FP64) in full
    w1 = synth.workload_c1()
    g1 = oracle.Grid.of(w1)
    d1 = oracle.forward(g1, w1.m_true, w1.src_pos, w1.q, w1.rec_pos)["d"]
    t0 = time.perf_counter()
    oracle.probed_gradient(g1, w1.m, w1.src_pos, w1.q, w1.rec_pos, d1, w1.Z)
    dt1 = time.perf_counter() - t0
    out["c1_full"] = {"value": round(2.0 * g1.N * g1.nt / dt1 / 1e9, 5),
                      "unit": "Gcell-updates/s", "seconds": round(dt1, 2),
                      "sample": "FP64 oracle, 2D two-layer 221x221, nt=1000, r=32, "
                                "forward+adjoint with probing + image, in full"}
    print("cpu baseline: 2D case done", file=sys.stderr, flush=True)
    # TTI: a 16 x 128 x 128 slab of the layered + salt TTI recipe, 12 steps
    tp, tn = 16, 12
    w3, an = synth.workload_tti(shape=(tp, 128, 128), nt=tn, r=64)
    g3 = oracle.Grid(3, w3.shape, w3.h, w3.dt, tn, min(w3.nb, (tp - 1) // 2), w3.c_ref, w3.R)
    rec3 = synth.plane_receivers(tp // 2 + 1, 128, 128)
    t0 = time.perf_counter()
    oracle.tti_probed_gradient(g3, w3.m, an, np.array([[tp // 2, 64.0, 64.0]]), w3.q, rec3,
                               np.zeros((tn, rec3.shape[0])), w3.Z)
    dt3 = time.perf_counter() - t0
    out["c3_tti_slab"] = {"value": round(2.0 * g3.N * tn / dt3 / 1e9, 6),
                          "unit": "Gcell-updates/s", "seconds": round(dt3, 2),
                          "sample": f"FP64 oracle, TTI {tp}x128x128 slab of the layered + salt "
                                    f"model, nt={tn}, r=64 on p and q, forward+adjoint with "
                                    f"probing + image"}
    print("cpu baseline: TTI slab done", file=sys.stderr, flush=True)
    return out, slab


def bench_precision(slab, shape, nt_full: int, r: int, k: int, variant: int):
    """The probe-GEMM operand forms side by side: bf16 (one MFMA), bf16 hi + lo
    (two MFMAs), float16 with per-chunk power-of-two scales (one MFMA) and the
    FP32 vector path.  Error: the GPU gradient (FP32 fields, each probe form)
    against the FP64 oracle's probed gradient on the oracle's z-slab of the
    bench model (same probes, same geometry).  Time: the full-grid gradient
    over the first nt_full steps."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth
    g = slab["grid"]
    m = torch.from_numpy(np.ascontiguousarray(slab["m"], np.float32)).cuda()
    q = torch.from_numpy(np.ascontiguousarray(slab["q"], np.float32)).cuda()
    Z = torch.from_numpy(slab["Z"]).cuda()
    d_obs = torch.from_numpy(np.ascontiguousarray(slab["d_obs"], np.float32)).cuda()
    gref = slab["grad"]
    wl = synth.workload_c2(nt=nt_full, r=r, k_block=k, shape=shape)
    mf, qf, Zf = (torch.from_numpy(a).cuda() for a in (wl.m, wl.q, wl.Z))
    dof = torch.zeros((nt_full, wl.rec_pos.shape[0]), device="cuda")
    pf = P.Plan.for_workload(wl, field="f32", probe="bf16x2", k_block=k)
    rows = []
    P.set_stencil_variant(variant)
    for probe in ("bf16", "bf16x2", "f16s", "f32"):
        fused = probe != "f32"
        plan = P.Plan(P.PlanSpec(3, g.shape, g.h, g.dt, g.nt, g.nb, g.c_ref, g.R, slab["c_ref"],
                                 "f32", probe, r, k, 1, slab["rec"].shape[0]))
        o = P.fwi_gradient(plan, m, slab["src"], q, slab["rec"], d_obs, Z, fused=fused)
        gg = o["grad"].double().cpu().numpy()
        err = float(np.linalg.norm(gg - gref) / np.linalg.norm(gref))
        errJ = abs(float(o["misfit"].item()) - slab["J"]) / slab["J"]
        full = P.Plan(P.PlanSpec(*[getattr(pf.spec, f) for f in ("ndim", "shape", "h", "dt", "nt",
                                                                  "nb", "c_ref", "R", "c_max")],
                                 "f32", probe, r, k, pf.spec.nsrc, pf.spec.nrec))
        work = full.workspace("cuda")
        bars = (full.empty_bar("cuda"), None if fused else full.empty_bar("cuda"))
        run = lambda: P.fwi_gradient(full, mf, wl.src_pos, qf, wl.rec_pos, dof, Zf,  # noqa: E731
                                     work=work, bars=bars, fused=fused)
        run()
        torch.cuda.synchronize()
        t = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        rows.append({"probe": probe, "imaging": "fused" if fused else "separate",
                     "grad_rel_err_vs_fp64_oracle": float(f"{err:.3e}"),
                     "misfit_rel_err": float(f"{errJ:.3e}"),
                     f"ms_full_grid_nt{nt_full}": round(ms, 1)})
        del o, work, bars, full, plan
        torch.cuda.empty_cache()
        print(f"precision: {probe} done", file=sys.stderr, flush=True)
    return {"error_case": f"oracle z-slab {g.shape[0]}x{g.shape[1]}x{g.shape[2]} of the bench "
                          f"model, nt={g.nt}, r={r}, k={k}",
            "timing_case": f"{shape[0]}x{shape[1]}x{shape[2]}, first {nt_full} steps",
            "forms": rows}


def bench_batched(nt: int):
    """16 shots on uneven windows 128^3 ... 256 x 320 x 320 (181,394,048 cells),
    nt steps, r = 64, k = 32, BF16X2 probes, fused imaging: one stencil launch
    per step for all shots; the whole gradient replayed as one HIP graph.
    Compared with the same 16 gradients run one shot at a time."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth
    wls = synth.workload_batched(nt=nt)
    specs, shots = [], []
    for wl in wls:
        specs.append(P.PlanSpec(3, wl.shape, wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R, 4725.0,
                                "f32", "bf16x2", wl.r, wl.k_block, 1, wl.rec_pos.shape[0]))
        shots.append(dict(m=torch.from_numpy(wl.m).cuda(), src_pos=wl.src_pos,
                          q=torch.from_numpy(wl.q).cuda(), rec_pos=wl.rec_pos,
                          d_obs=torch.zeros((nt, wl.rec_pos.shape[0]), device="cuda"),
                          Z=torch.from_numpy(wl.Z).cuda()))
    cells = sum(int(np.prod(sp.shape)) for sp in specs)
    del wls
    # the batch's own stencil variant and z-split target (128 steps each)
    from paper_2201_06914_amd.tune import autotune_batch
    tuned = autotune_batch(specs, shots)
    variant, blocks = tuned["best"]
    kb = tuned["k_block"]
    print(f"batched: tuned variant {variant}, z-split target {blocks}, k {kb}", file=sys.stderr,
          flush=True)
    import dataclasses
    specs = [dataclasses.replace(sp, k_block=kb) for sp in specs]
    blocks_before = P.api.get_stencil_blocks()
    P.set_stencil_blocks(blocks)
    B = P.Batch(specs)
    P.set_stencil_blocks(blocks_before)
    outs = B.outputs()
    J = torch.empty(len(shots), dtype=torch.float64, device="cuda")
    work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device="cuda")
    P.set_stencil_variant(variant)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3

    t_capture = timed(lambda: B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=True,
                                             work=work))
    print("batched: graph captured", file=sys.stderr, flush=True)
    t_graph = min(timed(lambda: B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=True,
                                               work=work)) for _ in range(2))
    g_graph = [o["grad"].clone() for o in outs]
    t_eager = timed(lambda: B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=False,
                                           work=work))
    same = all(torch.equal(a, o["grad"]) for a, o in zip(g_graph, outs))
    print("batched: eager done", file=sys.stderr, flush=True)
    del work, g_graph
    torch.cuda.empty_cache()

    def one_by_one():
        for sp, sh, o in zip(specs, shots, outs):
            plan = P.Plan(sp)
            P.fwi_gradient(plan, sh["m"], sh["src_pos"], sh["q"], sh["rec_pos"], sh["d_obs"],
                           sh["Z"], bars=(o["Ubar"], None), fused=True)
    t_single = timed(one_by_one)
    print("batched: one-by-one done", file=sys.stderr, flush=True)
    return {"workload": f"16 shots, windows 128^3..256x320x320 ({cells} cells), nt={nt}, "
                        f"r=64, k={kb} (autotuned), bf16x2, fused imaging",
            "k_block": kb, "autotune_k_ms_per_step": tuned.get("k_ms_per_step"),
            "value": round(2.0 * cells * nt / (t_graph * 1e-3) / 1e9, 2),
            "unit": "Gcell-updates/s", "ms_per_gradient_graph": round(t_graph, 1),
            "ms_per_gradient_eager": round(t_eager, 1),
            "ms_first_call_with_capture": round(t_capture, 1),
            "ms_one_shot_at_a_time": round(t_single, 1),
            "speedup_vs_one_shot_at_a_time": round(t_single / t_graph, 3),
            "graph_equals_eager": bool(same), "stencil_variant": variant,
            "z_split_target": blocks, "autotune_ms_per_step": tuned["ms_per_step"]}


def bench_rsweep(n: int, nt: int, variant: int):
    """300^3 salt model, 4 shots, nt steps: the probed FWI gradient (4 shots
    batched, BF16X2, fused imaging) for r = 16, 32, 64, 128 against the exact
    FP32 gradient with uniform checkpointing, plus a central finite difference
    of the misfit along a smooth direction.  d_obs is modelled from the true
    model; the gradient is taken at the smoothed model."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth
    h, dt, nb = 12.5, 1e-3, 10
    m_true, m0 = synth.model_salt_300(n)
    srcs, rec = synth.shots_salt_300(n)
    q = torch.from_numpy(synth.source_signature(nt, dt, 10.0, h, 3).astype(np.float32)).cuda()
    mt, mb = torch.from_numpy(m_true).cuda(), torch.from_numpy(m0).cuda()
    N = n ** 3

    def spec(r, k=32):
        return P.PlanSpec(3, (n, n, n), h, dt, nt, nb, 4500.0, 1e-3, 4500.0, "f32", "bf16x2", r,
                          k, 1, rec.shape[0])
    # observed data (untimed setup)
    p_obs = P.Plan(spec(16))
    dobs = [P.rtm_forward_probe(p_obs, mt, s, q, rec)["d"] for s in srcs]
    del mt
    torch.cuda.empty_cache()
    print("rsweep: observed data modelled", file=sys.stderr, flush=True)

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t) * 1e3
    # this grid's own stencil choice (the headline's tuned z-split need not
    # suit it); every run below, exact and probed, uses it
    pe = P.Plan(spec(16))
    tuned = P.autotune_stencil(pe, mb, steps=10)
    print(f"rsweep: stencil variant {tuned['best']}, z-split {tuned['blocks']}", file=sys.stderr,
          flush=True)
    variant = tuned["best"]
    # exact gradient, 4 shots
    ewb = P.exact_workspace_bytes(pe)
    ework = torch.empty(ewb, dtype=torch.uint8, device="cuda")

    def exact_all():
        g = torch.zeros(N, dtype=torch.float64, device="cuda")
        J = 0.0
        for s, d in zip(srcs, dobs):
            o = P.fwi_gradient_exact(pe, mb, s, q, rec, d, work=ework)
            g += o["grad"].double()
            J += float(o["misfit"].item())
        return g, J
    (ge, Je), t_exact = timed(exact_all)
    del ework
    torch.cuda.empty_cache()
    print("rsweep: exact done", file=sys.stderr, flush=True)
    # finite difference along a smooth direction (FP64 misfits)
    rng = np.random.default_rng(400)
    dm = synth.smooth(rng.standard_normal((n, n, n)).astype(np.float32), 8.0).ravel()
    dm = torch.from_numpy((dm / np.abs(dm).max() * 0.01 * m0).astype(np.float32)).cuda()

    def misfit_at(mm):
        J = 0.0
        for s, d in zip(srcs, dobs):
            dp = P.rtm_forward_probe(p_obs, mm, s, q, rec)["d"]
            J += 0.5 * float(((dp.double() - d.double()) ** 2).sum())
        return J
    eps = 1.0
    fd = (misfit_at(mb + eps * dm) - misfit_at(mb - eps * dm)) / (2 * eps)
    lin_exact = float((ge * dm.double()).sum())
    rows = []
    for r, k in ((16, 32), (32, 32), (64, 32), (128, 32), (64, 64), (64, 128), (128, 64),
                 (128, 128)):
        B = P.Batch([spec(r, k)] * 4)
        shots = [dict(m=mb, src_pos=s, q=q, rec_pos=rec, d_obs=d,
                      Z=torch.from_numpy(synth.rademacher(nt, r, 300 + 10 * i + r)).cuda())
                 for i, (s, d) in enumerate(zip(srcs, dobs))]
        outs = B.outputs()
        J = torch.empty(4, dtype=torch.float64, device="cuda")
        work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device="cuda")
        P.set_stencil_variant(variant)
        B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=True, work=work)   # capture
        _, t_pr = timed(lambda: B.fwi_gradient(shots, outs=outs, misfit=J, use_graph=True,
                                                 work=work))
        gp = sum(o["grad"].double() for o in outs)
        err = float(torch.linalg.vector_norm(gp - ge) / torch.linalg.vector_norm(ge))
        cos = float((gp * ge).sum() / (torch.linalg.vector_norm(gp) * torch.linalg.vector_norm(ge)))
        rows.append({"r": r, "k": k, "ms": round(t_pr, 1),
                     "speedup_vs_exact": round(t_exact / t_pr, 3),
                     "grad_rel_err": round(err, 4), "cosine": round(cos, 4),
                     "fd_rel_diff": round(abs(float((gp * dm.double()).sum()) - fd) / abs(fd), 4),
                     "memory_gb_4_shots": round((B.workspace_bytes + sum(o["Ubar"].numel() * 4
                                                                          for o in outs)) / 1e9, 2),
                     "memory_gb_per_shot": round((B.workspace_bytes + sum(o["Ubar"].numel() * 4
                                                                          for o in outs)) / 4e9, 2)})
        del B, outs, work, shots
        torch.cuda.empty_cache()
        print(f"rsweep: r={r} k={k} done", file=sys.stderr, flush=True)
    # range-finder probes: Q = orth(H Omega) per shot (space sketch on MFMA),
    # real probes split bf16 hi + lo on MFMA, fused imaging, scale -1
    rf_rows = []
    for r in (16, 32, 64):
        pr = P.Plan(P.PlanSpec(3, (n, n, n), h, dt, nt, nb, 4500.0, 1e-3, 4500.0, "f32", "bf16x2",
                               r, 32, 1, rec.shape[0]))
        wb = P.rf_workspace_bytes(pr)
        rwork = torch.empty(wb, dtype=torch.uint8, device="cuda")

        def rf_all():
            g = torch.zeros(N, dtype=torch.float64, device="cuda")
            for i, (s, d) in enumerate(zip(srcs, dobs)):
                o = P.fwi_gradient_rf(pr, mb, s, q, rec, d, 300 + 10 * i + r, work=rwork)
                g += o["grad"].double()
                del o
            return g
        P.set_stencil_variant(variant)
        gq, t_rf = timed(rf_all)
        err = float(torch.linalg.vector_norm(gq - ge) / torch.linalg.vector_norm(ge))
        cos = float((gq * ge).sum() / (torch.linalg.vector_norm(gq) * torch.linalg.vector_norm(ge)))
        rf_rows.append({"r": r, "ms": round(t_rf, 1), "speedup_vs_exact": round(t_exact / t_rf, 3),
                        "grad_rel_err": round(err, 5), "cosine": round(cos, 5),
                        "fd_rel_diff": round(abs(float((gq * dm.double()).sum()) - fd) / abs(fd), 5),
                        "memory_gb_per_shot": round((wb + r * pr.Npad * 4) / 1e9, 2)})
        del rwork, gq
        torch.cuda.empty_cache()
        print(f"rsweep: range finder r={r} done", file=sys.stderr, flush=True)
    return {"workload": f"{n}^3 salt model, 4 shots, nt={nt}, h=12.5 m, 10 Hz, gradient at the "
                        f"smoothed model, d_obs modelled from the true model",
            "stencil": {"variant": tuned["best"], "z_split_target": tuned["blocks"]},
            "range_finder": rf_rows,
            "exact_ms": round(t_exact, 1),
            "exact_memory_gb_per_shot": round(ewb / 1e9, 2),
            "full_history_gb_per_shot": round(nt * N * 4 / 1e9, 1),
            "fd_vs_exact_rel_diff": round(abs(lin_exact - fd) / abs(fd), 5),
            "misfit": Je, "probed": rows}


def bench_fwi(n: int, nt: int, iters: int, r: int, variant: int):
    """FWI on the 300^3 salt model with 4 shots: `iters` iterations with
    stacked probed gradients (every shot draws fresh probes each iteration;
    r probes, k = 32, BF16X2, fused imaging, shots batched into one stacked
    gradient) and as many with the exact gradient (uniform checkpointing),
    each followed by a backtracking line search on the misfit.  Misfit and
    relative model error ||m - m_true|| / ||m0 - m_true|| per iteration."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth
    from paper_2201_06914_amd import fwi
    h, dt, nb = 12.5, 1e-3, 10
    m_true, m0 = synth.model_salt_300(n)
    srcs, rec = synth.shots_salt_300(n)
    q = torch.from_numpy(synth.source_signature(nt, dt, 10.0, h, 3).astype(np.float32)).cuda()
    mt, mb = torch.from_numpy(m_true).cuda(), torch.from_numpy(m0).cuda()
    m_min, m_max = 0.8 * float(m_true.min()), 1.2 * float(m_true.max())
    spec = P.PlanSpec(3, (n, n, n), h, dt, nt, nb, 4500.0, 1e-3, float(1.0 / np.sqrt(m_min)),
                      "f32", "bf16x2", r, 32, 1, rec.shape[0])
    p_obs = P.Plan(spec)
    shots = [fwi.Shot(s, q, rec, P.rtm_forward_probe(p_obs, mt, s, q, rec)["d"]) for s in srcs]
    P.autotune_stencil(p_obs, mb, steps=10)   # this grid's stencil choice, applied
    del p_obs
    torch.cuda.empty_cache()
    out = {}
    for name, exact in (("probed", False), ("exact", True)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = fwi.fwi(spec, mb, shots, iters=iters, seed=500, step=0.02, m_min=m_min,
                      m_max=m_max, exact=exact, m_true=mt)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        out[name] = {"misfit": [round(x["misfit"], 6) for x in res["history"]]
                     + [round(res["final_misfit"], 6)],
                     "model_err": [round(x["model_err"], 5) for x in res["history"]]
                     + [round(res["final_model_err"], 5)],
                     "alpha": [x["alpha"] for x in res["history"]],
                     "trials": [x["trials"] for x in res["history"]],
                     "seconds": round(sec, 1)}
        del res
        torch.cuda.empty_cache()
        print(f"fwi: {name} done", file=sys.stderr, flush=True)
    return {"workload": f"{n}^3 salt model, 4 shots stacked, nt={nt}, r={r} (fresh probes per "
                        f"shot and iteration), k=32, bf16x2, fused; exact: checkpointed FP32",
            "iterations": iters, **out}


def bench_tti(shape, nt: int, r: int, stride: int):
    """Pseudo-acoustic TTI gradient, one shot: layered model with a salt
    ellipsoid, smooth eps / delta / tilt / azimuth fields, r probes on both
    fields (p, q), BF16X2 probe GEMM with fused imaging.  The TTI step (all of
    its kernels) is timed with HIP events on every stride-th step."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth
    wl, an = synth.workload_tti(shape=shape, nt=nt, r=r)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2", c_max=wl.c_ref)
    m = torch.from_numpy(wl.m).cuda()
    aniso = torch.from_numpy(an).cuda()
    del an
    q = torch.from_numpy(wl.q).cuda()
    Z = torch.from_numpy(wl.Z).cuda()
    d_obs = torch.zeros((nt, wl.rec_pos.shape[0]), device="cuda")
    from paper_2201_06914_amd.api import tti_workspace
    work = tti_workspace(plan, "cuda")
    print("tti: inputs resident", file=sys.stderr, flush=True)
    P.profile_enable(stride)
    from paper_2201_06914_amd.api import KERNEL_KINDS
    for k in KERNEL_KINDS:
        P.profile_read(k)
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = P.fwi_gradient_tti(plan, m, aniso, wl.src_pos, q, wl.rec_pos, d_obs, Z, fused=True,
                             work=work)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3
    f_ms, f_n = P.profile_read("tti_step")
    a_ms, a_n = P.profile_read("tti_step_adj")
    P.profile_enable(0)
    N = int(np.prod(shape))
    f_us = f_ms / max(f_n, 1) * 1e3
    a_us = a_ms / max(a_n, 1) * 1e3
    avg_us = 0.5 * (f_us + a_us)
    # algorithmic bytes of one step per cell: read p, q, their previous
    # levels, m and the five coefficients; write the two new levels (FP32)
    bpc = 12 * 4
    finite = bool(torch.isfinite(out["grad"]).all().item())
    print("tti: gradient done", file=sys.stderr, flush=True)
    tr = measured_traffic("tti", shape, r=r, k=32)

    def entry(kernel, key, us, n):
        gbs = bpc * N / (us * 1e-6) / 1e9
        e = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": round(tr[key]) if tr else None,
             "traffic_source": PMC_SOURCE if tr else None, "kernel": kernel,
             "avg_launch_us": round(us, 1), "launches_timed": n, "bytes_per_cell": bpc}
        v = valu_entry("tti", shape, key, us, N, r=r, k=32)
        if v:
            e["valu"] = v
        return e
    kern = {"tti_forward": entry("k_tti_ffused_ring (forward step, LDS plane ring, 3 planes per "
                                 "loop trip)",
                                 "tti_ffused", f_us, f_n),
            "tti_transpose": entry("k_tti_afused_dq (transpose step, LDS halo queues, one "
                                   "barrier per plane, p equation merged per axis, 6 planes "
                                   "per loop trip)", "tti_afused", a_us, a_n)}
    gbs = bpc * N / (avg_us * 1e-6) / 1e9
    return {"workload": f"TTI {shape[0]}x{shape[1]}x{shape[2]}, nt={nt}, r={r} on p and q, "
                        f"k=32, bf16x2, fused imaging, one shot",
            "value": round(2.0 * N * nt / (ms * 1e-3) / 1e9, 2), "unit": "Gcell-updates/s",
            "ms_per_gradient": round(ms, 1),
            "step_avg_us": round(avg_us, 1), "step_count_timed": f_n + a_n,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "traffic": round(0.5 * (tr["tti_ffused"] + tr["tti_afused"])) if tr
                         else None, "bytes_per_cell": bpc,
                         "note": "mean of the forward and transpose steps"},
            "roofline_kernels": kern,
            "misfit": float(out["misfit"].item()), "grad_finite": finite}


def hbm_copy_gbps(mib: int = 2048, reps: int = 5) -> float:
    """Measured HBM ceiling of a read-once / write-once kernel: the library's
    16-byte-vector streaming copy (rtm_device_copy) of mib MiB, read + write
    bytes over its HIP-event time on the stream it runs on."""
    import torch

    from paper_2201_06914_amd.api import device_copy
    nel = mib * (1 << 20) // 4
    x = torch.ones(nel, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    device_copy(x, y)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        device_copy(x, y)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    del x, y
    return 2.0 * nel * 4 / (ms * 1e-3) / 1e9


def bench_gathers(shape, r: int, nh: int):
    """Subsurface-offset image volume (Eq. 4) at the TTI grid: 2 nh + 1
    offsets along x from the p and q compressed fields (r probes each).  The
    kernel's cost does not depend on the values; the fields are seeded
    Gaussian noise of the compressed fields' shape."""
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    plan = P.Plan(P.PlanSpec(3, shape, 12.5, 1e-3, 64, 10, 4500.0, 1e-3, 4500.0, "f32", "bf16x2",
                             r, 32, 1, 1))
    gen = torch.Generator(device="cuda").manual_seed(11)
    nb = 2 * r * plan.Npad
    U = torch.randn(nb, generator=gen, device="cuda")
    V = torch.randn(nb, generator=gen, device="cuda")
    G = torch.empty((2 * nh + 1, plan.N), device="cuda")
    P.rtm_offset_gathers(plan, U, V, nh, nfield=2, out=G)       # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 3
    ev[0].record()
    for _ in range(reps):
        P.rtm_offset_gathers(plan, U, V, nh, nfield=2, out=G)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    N = int(np.prod(shape))
    alg = (2 * nb + (2 * nh + 1) * N) * 4.0
    macs = 2.0 * r * N * (2 * nh + 1)
    # the FP32 path is an MFMA contraction (v_mfma_f32_16x16x4f32): dense
    # FP32 matrix peak 157.3 TFLOP/s; achieved counts the needed products only
    tflops = 2 * macs / (ms * 1e-3) / 1e12
    tr = measured_traffic("gathers", shape, r=r, nh=nh)
    traffic = round(tr["gathers"] / 1e9, 2) if tr and "gathers" in tr else None
    return {"workload": f"{shape[0]}x{shape[1]}x{shape[2]}, {2 * nh + 1} offsets along x, r={r} "
                        f"on p and q, fp32", "ms": round(ms, 2),
            "GBps_algorithmic": round(alg / (ms * 1e-3) / 1e9, 1),
            "roofline": {"bound": "mfma", "achieved": round(tflops, 2), "peak": 157.3,
                         "unit": "TFLOP/s", "frac": round(tflops / 157.3, 3),
                         "hbm_frac": round(alg / (ms * 1e-3) / 8e12, 3)},
            "algorithmic_gb": round(alg / 1e9, 2), "traffic_gb": traffic,
            "output_gb": round((2 * nh + 1) * N * 4 / 1e9, 2)}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "the benchmark measures one GPU only; --gpus must be 1 "
                                   "(shot or z-slab sharding across GPUs is not built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2201_06914_amd as P
    import synth

    wl = synth.workload_c2(nt=a.nt, k_block=a.k_block)
    N, nt, r, k = wl.N, wl.nt, wl.r, a.k_block
    plan = P.Plan.for_workload(wl, field="f32", probe=a.probe, k_block=k)
    m = torch.from_numpy(wl.m).cuda()
    q = torch.from_numpy(wl.q).cuda()
    Z = torch.from_numpy(wl.Z).cuda()
    d_obs = torch.zeros((nt, wl.rec_pos.shape[0]), dtype=torch.float32, device="cuda")
    bars = (plan.empty_bar("cuda"), None if not a.unfused else plan.empty_bar("cuda"))
    work = plan.workspace("cuda")
    src, rec = wl.src_pos, wl.rec_pos
    del wl
    if a.stencil_variant is None:
        tune = P.autotune_stencil(plan, m, work=work, steps=20)
    else:
        P.set_stencil_variant(a.stencil_variant)
        P.set_stencil_blocks(a.stencil_blocks or 2048)
        tune = {"best": a.stencil_variant, "blocks": a.stencil_blocks or 2048, "fixed": True}
    print(f"stencil variant {tune}", file=sys.stderr, flush=True)

    fused = not a.unfused

    def step(fz=fused):
        return P.fwi_gradient(plan, m, src, q, rec, d_obs, Z, work=work, bars=bars, fused=fz)

    for i in range(a.warmup):
        step()
        torch.cuda.synchronize()
        print(f"warmup step {i} done", file=sys.stderr, flush=True)
    P.profile_enable(a.prof_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        out = step()
        if i + 1 < a.steps:      # one host round trip per step, for progress output
            out["misfit"].item()
            print(f"timed step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    P.profile_enable(0)
    ms_step = (t1 - t0) / a.steps * 1e3
    value = 2.0 * N * nt / (ms_step / 1e3) / 1e9
    st_ms, st_n = P.profile_read("stencil")
    pf_ms, pf_n = P.profile_read("probe")
    pa_ms, pa_n = P.profile_read("probe_adj")
    im_ms, im_n = P.profile_read("image")
    misfit = float(out["misfit"].item())
    finite = bool(torch.isfinite(out["grad"]).all().item())
    # one step of the other variant, for comparison
    other_ms, other_misfit = None, None
    if not a.no_other:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if fused:
            other = P.fwi_gradient(plan, m, src, q, rec, d_obs, Z, work=work)
        else:
            other = step(True)
        torch.cuda.synchronize()
        other_ms = (time.perf_counter() - t2) * 1e3
        other_misfit = float(other["misfit"].item())
        del other
        torch.cuda.empty_cache()
    # the exact gradient (Eq. 2, FP32, uniform checkpointing) on the same inputs
    exact = None
    ge = None
    g_probed = out["grad"].double()
    del out
    torch.cuda.empty_cache()
    if not a.no_exact:
        ewb = P.exact_workspace_bytes(plan)
        ework = torch.empty(ewb, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ex = P.fwi_gradient_exact(plan, m, src, q, rec, d_obs, work=ework)
        torch.cuda.synchronize()
        ex_ms = (time.perf_counter() - t3) * 1e3
        ge = ex["grad"].double()
        err = float(torch.linalg.vector_norm(g_probed - ge) / torch.linalg.vector_norm(ge))
        cos = float((g_probed * ge).sum() / (torch.linalg.vector_norm(g_probed)
                                             * torch.linalg.vector_norm(ge)))
        probed_bytes = plan.workspace_bytes + r * plan.Npad * 4     # ring + Ubar (fused)
        full_hist = nt * N * 4.0
        exact = {"exact_ms_per_step": round(ex_ms, 1),
                 "speedup_vs_exact": round(ex_ms / ms_step, 3),
                 "grad_rel_err_vs_exact": round(err, 4), "grad_cosine_vs_exact": round(cos, 4),
                 "misfit_rel_diff": abs(float(ex["misfit"].item()) - misfit) / misfit,
                 "memory_gb": {"probed_ring_plus_ubar": round(probed_bytes / 1e9, 2),
                               "exact_checkpointed": round(ewb / 1e9, 2),
                               "full_history_fp32": round(full_hist / 1e9, 1)},
                 "memory_reduction_vs_full_history": round(full_hist / probed_bytes, 1),
                 "memory_ratio_vs_checkpointed": round(ewb / probed_bytes, 2)}
        del ework, ex
        torch.cuda.empty_cache()
        print("exact comparator done", file=sys.stderr, flush=True)
    # probe block length: the same gradient with k = 64 and 128 (the ring grows
    # to k + 2 levels, the compressed field is read and written once per block)
    ksweep = None
    if not a.no_ksweep:
        import dataclasses
        ksweep = [{"k": k, "ms": round(ms_step, 1),
                   "probe_fwd_avg_us": round(pf_ms / max(pf_n, 1) * 1e3, 1),
                   "probe_adj_avg_us": round(pa_ms / max(pa_n, 1) * 1e3, 1),
                   "memory_gb_ring_plus_ubar": round((plan.workspace_bytes + r * plan.Npad * 4)
                                                     / 1e9, 2)}]
        if exact:
            ksweep[0]["speedup_vs_exact"] = exact["speedup_vs_exact"]
            ksweep[0]["grad_rel_err_vs_exact"] = exact["grad_rel_err_vs_exact"]
        for k2 in (64, 128):
            if k2 == k:
                continue
            p2 = P.Plan(dataclasses.replace(plan.spec, k_block=k2))
            w2 = p2.workspace("cuda")
            P.profile_enable(a.prof_stride)
            for kk in ("probe", "probe_adj"):
                P.profile_read(kk)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            o2 = P.fwi_gradient(p2, m, src, q, rec, d_obs, Z, work=w2, bars=bars, fused=fused)
            torch.cuda.synchronize()
            ms2 = (time.perf_counter() - t4) * 1e3
            P.profile_enable(0)
            f_ms, f_n = P.profile_read("probe")
            b_ms, b_n = P.profile_read("probe_adj")
            g2 = o2["grad"].double()
            row = {"k": k2, "ms": round(ms2, 1),
                   "value": round(2.0 * N * nt / (ms2 * 1e-3) / 1e9, 2),
                   "probe_fwd_avg_us": round(f_ms / max(f_n, 1) * 1e3, 1),
                   "probe_adj_avg_us": round(b_ms / max(b_n, 1) * 1e3, 1),
                   "probe_ms_per_gradient": round(f_ms + b_ms, 1),
                   "memory_gb_ring_plus_ubar": round((p2.workspace_bytes + r * plan.Npad * 4)
                                                     / 1e9, 2),
                   "grad_rel_diff_vs_k32": round(float(torch.linalg.vector_norm(g2 - g_probed)
                                                       / torch.linalg.vector_norm(g_probed)), 8)}
            if ge is not None:
                row["speedup_vs_exact"] = round(exact["exact_ms_per_step"] / ms2, 3)
                row["grad_rel_err_vs_exact"] = round(float(torch.linalg.vector_norm(g2 - ge)
                                                           / torch.linalg.vector_norm(ge)), 4)
            ksweep.append(row)
            del o2, g2, w2, p2
            torch.cuda.empty_cache()
            print(f"k sweep: k={k2} done", file=sys.stderr, flush=True)
        from paper_2201_06914_amd.tune import autotune_k_block
        kt = autotune_k_block(plan.spec, m, src, q, rec, Z, candidates=(16, 32, 64, 128))
        ksweep.append({"autotuned_k": kt["best"], "ms_per_step_256": kt["ms_per_step"],
                       "memory_gb": kt["memory_gb"]})
        torch.cuda.empty_cache()
        print(f"k autotune: {kt['best']}", file=sys.stderr, flush=True)
    del g_probed, ge
    torch.cuda.empty_cache()

    # algorithmic bytes (FP32 fields, FP32 compressed fields)
    st_bytes = 16.0 * N                                   # read u^n, u^{n-1}, m; write u^{n+1}
    nblk = math.ceil(nt / k)
    kbs = [min(k, nt - b * k) for b in range(nblk)]
    # forward blocks read kb + 2 levels (u_tt) and read + write Ubar; adjoint
    # blocks read kb levels and either read + write Vbar, or (fused) read Ubar
    # and read + write the image
    fwd_b = sum((4.0 * (kb + 2) + 8.0 * r) * N for kb in kbs)
    adj_b = sum((4.0 * kb + (4.0 * r + 8.0 if fused else 8.0 * r)) * N for kb in kbs)
    st_avg = st_ms / max(st_n, 1)
    st_ach = st_bytes / (st_avg * 1e-3) / 1e9
    pf_ach = fwd_b * a.steps / (pf_ms * 1e-3) / 1e9 if pf_n else 0.0
    pa_ach = adj_b * a.steps / (pa_ms * 1e-3) / 1e9 if pa_n else 0.0
    mfma_flop = (2 if a.probe == "bf16x2" else 1) * 2.0 * r * 16 * math.ceil(k / 16) * N * nblk
    tr = measured_traffic("acoustic", (384, 512, 512), r=r, k=k) if fused else None
    tr_src = ("stored rocprofv3 --pmc record profiles/pmc_traffic.json (FETCH_SIZE + WRITE_SIZE "
              "per dispatch, copy-calibrated), taken on these kernel sources (hash match), not "
              "measured in this run") if tr else None

    def entry(kernel, ach, avg_ms, n, bpl, ms_per_step, traffic, extra=None):
        e = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
             "traffic_source": tr_src if traffic is not None else None,
             "kernel": kernel, "avg_launch_us": round(avg_ms * 1e3, 2), "launches_timed": n,
             "bytes_per_launch": bpl, "ms_per_step": round(ms_per_step, 1)}
        e.update(extra or {})
        return e
    kern = {
        "probe_forward": entry(
            f"k_probe_mfma_fast (forward probe GEMM on u_tt, {a.probe}, k={k})", pf_ach,
            pf_ms / max(pf_n, 1), pf_n, fwd_b / nblk, pf_ms / a.steps,
            round(tr["probe_fwd"]) if tr else None,
            {"bytes_per_cell_per_block": 4 * (k + 2) + 8 * r,
             "mfma_tflops": round(mfma_flop * a.steps / (pf_ms * 1e-3) / 1e12, 2) if pf_n
             else None}),
        "probe_adjoint": entry(
            "k_probe_mfma_fast (adjoint probe GEMM" + (" with fused imaging)" if fused else ")"),
            pa_ach, pa_ms / max(pa_n, 1), pa_n, adj_b / nblk, pa_ms / a.steps,
            round(tr["probe_adj"]) if tr else None,
            {"bytes_per_cell_per_block": 4 * k + (4 * r + 8 if fused else 8 * r)}),
        "stencil": entry(
            f"k_stencil3d_tiled (variant {tune['best']}, z-march alternating)", st_ach, st_avg,
            st_n, st_bytes,
            st_avg * 2 * nt, round(tr["stencil"]) if tr else None,
            {"bytes_per_cell": 16, "z_split_target": tune.get("blocks"),
             "autotune_us": tune.get("us")}),
    }
    if fused:
        for name, key in (("probe_forward", "probe_fwd"), ("probe_adjoint", "probe_adj"),
                          ("stencil", "stencil")):
            v = valu_entry("acoustic", (384, 512, 512), key, kern[name]["avg_launch_us"], N,
                           r=r, k=k)
            if v:
                kern[name]["valu"] = v
    dom = max(kern, key=lambda kk: kern[kk]["ms_per_step"])
    pr_bytes_step = fwd_b + adj_b
    path_bytes = 2 * nt * st_bytes + pr_bytes_step
    rec_line = {
        "metric": "Gcell-updates/s fwd+adj w/ probing, %HBM peak; gradient rel. error vs exact",
        "value": round(value, 2), "unit": "Gcell-updates/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms_step, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3d-layered-384x512x512-nt{nt}-r{r}-k{k}", "grid": [384, 512, 512],
                   "nt": nt, "r": r, "k_block": k, "probe_operand": a.probe, "shots": 1,
                   "imaging": "fused" if fused else "separate", "parallelism": "single-gpu"},
        "roofline": dict(kern[dom], dominant=dom),
        "roofline_kernels": kern,
        "hbm_frac_path": round(path_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "grad_rel_err_vs_exact": exact["grad_rel_err_vs_exact"] if exact else None,
        "exact_comparator": exact,
        "k_sweep": ksweep,
        "misfit": misfit, "grad_finite": finite,
        ("unfused_ms_per_step" if fused else "fused_ms_per_step"):
            round(other_ms, 1) if other_ms is not None else None,
        "misfit_same_in_both": misfit == other_misfit if other_ms is not None else None,
        "image_avg_ms": round(im_ms / max(im_n, 1), 2),
    }
    try:
        cp = hbm_copy_gbps()
        rec_line["hbm_copy_GBps"] = round(cp, 1)
        rec_line["hbm_copy_kernel"] = "rtm_device_copy (k_copy_x4, 16-byte vectors), 2 GiB, HIP events"
        for e in kern.values():
            e["frac_of_copy"] = round(e["achieved"] / cp, 4)
        rec_line["roofline"]["frac_of_copy"] = kern[dom]["frac_of_copy"]
    except Exception as e:
        rec_line["hbm_copy_GBps"] = {"error": f"{type(e).__name__}: {e}"}
    if a.copy_calib_mb:      # a plain copy of known size, for PMC calibration
        from paper_2201_06914_amd.api import device_copy
        nel = a.copy_calib_mb * (1 << 20) // 4
        x = torch.ones(nel, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            device_copy(x, y)
        torch.cuda.synchronize()
        del x, y
    if not a.no_batched:
        del bars, work, m, q, Z, d_obs
        if "out" in locals():
            del out
        torch.cuda.empty_cache()
        try:
            rec_line["batched"] = bench_batched(a.batched_nt)
        except Exception as e:  # a failing section must not lose the headline line
            rec_line["batched"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not a.no_rsweep:
        torch.cuda.empty_cache()
        try:
            rec_line["rsweep"] = bench_rsweep(a.rsweep_n, a.rsweep_nt,
                                              tune["best"] if tune["best"] >= 1 else 7)
        except Exception as e:
            rec_line["rsweep"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not a.no_fwi:
        torch.cuda.empty_cache()
        try:
            rec_line["fwi"] = bench_fwi(a.rsweep_n, a.rsweep_nt, a.fwi_iters, 64,
                                        tune["best"] if tune["best"] >= 1 else 7)
        except Exception as e:
            rec_line["fwi"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not a.no_tti:
        torch.cuda.empty_cache()
        try:
            rec_line["tti"] = bench_tti((300, 400, 400), a.tti_nt, 64, a.prof_stride)
        except Exception as e:
            rec_line["tti"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not a.no_gathers:
        torch.cuda.empty_cache()
        try:
            rec_line["offset_gathers"] = bench_gathers((300, 400, 400), 64, 40)
        except Exception as e:
            rec_line["offset_gathers"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        torch.cuda.empty_cache()
        rec_line["cpu_baseline"], slab = cpu_baseline(a.cpu_planes, a.cpu_nt, r)
        try:
            rec_line["precision"] = bench_precision(slab, (384, 512, 512), 256, r, k,
                                                    tune["best"] if tune["best"] >= 1 else 7)
        except Exception as e:
            rec_line["precision"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(rec_line), flush=True)


if __name__ == "__main__":
    main()
