"""Autotuning of the sweep parameters that are not fixed by the method.

- autotune_k_block: the probe-block length k.  The level ring holds k + 2
  levels and the compressed field is read and written once per block, so the
  probe traffic per step falls as 1/k while the ring grows linearly in k.
  Each candidate whose workspace plus compressed field fits the memory limit
  runs the probed gradient over a truncated number of steps (a multiple of
  every candidate, so every block is full); the fastest per step wins.
- autotune_batch: the stencil kernel variant and the z-split target of a
  batch's tile table (rtm_set_stencil_blocks at rtm_batch_create), timed on
  the batch itself over a truncated number of steps.

Both only time library calls.  Choices are cached in a JSON file (default:
the RTM_TUNE_CACHE environment variable) keyed by the device architecture,
the grid(s), the field dtype, the probe dtype and r.
"""
from __future__ import annotations

import dataclasses
import json
import os
import time

import torch

from . import api


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name)


def _cache_get(cache, key):
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        return table.get(key)
    return None


def _cache_put(cache, key, value):
    if not cache:
        return
    table = {}
    if os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    table[key] = value
    with open(cache, "w") as f:
        json.dump(table, f, indent=1)


def _timed(fn, reps: int = 1) -> float:
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) * 1e3 / reps


def autotune_k_block(spec: api.PlanSpec, m, src_pos, q, rec_pos, Z, candidates=(16, 32, 64, 128),
                     steps: int = 256, mem_limit: int | None = None, fused: bool = True,
                     cache: str | None = None) -> dict:
    """Times fwi_gradient over the first `steps` time steps (q, Z and the data
    truncated; `steps` a multiple of every candidate) for each probe-block
    length k in `candidates` whose memory (workspace + Ubar, + Vbar when not
    fused) stays below mem_limit (default: 90 % of the free device memory).
    Returns {"best": k, "ms_per_step": {k: ms}, "memory_gb": {k: GB}}."""
    if cache is None:
        cache = os.environ.get("RTM_TUNE_CACHE") or None
    dev = m.device
    key = (f"kblock|{_arch(dev)}|{'x'.join(map(str, spec.shape))}|{spec.field}|{spec.probe}|"
           f"r{spec.r}|{'fused' if fused else 'separate'}")
    hit = _cache_get(cache, key)
    if hit:
        return dict(hit, cached=True)
    if mem_limit is None:
        free, _ = torch.cuda.mem_get_info(dev)
        mem_limit = int(0.9 * free)
    nt = min(steps, spec.nt)
    qt, Zt = q[:nt].contiguous(), Z[:nt].contiguous()
    d_obs = torch.zeros((nt, spec.nrec), dtype=m.dtype, device=dev)
    times, mem = {}, {}
    for k in candidates:
        if k > 128 and spec.probe in ("bf16", "bf16x2", "f16s"):
            continue
        sp = dataclasses.replace(spec, k_block=k, nt=nt)
        plan = api.Plan(sp)
        need = plan.workspace_bytes + (1 if fused else 2) * spec.r * plan.Npad * plan.dtype.itemsize
        mem[k] = round(need / 1e9, 2)
        if need > mem_limit:
            continue
        work = plan.workspace(dev)
        bars = (plan.empty_bar(dev), None if fused else plan.empty_bar(dev))

        def run():
            api.fwi_gradient(plan, m, src_pos, qt, rec_pos, d_obs, Zt, work=work, bars=bars,
                             fused=fused)
        run()                                    # first call: code objects, clocks
        times[k] = round(_timed(run) / nt, 4)
        del work, bars, plan
        torch.cuda.empty_cache()
    if not times:
        raise RuntimeError("no probe-block length fits the memory limit")
    best = min(times, key=times.get)
    res = {"best": best, "ms_per_step": times, "memory_gb": mem, "steps_timed": nt}
    _cache_put(cache, key, res)
    return dict(res, cached=False)


def autotune_batch(specs, shots, variants=(1, 3, 7, 11, 12), blocks=(2048, 4096, 8192),
                   steps: int = 128, cache: str | None = None, k_blocks=(32, 64, 128)) -> dict:
    """Times the batched gradient over the first `steps` time steps (a
    multiple of every k) for every (stencil variant, z-split target) pair,
    recreating the batch for each target (the tile table is fixed when a
    batch is created), then, with the best pair, every probe-block length in
    k_blocks whose memory fits.  shots: the per-shot input dicts of
    Batch.fwi_gradient.  Applies nothing; returns {"best": (variant, blocks),
    "k_block": k, ...}.  Apply with api.set_stencil_blocks(blocks) before
    creating the batch (with k_block = k in its descriptors) and
    api.set_stencil_variant(variant) before running it."""
    if cache is None:
        cache = os.environ.get("RTM_TUNE_CACHE") or None
    dev = shots[0]["m"].device
    key = ("batch|" + _arch(dev) + "|" + ";".join("x".join(map(str, s.shape)) for s in specs)
           + f"|{specs[0].field}|{specs[0].probe}|r{specs[0].r}|k{','.join(map(str, k_blocks))}")
    hit = _cache_get(cache, key)
    if hit:
        hit = dict(hit, cached=True)
        hit["best"] = tuple(hit["best"])
        return hit
    nt = min(steps, specs[0].nt)
    tspecs = [dataclasses.replace(s, nt=nt) for s in specs]
    tshots = [dict(sh, q=sh["q"][:nt].contiguous(), Z=sh["Z"][:nt].contiguous(),
                   d_obs=sh["d_obs"][:nt].contiguous()) for sh in shots]
    ms = {}
    blocks_before = api.get_stencil_blocks()
    for b in blocks:
        api.set_stencil_blocks(b)
        B = api.Batch(tspecs)
        outs = B.outputs(dev)
        J = torch.empty(len(shots), dtype=torch.float64, device=dev)
        work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device=dev)
        for v in variants:
            api.set_stencil_variant(v)
            B.fwi_gradient(tshots, outs=outs, misfit=J, work=work)
            ms[f"{v}/{b}"] = round(_timed(lambda: B.fwi_gradient(tshots, outs=outs, misfit=J,
                                                                   work=work)) / nt, 4)
        del B, outs, work
        torch.cuda.empty_cache()
    best = min(ms, key=ms.get)
    v, b = (int(x) for x in best.split("/"))
    # then the probe-block length with that stencil choice (memory permitting)
    kms = {}
    if k_blocks:
        free, _ = torch.cuda.mem_get_info(dev)
        api.set_stencil_blocks(b)
        api.set_stencil_variant(v)
        for k in k_blocks:
            kspecs = [dataclasses.replace(sp, k_block=k) for sp in tspecs]
            B = api.Batch(kspecs)
            need = B.workspace_bytes + sum(sp.r * ((n + 31) // 32 * 32) * 4
                                           for sp, n in zip(kspecs, B.N))
            if need > 0.9 * free:
                continue
            outs = B.outputs(dev, stack=False)
            J = torch.empty(len(shots), dtype=torch.float64, device=dev)
            work = torch.empty(B.workspace_bytes, dtype=torch.uint8, device=dev)
            B.fwi_gradient(tshots, outs=outs, misfit=J, work=work)
            kms[k] = round(_timed(lambda: B.fwi_gradient(tshots, outs=outs, misfit=J,
                                                         work=work)) / nt, 4)
            del B, outs, work
            torch.cuda.empty_cache()
    api.set_stencil_blocks(blocks_before)
    kbest = min(kms, key=kms.get) if kms else specs[0].k_block
    res = {"best": [v, b], "k_block": kbest, "ms_per_step": ms, "k_ms_per_step": kms,
           "steps_timed": nt}
    _cache_put(cache, key, res)
    return dict(res, best=(v, b), cached=False)
