"""Python binding of librtm: same names as the C ABI, torch tensors in and out.

Only argument marshalling happens here - every step of the sweeps runs in the
HIP kernels of librtm.so.  PyTorch provides device memory (outputs and the
workspace) and the current HIP stream.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib

_FIELD = {"f64": _lib.RTM_F64, "f32": _lib.RTM_F32}
_PROBE = {"f64": _lib.RTM_F64, "f32": _lib.RTM_F32, "bf16": _lib.RTM_BF16,
          "bf16x2": _lib.RTM_BF16X2, "f16s": _lib.RTM_F16S}
_TORCH = {"f64": torch.float64, "f32": torch.float32}


class RtmError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = _lib.load()
        msg = L.rtm_status_str(code).decode()
        detail = L.rtm_last_error().decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))
        self.code = code


def _check(code: int, where: str):
    if code != 0:
        raise RtmError(code, where)


@dataclasses.dataclass(frozen=True)
class PlanSpec:
    ndim: int
    shape: tuple          # (nz, ny, nx)
    h: float
    dt: float
    nt: int
    nb: int
    c_ref: float
    R: float
    c_max: float
    field: str = "f32"    # "f64" | "f32"
    probe: str = "bf16x2" # "f64" | "f32" | "bf16" | "bf16x2" | "f16s"
    r: int = 1
    k_block: int = 32
    nsrc: int = 1
    nrec: int = 0


class Plan:
    """Owns an rtm_plan (host object).  Immutable after creation."""

    def __init__(self, spec: PlanSpec):
        L = _lib.load()
        self.spec = spec
        d = _lib.RtmDesc()
        d.ndim = spec.ndim
        d.nz, d.ny, d.nx = (int(s) for s in spec.shape)
        d.h, d.dt, d.nt, d.nb = spec.h, spec.dt, spec.nt, spec.nb
        d.c_ref, d.R, d.c_max = spec.c_ref, spec.R, spec.c_max
        d.field_dtype = _FIELD[spec.field]
        d.probe_dtype = _PROBE[spec.probe]
        d.r, d.k_block, d.nsrc, d.nrec = spec.r, spec.k_block, spec.nsrc, spec.nrec
        h = ctypes.c_void_p()
        _check(L.rtm_plan_create(ctypes.byref(d), ctypes.byref(h)), "rtm_plan_create")
        self._h = h
        self._destroy = L.rtm_plan_destroy
        n = ctypes.c_size_t()
        _check(L.rtm_plan_workspace_bytes(h, ctypes.byref(n)), "rtm_plan_workspace_bytes")
        self.workspace_bytes = int(n.value)
        self.N = int(np.prod(spec.shape))
        self.Npad = (self.N + 31) // 32 * 32      # compressed fields: whole 32-cell tiles
        self.dtype = _TORCH[spec.field]

    @classmethod
    def for_workload(cls, wl, field: str = "f32", probe: str = "bf16x2", k_block=None,
                     c_max=None) -> "Plan":
        m = np.asarray(wl.m, dtype=np.float64)
        vmax = float(np.sqrt(1.0 / m.min())) if c_max is None else c_max
        return cls(PlanSpec(wl.ndim, tuple(wl.shape), wl.h, wl.dt, wl.nt, wl.nb, wl.c_ref, wl.R,
                            vmax, field, probe, wl.r, k_block or wl.k_block,
                            int(np.shape(wl.src_pos)[0]), int(np.shape(wl.rec_pos)[0])))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def empty_bar(self, device="cuda") -> torch.Tensor:
        """A compressed-field buffer: tile-major [Npad/32][r][32]."""
        return torch.empty((self.Npad // 32, self.spec.r, 32), dtype=self.dtype, device=device)


def _desc(spec: PlanSpec) -> _lib.RtmDesc:
    d = _lib.RtmDesc()
    d.ndim = spec.ndim
    d.nz, d.ny, d.nx = (int(v) for v in spec.shape)
    d.h, d.dt, d.nt, d.nb = spec.h, spec.dt, spec.nt, spec.nb
    d.c_ref, d.R, d.c_max = spec.c_ref, spec.R, spec.c_max
    d.field_dtype = _FIELD[spec.field]
    d.probe_dtype = _PROBE[spec.probe]
    d.r, d.k_block, d.nsrc, d.nrec = spec.r, spec.k_block, spec.nsrc, spec.nrec
    return d


class Batch:
    """Several shots (sub-domain windows of different sizes) advanced together:
    one stencil launch per time step for all shots, optional HIP-graph replay
    of the whole gradient (rtm_batch_create / fwi_gradient_batched)."""

    def __init__(self, specs):
        L = _lib.load()
        self.specs = list(specs)
        arr = (_lib.RtmDesc * len(self.specs))(*[_desc(sp) for sp in self.specs])
        h = ctypes.c_void_p()
        _check(L.rtm_batch_create(arr, len(self.specs), ctypes.byref(h)), "rtm_batch_create")
        self._h = h
        self._destroy = L.rtm_batch_destroy
        n = ctypes.c_size_t()
        _check(L.rtm_batch_workspace_bytes(h, ctypes.byref(n)), "rtm_batch_workspace_bytes")
        self.workspace_bytes = int(n.value)
        self.N = [int(np.prod(sp.shape)) for sp in self.specs]
        self.Npad = [(n_ + 31) // 32 * 32 for n_ in self.N]
        self._stream = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._destroy(h)
            self._h = None

    def outputs(self, device="cuda", stack: bool = False) -> list:
        """Preallocated per-shot outputs (reuse them to replay a captured graph).
        stack=True gives every shot the same gradient buffer (the shots must
        share one grid): fwi_gradient then returns the stacked gradient, the
        sum over shots, in each outs[i]["grad"]."""
        outs = []
        shared = None
        if stack:
            if len({tuple(sp.shape) for sp in self.specs}) != 1:
                raise ValueError("stacking needs every shot on the same grid")
            shared = torch.empty(self.N[0], dtype=torch.float32, device=device)
        for sp, n, npad in zip(self.specs, self.N, self.Npad):
            outs.append({"Ubar": torch.empty((npad // 32, sp.r, 32), dtype=torch.float32,
                                             device=device),
                         "resid": torch.empty((sp.nt, sp.nrec), dtype=torch.float32, device=device),
                         "grad": shared if stack else torch.empty(n, dtype=torch.float32,
                                                                  device=device)})
        return outs

    def stream_status(self, work: torch.Tensor) -> bool:
        """True if the last fwi_gradient call on `work` kept every checked value
        finite; False if it met a NaN or an infinity.  Synchronizes."""
        code = _lib.load().rtm_batch_stream_status(self._h, ctypes.c_void_p(work.data_ptr()),
                                                   _stream(work.device))
        if code == _lib.RTM_E_NONFINITE:
            return False
        _check(code, "rtm_batch_stream_status")
        return True

    def fwi_gradient(self, shots, outs=None, misfit=None, use_graph=False, work=None):
        """shots: per shot dict(m, src_pos, q, rec_pos, d_obs, Z).  Returns
        (outs, misfit) with outs[i] = dict(Ubar, resid, grad)."""
        dev = shots[0]["m"].device
        outs = outs if outs is not None else self.outputs(dev)
        misfit = misfit if misfit is not None else torch.empty(len(shots), dtype=torch.float64,
                                                               device=dev)
        if work is None:
            work = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
        io = (_lib.ShotIO * len(shots))()
        keep = []
        for i, (sp, sh, o) in enumerate(zip(self.specs, shots, outs)):
            sa, sap = _pos(sh["src_pos"], sp.nsrc, "src_pos")
            ra, rap = _pos(sh["rec_pos"], sp.nrec, "rec_pos")
            keep += [sa, ra]
            io[i].m = _dev(sh["m"], torch.float32, self.N[i], "m")
            io[i].src_pos = sap
            io[i].q = _dev(sh["q"], torch.float32, sp.nt * sp.nsrc, "q")
            io[i].rec_pos = rap
            io[i].d_obs = _dev(sh["d_obs"], torch.float32, sp.nt * sp.nrec, "d_obs")
            io[i].Z = _dev(sh["Z"], torch.int8, sp.nt * sp.r, "Z")
            io[i].Ubar = _dev(o["Ubar"], torch.float32, sp.r * self.Npad[i], "Ubar")
            io[i].resid = _dev(o["resid"], torch.float32, sp.nt * sp.nrec, "resid")
            io[i].grad = _dev(o["grad"], torch.float32, self.N[i], "grad")
        L = _lib.load()
        if use_graph:
            # a capture needs a non-default stream (default priority)
            if self._stream is None:
                self._stream = torch.cuda.Stream(device=dev)
            cur = torch.cuda.current_stream(dev)
            self._stream.wait_stream(cur)
            with torch.cuda.stream(self._stream):
                code = L.fwi_gradient_batched(self._h, io, _dev(misfit, torch.float64,
                                                                len(shots), "misfit"), 1,
                                              ctypes.c_void_p(work.data_ptr()), work.numel(),
                                              _stream(dev))
            cur.wait_stream(self._stream)
        else:
            code = L.fwi_gradient_batched(self._h, io, _dev(misfit, torch.float64, len(shots),
                                                            "misfit"), 0,
                                          ctypes.c_void_p(work.data_ptr()), work.numel(),
                                          _stream(dev))
        _check(code, "fwi_gradient_batched")
        return outs, misfit


def cfl_bound(ndim: int) -> float:
    return float(_lib.load().rtm_cfl_bound(ndim))


def set_stencil_variant(v: int) -> None:
    _lib.load().rtm_set_stencil_variant(int(v))


N_STENCIL_VARIANTS = 14


def set_probe_nt(on: bool) -> None:
    """Non-temporal compressed-field traffic in the probe kernels (default on)."""
    _lib.load().rtm_set_probe_nt(1 if on else 0)


def set_probe_grid(update: int, fused: int) -> None:
    """Workgroups of one probe-GEMM launch for the in-place update kernels and
    for the fused adjoint imaging kernel: -1 automatic (default), -2 work
    queue, 0 one per four tiles, > 0 at most that many."""
    _lib.load().rtm_set_probe_grid(int(update), int(fused))


def set_graph(on: bool) -> None:
    """fwi_gradient captures and replays HIP graphs (per set of arguments)."""
    _lib.load().rtm_set_graph(1 if on else 0)


def set_stencil_alternate(on: bool) -> None:
    """Tiled stencil marches z up / down on alternate steps (default on)."""
    _lib.load().rtm_set_stencil_alternate(1 if on else 0)


_STENCIL_BLOCKS = [2048]    # the value last set in this process (the library's default)


def set_stencil_blocks(blocks: int) -> None:
    _lib.load().rtm_set_stencil_blocks(int(blocks))
    _STENCIL_BLOCKS[0] = int(blocks) if blocks > 0 else 2048


def get_stencil_blocks() -> int:
    return _STENCIL_BLOCKS[0]


def autotune_stencil(plan: Plan, m, work=None, steps: int = 20, apply: bool = True,
                     cache: str | None = None, blocks=(768, 1024, 1536, 2048, 4096)) -> dict:
    """Times every stencil variant on this plan's grid (after checking each
    against the one-thread-per-cell kernel bit for bit, in both z-marching
    directions) for each z-split target in `blocks`, and with apply=True
    selects the fastest (variant, target) pair.  `cache`: a JSON file keyed by
    (arch, grid, dtype) that stores the choice across runs (default: the
    RTM_TUNE_CACHE environment variable, if set)."""
    import json
    import os
    if cache is None:
        cache = os.environ.get("RTM_TUNE_CACHE") or None
    key = None
    if cache:
        props = torch.cuda.get_device_properties(m.device)
        arch = getattr(props, "gcnArchName", props.name)
        key = f"{arch}|{plan.spec.ndim}|{'x'.join(map(str, plan.spec.shape))}|{plan.spec.field}"
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                if apply:
                    set_stencil_variant(table[key]["best"])
                    set_stencil_blocks(table[key].get("blocks", 2048))
                return dict(table[key], cached=True)
    work = _work(plan, work, m.device)
    blocks_before = get_stencil_blocks()
    last = N_STENCIL_VARIANTS if plan.spec.ndim == 3 else 1
    us_all, mism_all = {}, [0] * last
    best = (None, None, float("inf"))
    for b in blocks:
        set_stencil_blocks(b)
        bv = ctypes.c_int32()
        us = (ctypes.c_float * N_STENCIL_VARIANTS)()
        mism = (ctypes.c_int64 * N_STENCIL_VARIANTS)()
        _check(_lib.load().rtm_autotune_stencil(plan.handle, _dev(m, plan.dtype, plan.N, "m"),
                                                ctypes.c_void_p(work.data_ptr()), work.numel(),
                                                int(steps), ctypes.byref(bv), us, mism,
                                                _stream(m.device)), "rtm_autotune_stencil")
        us_all[b] = [round(float(us[i]), 2) for i in range(last)]
        mism_all = [max(mism_all[i], int(mism[i])) for i in range(last)]
        v = int(bv.value)
        if us_all[b][v] < best[2]:
            best = (v, b, us_all[b][v])
    res = {"best": best[0], "blocks": best[1], "us": us_all, "mismatch": mism_all, "cached": False}
    set_stencil_blocks(res["blocks"] if apply else blocks_before)
    if apply:
        set_stencil_variant(res["best"])
    if cache and key:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = {k: v for k, v in res.items() if k != "cached"}
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return res


KERNEL_KINDS = {"stencil": 0, "probe": 1, "image": 2, "probe_adj": 3, "tti_step": 4,
                "tti_step_adj": 5}


def profile_enable(stride: int) -> None:
    """Time every stride-th stencil launch and every probe / image launch with
    HIP events on the sweep's stream (0 = off)."""
    _lib.load().rtm_profile_enable(int(stride))


def profile_read(kind: str):
    """(total_ms, count) of the timed launches of one kernel kind."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(_lib.load().rtm_profile_read(KERNEL_KINDS[kind], ctypes.byref(ms), ctypes.byref(n)),
           "rtm_profile_read")
    return float(ms.value), int(n.value)


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def _dev(t: torch.Tensor, dtype, numel: int, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _pos(p, n: int, name: str):
    if p is None:
        return None, None
    a = np.ascontiguousarray(np.reshape(p, (-1, 3)), dtype=np.float64)
    if a.shape[0] != n:
        raise ValueError(f"{name} has {a.shape[0]} points, the plan expects {n}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _z(plan: Plan, Z: torch.Tensor):
    s = plan.spec
    if Z is None:
        return None, _lib.RTM_I8
    if Z.dtype == torch.int8:
        zt = _lib.RTM_I8
    elif Z.dtype == plan.dtype:
        zt = _PROBE[s.field]
    else:
        raise TypeError("Z must be int8 (+-1) or the plan's field dtype")
    return _dev(Z, Z.dtype, s.nt * s.r, "Z"), zt


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _work(plan: Plan, work, device):
    if work is None:
        work = plan.workspace(device)
    if work.numel() < plan.workspace_bytes or not work.is_cuda:
        raise ValueError("workspace too small")
    return work


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def rtm_forward_probe(plan: Plan, m, src_pos, q, rec_pos=None, Z=None, what: str = "utt",
                      want_d: bool = True, final: bool = False, work=None) -> dict:
    s = plan.spec
    dev = m.device
    out = {}
    d = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev) if want_d else None
    U = plan.empty_bar(dev) if Z is not None else None
    F = torch.empty((2, plan.N), dtype=plan.dtype, device=dev) if final else None
    work = _work(plan, work, dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos") if want_d else (None, None)
    zp, zt = _z(plan, Z)
    code = _lib.load().rtm_forward_probe(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp, _dev(d, plan.dtype, s.nt * s.nrec, "d"),
        zp, zt, _lib.RTM_PROBE_UTT if what == "utt" else _lib.RTM_PROBE_U,
        _dev(U, plan.dtype, s.r * plan.Npad, "Ubar"), _dev(F, plan.dtype, 2 * plan.N, "final"),
        ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev))
    _check(code, "rtm_forward_probe")
    if d is not None:
        out["d"] = d
    if U is not None:
        out["Ubar"] = U
    if F is not None:
        out["final"] = F
    return out


def rtm_forward_probe_range(plan: Plan, m, src_pos, q, rec_pos, Z, n_begin: int, n_end: int,
                            state_in=None, Ubar=None, d=None, what: str = "utt",
                            work=None) -> dict:
    """Forward sweep over steps n_begin .. n_end - 1 (ends on probe-block
    boundaries) from state_in = (u^{n_begin}, u^{n_begin - 1}); Ubar and d
    carry over from the previous range (fresh ones when n_begin = 0).
    Returns {"d", "Ubar", "state"} with state = (u^{n_end}, u^{n_end - 1})."""
    s = plan.spec
    dev = m.device
    if d is None:
        d = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev)
    U = Ubar if Ubar is not None else plan.empty_bar(dev)
    F = torch.empty((2, plan.N), dtype=plan.dtype, device=dev)
    work = _work(plan, work, dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    zp, zt = _z(plan, Z)
    code = _lib.load().rtm_forward_probe_range(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp, _dev(d, plan.dtype, s.nt * s.nrec, "d"),
        zp, zt, _lib.RTM_PROBE_UTT if what == "utt" else _lib.RTM_PROBE_U,
        _dev(U, plan.dtype, s.r * plan.Npad, "Ubar"), int(n_begin), int(n_end),
        _dev(state_in, plan.dtype, 2 * plan.N, "state_in"), _dev(F, plan.dtype, 2 * plan.N, "state"),
        ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev))
    _check(code, "rtm_forward_probe_range")
    return {"d": d, "Ubar": U, "state": F}


def rtm_adjoint_probe(plan: Plan, m, rec_pos, res, Z=None, src_pos=None, want_qadj=False,
                      work=None) -> dict:
    s = plan.spec
    dev = m.device
    V = plan.empty_bar(dev) if Z is not None else None
    qa = torch.empty((s.nt, s.nsrc), dtype=plan.dtype, device=dev) if want_qadj else None
    work = _work(plan, work, dev)
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    sp, spp = _pos(src_pos, s.nsrc, "src_pos") if want_qadj else (None, None)
    zp, zt = _z(plan, Z)
    code = _lib.load().rtm_adjoint_probe(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), rpp,
        _dev(res, plan.dtype, s.nt * s.nrec, "res"), spp,
        _dev(qa, plan.dtype, s.nt * s.nsrc, "qadj"), zp, zt,
        _dev(V, plan.dtype, s.r * plan.Npad, "Vbar"), ctypes.c_void_p(work.data_ptr()),
        work.numel(), _stream(dev))
    _check(code, "rtm_adjoint_probe")
    out = {}
    if V is not None:
        out["Vbar"] = V
    if qa is not None:
        out["qadj"] = qa
    return out


def rtm_image(plan: Plan, Ubar, Vbar, scale: float | None = None) -> torch.Tensor:
    s = plan.spec
    scale = 1.0 / s.r if scale is None else scale
    img = torch.empty(plan.N, dtype=plan.dtype, device=Ubar.device)
    _check(_lib.load().rtm_image(
        plan.handle, _dev(Ubar, plan.dtype, s.r * plan.Npad, "Ubar"),
        _dev(Vbar, plan.dtype, s.r * plan.Npad, "Vbar"), float(scale),
        _dev(img, plan.dtype, plan.N, "image"), _stream(Ubar.device)), "rtm_image")
    return img


def fwi_gradient(plan: Plan, m, src_pos, q, rec_pos, d_obs, Z, work=None, bars=None,
                 fused: bool = False) -> dict:
    """Probed FWI gradient.  `bars` may pass preallocated (Ubar, Vbar).  With
    fused=True (BF16 probe paths) the imaging condition is folded into the
    adjoint probe blocks and no Vbar is produced."""
    s = plan.spec
    dev = m.device
    if bars is None:
        U = plan.empty_bar(dev)
        V = None if fused else plan.empty_bar(dev)
    else:
        U, V = bars
        if fused:
            V = None
    res = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev)
    g = torch.empty(plan.N, dtype=plan.dtype, device=dev)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    work = _work(plan, work, dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")   # keep the arrays alive over the call
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    zp, zt = _z(plan, Z)
    code = _lib.load().fwi_gradient(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d_obs, plan.dtype, s.nt * s.nrec, "d_obs"), zp, zt,
        _dev(U, plan.dtype, s.r * plan.Npad, "Ubar"), _dev(V, plan.dtype, s.r * plan.Npad, "Vbar"),
        _dev(res, plan.dtype, s.nt * s.nrec, "resid"), _dev(g, plan.dtype, plan.N, "grad"),
        _dev(J, torch.float64, 1, "misfit"), ctypes.c_void_p(work.data_ptr()), work.numel(),
        _stream(dev))
    _check(code, "fwi_gradient")
    return {"grad": g, "misfit": J, "Ubar": U, "Vbar": V, "resid": res}


def fwi_gradient_noalloc(plan: Plan, m, src_pos, q, rec_pos, d_obs, Z, bars, resid, grad,
                         misfit) -> None:
    """fwi_gradient with the workspace in the library's static device array
    (no device allocation in the call): every output is passed in.  bars =
    (Ubar, Vbar) with Vbar None for fused imaging; resid [nt][nrec], grad [N]
    of the plan's dtype, misfit FP64 [1]."""
    s = plan.spec
    dev = m.device
    U, V = bars
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    zp, zt = _z(plan, Z)
    code = _lib.load().fwi_gradient_noalloc(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d_obs, plan.dtype, s.nt * s.nrec, "d_obs"), zp, zt,
        _dev(U, plan.dtype, s.r * plan.Npad, "Ubar"), _dev(V, plan.dtype, s.r * plan.Npad, "Vbar"),
        _dev(resid, plan.dtype, s.nt * s.nrec, "resid"), _dev(grad, plan.dtype, plan.N, "grad"),
        _dev(misfit, torch.float64, 1, "misfit"), _stream(dev))
    _check(code, "fwi_gradient_noalloc")


def fwi_gradient_exact(plan: Plan, m, src_pos, q, rec_pos, d_obs, checkpoint_every: int = 0,
                       work=None) -> dict:
    """Exact gradient (Eq. 2) with uniform checkpointing; the comparator of
    the probed gradient.  checkpoint_every = 0 picks ceil(sqrt(2 nt))."""
    s = plan.spec
    dev = m.device
    L = _lib.load()
    n = ctypes.c_size_t()
    _check(L.rtm_exact_workspace_bytes(plan.handle, int(checkpoint_every), ctypes.byref(n)),
           "rtm_exact_workspace_bytes")
    if work is None or work.numel() < n.value:
        work = torch.empty(n.value, dtype=torch.uint8, device=dev)
    res = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev)
    g = torch.empty(plan.N, dtype=plan.dtype, device=dev)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    code = L.fwi_gradient_exact(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d_obs, plan.dtype, s.nt * s.nrec, "d_obs"), int(checkpoint_every),
        _dev(res, plan.dtype, s.nt * s.nrec, "resid"), _dev(g, plan.dtype, plan.N, "grad"),
        _dev(J, torch.float64, 1, "misfit"), ctypes.c_void_p(work.data_ptr()), work.numel(),
        _stream(dev))
    _check(code, "fwi_gradient_exact")
    return {"grad": g, "misfit": J, "resid": res, "workspace_bytes": int(n.value)}


def rtm_offset_gathers(plan: Plan, Ubar, Vbar, nh: int, scale=None, nfield: int = 1,
                       out=None) -> torch.Tensor:
    """Eq. 4 along x: [2 nh + 1][N] image volume, offset -nh first; scale
    defaults to 1/r."""
    s = plan.spec
    dev = Ubar.device
    nb = nfield * s.r * plan.Npad
    G = out if out is not None else torch.empty((2 * nh + 1, plan.N), dtype=plan.dtype,
                                                device=dev)
    _check(_lib.load().rtm_offset_gathers(
        plan.handle, _dev(Ubar, plan.dtype, nb, "Ubar"), _dev(Vbar, plan.dtype, nb, "Vbar"),
        int(nfield), int(nh), float(1.0 / s.r if scale is None else scale),
        _dev(G, plan.dtype, (2 * nh + 1) * plan.N, "gathers"), _stream(dev)),
        "rtm_offset_gathers")
    return G


def rtm_residual(plan: Plan, d_pred, d_obs, resid=None, work=None):
    """(resid, misfit): resid = d_pred - d_obs, misfit = 1/2 sum resid^2 (FP64,
    device tensor [1]).  resid may be d_pred itself."""
    s = plan.spec
    dev = d_pred.device
    resid = resid if resid is not None else torch.empty_like(d_pred)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    work = _work(plan, work, dev)
    n = s.nt * s.nrec
    _check(_lib.load().rtm_residual(plan.handle, _dev(d_pred, plan.dtype, n, "d_pred"),
                                    _dev(d_obs, plan.dtype, n, "d_obs"),
                                    _dev(resid, plan.dtype, n, "resid"),
                                    _dev(J, torch.float64, 1, "misfit"),
                                    ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev)),
           "rtm_residual")
    return resid, J


def stream_status(plan: Plan, work: torch.Tensor) -> bool:
    """True if the last sweeping call on this workspace kept every checked
    value finite (final wavefield levels, gradient / image, misfit); False if
    it met a NaN or an infinity.  Synchronizes the current stream."""
    code = _lib.load().rtm_stream_status(plan.handle, ctypes.c_void_p(work.data_ptr()),
                                         _stream(work.device))
    if code == _lib.RTM_E_NONFINITE:
        return False
    _check(code, "rtm_stream_status")
    return True


def rf_workspace_bytes(plan: Plan) -> int:
    n = ctypes.c_size_t()
    _check(_lib.load().rtm_rf_workspace_bytes(plan.handle, ctypes.byref(n)),
           "rtm_rf_workspace_bytes")
    return int(n.value)


def _rf_work(plan: Plan, work, device):
    n = rf_workspace_bytes(plan)
    if work is None:
        work = torch.empty(n, dtype=torch.uint8, device=device)
    if work.numel() < n or not work.is_cuda:
        raise ValueError("workspace too small for the range-finder calls")
    return work


def rtm_sketch(plan: Plan, m, src_pos, q, seed: int, work=None) -> torch.Tensor:
    """Y [nt][r] (FP64): the space sketch H Omega of the u_tt history."""
    s = plan.spec
    dev = m.device
    work = _rf_work(plan, work, dev)
    Y = torch.empty((s.nt, s.r), dtype=torch.float64, device=dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    _check(_lib.load().rtm_sketch(plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
                                  _dev(q, plan.dtype, s.nt * s.nsrc, "q"), int(seed),
                                  _dev(Y, torch.float64, s.nt * s.r, "Y"),
                                  ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev)),
           "rtm_sketch")
    return Y


def rtm_orthonormalize(plan: Plan, Y, work=None) -> torch.Tensor:
    """Q [nt][r] (field dtype): orthonormal columns spanning the columns of Y."""
    s = plan.spec
    dev = Y.device
    work = _rf_work(plan, work, dev)
    Q = torch.empty((s.nt, s.r), dtype=plan.dtype, device=dev)
    _check(_lib.load().rtm_orthonormalize(plan.handle, _dev(Y, torch.float64, s.nt * s.r, "Y"),
                                          _dev(Q, plan.dtype, s.nt * s.r, "Q"),
                                          ctypes.c_void_p(work.data_ptr()), work.numel(),
                                          _stream(dev)), "rtm_orthonormalize")
    return Q


def fwi_gradient_rf(plan: Plan, m, src_pos, q, rec_pos, d_obs, seed: int, fused=None,
                    work=None) -> dict:
    """Probed gradient with range-finder probes Q = orth(H Omega), scale -1.
    fused (default: on for BF16X2 plans) folds the imaging into the adjoint
    probe blocks and stores no Vbar."""
    s = plan.spec
    dev = m.device
    work = _rf_work(plan, work, dev)
    if fused is None:
        fused = s.probe == "bf16x2"
    Q = torch.empty((s.nt, s.r), dtype=plan.dtype, device=dev)
    U = plan.empty_bar(dev)
    V = None if fused else plan.empty_bar(dev)
    res = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev)
    g = torch.empty(plan.N, dtype=plan.dtype, device=dev)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    nb = s.r * plan.Npad
    _check(_lib.load().fwi_gradient_rf(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), spp,
        _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d_obs, plan.dtype, s.nt * s.nrec, "d_obs"), int(seed),
        _dev(Q, plan.dtype, s.nt * s.r, "Q"), _dev(U, plan.dtype, nb, "Ubar"),
        _dev(V, plan.dtype, nb, "Vbar"), _dev(res, plan.dtype, s.nt * s.nrec, "resid"),
        _dev(g, plan.dtype, plan.N, "grad"), _dev(J, torch.float64, 1, "misfit"),
        ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev)), "fwi_gradient_rf")
    return {"grad": g, "misfit": J, "Q": Q, "Ubar": U, "Vbar": V, "resid": res}


def set_exact_fused(on: bool) -> None:
    _lib.load().rtm_set_exact_fused(1 if on else 0)


def set_tti_blocks(forward: int, transpose: int) -> None:
    """z-split targets (workgroups per launch) of the tiled TTI forward and
    transpose steps (<= 0: the default)."""
    _lib.load().rtm_set_tti_blocks(int(forward), int(transpose))


def set_tti_shape(shape: int) -> None:
    _lib.load().rtm_set_tti_shape(int(shape))


def exact_workspace_bytes(plan: Plan, checkpoint_every: int = 0) -> int:
    n = ctypes.c_size_t()
    _check(_lib.load().rtm_exact_workspace_bytes(plan.handle, int(checkpoint_every),
                                                 ctypes.byref(n)), "rtm_exact_workspace_bytes")
    return int(n.value)


def rtm_bar_to_rows(plan: Plan, bar) -> torch.Tensor:
    """Tile-major compressed field -> [r][N] rows (a copy, made on the GPU)."""
    s = plan.spec
    rows = torch.empty((s.r, plan.N), dtype=plan.dtype, device=bar.device)
    _check(_lib.load().rtm_bar_to_rows(plan.handle, _dev(bar, plan.dtype, s.r * plan.Npad, "bar"),
                                       _dev(rows, plan.dtype, s.r * plan.N, "rows"),
                                       _stream(bar.device)), "rtm_bar_to_rows")
    return rows


def bar_index(plan: Plan, cells, rows=None) -> np.ndarray:
    """Flat positions in a tile-major compressed field of (row i, cell x) for
    the given cells (all rows, or the given rows): [len(rows)][len(cells)]."""
    x = np.asarray(cells, dtype=np.int64)
    i = np.arange(plan.spec.r, dtype=np.int64) if rows is None else np.asarray(rows, np.int64)
    return ((x[None, :] // 32) * plan.spec.r + i[:, None]) * 32 + x[None, :] % 32


def device_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Streaming copy src -> dst (same byte size, a multiple of 16) with the
    library's 16-byte-vector copy kernel: the HBM reference of the roofline."""
    nb = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda) or dst.numel() * dst.element_size() != nb:
        raise ValueError("device_copy needs two device tensors of the same byte size")
    _check(_lib.load().rtm_device_copy(ctypes.c_void_p(src.data_ptr()),
                                       ctypes.c_void_p(dst.data_ptr()), nb, _stream(src.device)),
           "rtm_device_copy")


def rtm_dot(plan: Plan, a, b, work=None) -> torch.Tensor:
    n = a.numel()
    out = torch.empty(1, dtype=torch.float64, device=a.device)
    work = _work(plan, work, a.device)
    _check(_lib.load().rtm_dot(plan.handle, _dev(a, plan.dtype, n, "a"),
                               _dev(b, plan.dtype, n, "b"), n, _dev(out, torch.float64, 1, "out"),
                               ctypes.c_void_p(work.data_ptr()), work.numel(),
                               _stream(a.device)), "rtm_dot")
    return out


# ---------------------------------------------------------------------------
# pseudo-acoustic TTI
# ---------------------------------------------------------------------------
def tti_workspace(plan: Plan, device="cuda") -> torch.Tensor:
    n = ctypes.c_size_t()
    _check(_lib.load().rtm_tti_workspace_bytes(plan.handle, ctypes.byref(n)),
           "rtm_tti_workspace_bytes")
    return torch.empty(int(n.value), dtype=torch.uint8, device=device)


def _bars2(plan: Plan, dev):
    return torch.empty((2, plan.Npad // 32, plan.spec.r, 32), dtype=plan.dtype, device=dev)


def rtm_tti_forward_probe(plan: Plan, m, aniso, src_pos, q, rec_pos=None, Z=None,
                          want_d: bool = True, work=None) -> dict:
    """aniso: [4][N] (eps, delta, theta, phi).  Ubar: [2][...] (p then q)."""
    s = plan.spec
    dev = m.device
    d = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev) if want_d else None
    U = _bars2(plan, dev) if Z is not None else None
    work = work if work is not None else tti_workspace(plan, dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos") if want_d else (None, None)
    zp, zt = _z(plan, Z)
    _check(_lib.load().rtm_tti_forward_probe(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), _dev(aniso, plan.dtype, 4 * plan.N, "aniso"),
        spp, _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d, plan.dtype, s.nt * s.nrec, "d"), zp, zt,
        _dev(U, plan.dtype, 2 * s.r * plan.Npad, "Ubar"), ctypes.c_void_p(work.data_ptr()),
        work.numel(), _stream(dev)), "rtm_tti_forward_probe")
    out = {}
    if d is not None:
        out["d"] = d
    if U is not None:
        out["Ubar"] = U
    return out


def rtm_tti_adjoint_probe(plan: Plan, m, aniso, rec_pos, res, Z=None, src_pos=None,
                          want_qadj=False, work=None) -> dict:
    s = plan.spec
    dev = m.device
    V = _bars2(plan, dev) if Z is not None else None
    qa = torch.empty((s.nt, s.nsrc), dtype=plan.dtype, device=dev) if want_qadj else None
    work = work if work is not None else tti_workspace(plan, dev)
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    sp, spp = _pos(src_pos, s.nsrc, "src_pos") if want_qadj else (None, None)
    zp, zt = _z(plan, Z)
    _check(_lib.load().rtm_tti_adjoint_probe(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), _dev(aniso, plan.dtype, 4 * plan.N, "aniso"),
        rpp, _dev(res, plan.dtype, s.nt * s.nrec, "res"), spp,
        _dev(qa, plan.dtype, s.nt * s.nsrc, "qadj"), zp, zt,
        _dev(V, plan.dtype, 2 * s.r * plan.Npad, "Vbar"), ctypes.c_void_p(work.data_ptr()),
        work.numel(), _stream(dev)), "rtm_tti_adjoint_probe")
    out = {}
    if V is not None:
        out["Vbar"] = V
    if qa is not None:
        out["qadj"] = qa
    return out


def tti_spectral_radius(plan: Plan, m, aniso, iters: int = 200, seed: int = 1,
                        work=None) -> float:
    """Power-iteration estimate of the spectral radius of m^{-1} A (TTI
    operator, no sponge); the leapfrog is stable for dt <= 2 / sqrt(rho)."""
    dev = m.device
    work = work if work is not None else tti_workspace(plan, dev)
    rho = ctypes.c_double()
    _check(_lib.load().rtm_tti_spectral_radius(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), _dev(aniso, plan.dtype, 4 * plan.N, "aniso"),
        int(iters), int(seed), ctypes.byref(rho), ctypes.c_void_p(work.data_ptr()), work.numel(),
        _stream(dev)), "rtm_tti_spectral_radius")
    return float(rho.value)


def fwi_gradient_tti(plan: Plan, m, aniso, src_pos, q, rec_pos, d_obs, Z, fused: bool = False,
                     work=None) -> dict:
    s = plan.spec
    dev = m.device
    U = _bars2(plan, dev)
    V = None if fused else _bars2(plan, dev)
    res = torch.empty((s.nt, s.nrec), dtype=plan.dtype, device=dev)
    g = torch.empty(plan.N, dtype=plan.dtype, device=dev)
    J = torch.empty(1, dtype=torch.float64, device=dev)
    work = work if work is not None else tti_workspace(plan, dev)
    sp, spp = _pos(src_pos, s.nsrc, "src_pos")
    rp, rpp = _pos(rec_pos, s.nrec, "rec_pos")
    zp, zt = _z(plan, Z)
    _check(_lib.load().fwi_gradient_tti(
        plan.handle, _dev(m, plan.dtype, plan.N, "m"), _dev(aniso, plan.dtype, 4 * plan.N, "aniso"),
        spp, _dev(q, plan.dtype, s.nt * s.nsrc, "q"), rpp,
        _dev(d_obs, plan.dtype, s.nt * s.nrec, "d_obs"), zp, zt,
        _dev(U, plan.dtype, 2 * s.r * plan.Npad, "Ubar"),
        _dev(V, plan.dtype, 2 * s.r * plan.Npad, "Vbar"), _dev(res, plan.dtype, s.nt * s.nrec, "resid"),
        _dev(g, plan.dtype, plan.N, "grad"), _dev(J, torch.float64, 1, "misfit"),
        ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(dev)), "fwi_gradient_tti")
    return {"grad": g, "misfit": J, "Ubar": U, "Vbar": V, "resid": res}
