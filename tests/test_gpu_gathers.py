"""Subsurface-offset image volume (Eq. 4) on the GPU against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import dev, host, rel, require_gpu, say

pytestmark = pytest.mark.gpu

import paper_2201_06914_amd as P  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _tile_major(rows, Npad):
    """[r][N] rows -> tile-major [Npad / 32][r][32]."""
    r, N = rows.shape
    out = np.zeros((Npad // 32, r, 32), dtype=rows.dtype)
    x = np.arange(N)
    for i in range(r):
        out[x // 32, i, x % 32] = rows[i]
    return out


def _plan(shape, r, field):
    ndim = 2 if shape[1] == 1 else 3
    return P.Plan(P.PlanSpec(ndim, shape, 10.0, 1e-3, 16, 1, 3000.0, 1e-3, 3000.0, field,
                             field, r, 16, 1, 1))


@pytest.mark.parametrize("shape,r,nh,field", [
    ((7, 1, 75), 12, 40, "f64"), ((5, 3, 130), 20, 64, "f64"), ((4, 1, 30), 8, 40, "f64"),
    ((6, 4, 97), 33, 40, "f32"), ((3, 5, 64), 16, 7, "f32"), ((5, 3, 70), 5, 0, "f64"),
    ((3, 3, 40), 3, 1, "f64"), ((4, 3, 66), 17, 33, "f32"), ((3, 1, 200), 9, 63, "f64"),
    ((3, 3, 150), 9, 47, "f32"), ((4, 3, 130), 20, 55, "f32"), ((3, 3, 140), 35, 64, "f32"),
    ((3, 3, 150), 11, 36, "f32"), ((4, 3, 30), 7, 41, "f32"), ((3, 4, 145), 18, 38, "f32"),
    ((3, 3, 300), 6, 40, "f32"), ((4, 3, 20), 3, 5, "f32"), ((3, 3, 129), 4, 0, "f32"),
    ((3, 3, 257), 13, 60, "f32")])
def test_offset_gathers_match_oracle(shape, r, nh, field):
    """Ragged rows (x not a multiple of the segment: 64 cells in FP64, 128 in
    FP32), rows of one to three FP32 segments and rows shorter than the
    offsets or a 32-cell tile; nh 0 .. 64 (FP64: one and two waves per probe
    slice, both V alignments; FP32: 1 .. 9 b tiles, products written out in
    one or two rounds); r below, at and between multiples of the 4-row MFMA
    step and of the probe chunk."""
    plan = _plan(shape, r, field)
    N = int(np.prod(shape))
    rng = np.random.default_rng(sum(shape) + r)
    U, V = rng.standard_normal((r, N)), rng.standard_normal((r, N))
    dt = torch.float64 if field == "f64" else torch.float32
    npdt = np.float64 if field == "f64" else np.float32
    Ut = dev(_tile_major(U.astype(npdt), plan.Npad), dt)
    Vt = dev(_tile_major(V.astype(npdt), plan.Npad), dt)
    G = host(P.rtm_offset_gathers(plan, Ut, Vt, nh))
    torch.cuda.synchronize()
    G0 = oracle.offset_gathers(U.astype(npdt), V.astype(npdt), shape, nh, 1.0 / r)
    e = rel(G, G0)
    say(f"  gathers {shape} r={r} nh={nh} {field}: {e:.2e}")
    assert e < (1e-13 if field == "f64" else 1e-5)


@pytest.mark.parametrize("field,r,nh", [("f64", 16, 10), ("f32", 40, 40), ("f32", 24, 60)])
def test_two_fields_are_summed(field, r, nh):
    shape = (4, 3, 70)
    plan = _plan(shape, r, field)
    N = int(np.prod(shape))
    rng = np.random.default_rng(5)
    npdt, dt = (np.float64, torch.float64) if field == "f64" else (np.float32, torch.float32)
    U = rng.standard_normal((2, r, N)).astype(npdt)
    V = rng.standard_normal((2, r, N)).astype(npdt)
    Ut = dev(np.concatenate([_tile_major(U[f], plan.Npad).ravel() for f in range(2)]), dt)
    Vt = dev(np.concatenate([_tile_major(V[f], plan.Npad).ravel() for f in range(2)]), dt)
    G = host(P.rtm_offset_gathers(plan, Ut, Vt, nh, scale=-0.5, nfield=2))
    torch.cuda.synchronize()
    G0 = sum(oracle.offset_gathers(U[f], V[f], shape, nh, -0.5) for f in range(2))
    e = rel(G, G0)
    say(f"  two fields {field} r={r} nh={nh}: {e:.2e}")
    assert e < (1e-13 if field == "f64" else 1e-5)


def test_zero_offset_equals_image_on_swept_fields():
    """The GPU's own compressed fields (forward u_tt and adjoint probes):
    offset 0 of the volume equals rtm_image in FP64 up to the order in which
    the probe products are summed."""
    wl = synth.workload_small_2d(shape=(30, 34), nt=64, r=16)
    plan = P.Plan.for_workload(wl, field="f64", probe="f64")
    m, q, Z = dev(wl.m, torch.float64), dev(wl.q, torch.float64), dev(wl.Z, torch.int8)
    f = P.rtm_forward_probe(plan, m, wl.src_pos, q, wl.rec_pos, Z=Z)
    res = dev(np.random.default_rng(2).standard_normal((wl.nt, wl.rec_pos.shape[0])),
              torch.float64)
    a = P.rtm_adjoint_probe(plan, m, wl.rec_pos, res, Z=Z)
    G = P.rtm_offset_gathers(plan, f["Ubar"], a["Vbar"], 40)
    im = P.rtm_image(plan, f["Ubar"], a["Vbar"], 1.0 / wl.r)
    torch.cuda.synchronize()
    e = rel(host(G[40]), host(im))
    say(f"  offset 0 vs image: {e:.2e}")
    assert e < 1e-14
