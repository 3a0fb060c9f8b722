"""Full-size parity: the 384 x 512 x 512 layered 3D grid (r = 128 probes,
k = 32, BF16X2 MFMA probing, FP32 fields) through fwi_gradient - the launch
configuration the benchmark times - truncated to nt = 64 steps so the FP64
oracle can follow it.  Traces (the whole 512 x 512 receiver plane) and the
misfit are compared in full; the compressed fields and the gradient on a
sample of cells (near the source, in the sponge, at grid corners, random)."""
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


def test_fullsize_layered_3d_gradient_truncated():
    require_gpu()
    nt = 64
    wl = synth.workload_c2(nt=nt)
    say(f"case: full-size {wl.shape} nt={nt} r={wl.r} k={wl.k_block} bf16x2 fwi_gradient")
    g = Grid.of(wl)
    idx = _sample_cells(wl.shape, wl.src_pos[0])
    d_obs = np.zeros((nt, wl.rec_pos.shape[0]), dtype=np.float32)
    plan = P.Plan.for_workload(wl, field="f32", probe="bf16x2")
    out = P.fwi_gradient(plan, dev(wl.m, torch.float32), wl.src_pos, dev(wl.q, torch.float32),
                         wl.rec_pos, dev(d_obs, torch.float32), dev(wl.Z, torch.int8))
    torch.cuda.synchronize()
    res = host(out["resid"])
    J = float(out["misfit"].item())
    ii = torch.from_numpy(idx).cuda()
    bi = torch.from_numpy(P.bar_index(plan, idx)).cuda()
    U = host(out["Ubar"].reshape(-1)[bi])
    V = host(out["Vbar"].reshape(-1)[bi])
    gr = host(out["grad"][ii])
    del out
    torch.cuda.empty_cache()
    say("  gpu done; oracle forward ...")
    Jo, go, f, a = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, wl.Z,
                                          sample_idx=idx)
    e = dict(d=rel(res, f["d"]), J=abs(J - Jo) / Jo, U=rel(U, f["Ubar"]), V=rel(V, a["Vbar"]),
             g=rel(gr, go))
    say("  " + "  ".join(f"{k} {v:.2e}" for k, v in e.items()))
    assert e["d"] < 1e-5 and e["J"] < 2e-5
    assert e["U"] < 1e-4 and e["V"] < 1e-4 and e["g"] < 1e-3
