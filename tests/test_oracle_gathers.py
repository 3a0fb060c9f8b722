"""Pins of the oracle's subsurface-offset image volume (Eq. 4): the zero
offset is the image of Eq. 3; with orthogonal probes (Hadamard, r = nt) it is
the full-history offset correlation sum_n u_tt^n[x + h] lam^n[x - h]; swapping
the fields mirrors the offsets; offsets that leave the row give zero."""
import numpy as np

import oracle
import synth
from oracle import Grid


def _case(nt=32):
    wl = synth.workload_small_2d(shape=(16, 18), nt=nt, r=8)
    g = Grid.of(wl)
    rng = np.random.default_rng(1)
    res = rng.standard_normal((nt, wl.rec_pos.shape[0]))
    return wl, g, res


def test_zero_offset_is_the_image():
    wl, g, res = _case()
    f = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z)
    a = oracle.adjoint(g, wl.m, wl.rec_pos, res, Z=wl.Z)
    G = oracle.offset_gathers(f["Ubar"], a["Vbar"], g.shape, 5, 1.0 / wl.r)
    im = oracle.image(f["Ubar"], a["Vbar"], 1.0 / wl.r)
    assert np.array_equal(G[5], im)


def test_orthogonal_probes_give_the_full_history_offset_correlation():
    wl, g, res = _case()
    H = synth.sylvester_hadamard(g.nt)
    f = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=H, hist=True)
    a = oracle.adjoint(g, wl.m, wl.rec_pos, res, Z=H, lam_hist=True)
    nh = 6
    G = oracle.offset_gathers(f["Ubar"], a["Vbar"], g.shape, nh, 1.0 / g.nt)
    nz, ny, nx = g.shape
    u = f["hist"].reshape(g.nt, nz, ny, nx)
    lam = a["hist"].reshape(g.nt, nz, ny, nx)
    for h in (-nh, -2, 0, 3, nh):
        want = np.zeros((nz, ny, nx))
        lo, hi = max(0, -h, h), min(nx, nx - h, nx + h)
        for x in range(lo, hi):
            want[:, :, x] = (u[:, :, :, x + h] * lam[:, :, :, x - h]).sum(axis=0)
        got = G[h + nh].reshape(nz, ny, nx)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), h


def test_swapping_fields_mirrors_offsets_and_edges_are_zero():
    rng = np.random.default_rng(3)
    shape = (3, 2, 11)
    U, V = rng.standard_normal((4, 66)), rng.standard_normal((4, 66))
    nh = 4
    G = oracle.offset_gathers(U, V, shape, nh, 0.25)
    Gs = oracle.offset_gathers(V, U, shape, nh, 0.25)
    assert np.allclose(Gs, G[::-1], rtol=0, atol=1e-15)
    Gr = G.reshape(2 * nh + 1, 3, 2, 11)
    for h in range(1, nh + 1):
        assert np.all(Gr[h + nh, :, :, 11 - h:] == 0) and np.all(Gr[h + nh, :, :, :h] == 0)
