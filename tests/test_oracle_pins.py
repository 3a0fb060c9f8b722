"""Pins of the FP64 oracle against facts fixed by mathematics or the paper.

None of these re-types the oracle's own formulas: each compares it with an
independent fact (published stencil weights, polynomial exactness, closed-form
Green's functions, transposition identities, finite differences of the misfit,
exactness of Eq. 3 for orthogonal probes, and the moments of the estimator in
Eq. 1).
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.ndimage import gaussian_filter

import oracle
import synth
from oracle import Grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _ricker(t, f0):
    a = (math.pi * f0 * (t - 1.0 / f0)) ** 2
    return (1.0 - 2.0 * a) * math.exp(-a)


# ---------------------------------------------------------------------------
# spatial operator
# ---------------------------------------------------------------------------
def test_laplacian_matches_published_weights():
    """An impulse in the interior reproduces Fornberg's 8th-order weights on
    every axis, with the centre weight counted once per axis."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fornberg_d2_order8.txt"))
            if l.strip() and not l.startswith("#")]
    w = {int(o): int(a) / int(b) for o, a, b in rows}
    h = 3.0
    for ndim, shape in ((2, (15, 1, 17)), (3, (13, 11, 12))):
        u = np.zeros(shape)
        c = tuple(s // 2 for s in shape)
        u[c] = 1.0
        L = oracle.laplacian(ndim, u, h) * h * h
        assert L[c] == pytest.approx(ndim * w[0], rel=1e-14)
        axes = (0, 2) if ndim == 2 else (0, 1, 2)
        for ax in axes:
            for j in range(1, 5):
                for sgn in (1, -1):
                    idx = list(c)
                    idx[ax] += sgn * j
                    assert L[tuple(idx)] == pytest.approx(w[j], rel=1e-14)
        assert np.count_nonzero(L) == 1 + 8 * len(axes)


@pytest.mark.parametrize("ndim", [2, 3])
def test_laplacian_exact_on_degree9_polynomials(ndim):
    """An 8th-order centred second difference is exact for polynomials of
    degree <= 9 on each axis (interior cells, away from the zero padding)."""
    h = 7.0
    if ndim == 3:
        nz, ny, nx = 24, 20, 22
    else:
        nz, ny, nx = 26, 1, 23
    z, y, x = np.meshgrid(np.arange(nz) * h / 50, np.arange(ny) * h / 50,
                          np.arange(nx) * h / 50, indexing="ij")
    if ndim == 3:
        u = x ** 9 + y ** 7 * z ** 2 + z ** 8 - 3 * x * y * z
        ex = (72 * x ** 7 + 42 * y ** 5 * z ** 2 + 2 * y ** 7 + 56 * z ** 6) / 2500.0
    else:
        u = x ** 9 + z ** 8 * x ** 3 + 5 * z * x
        ex = (72 * x ** 7 + 6 * z ** 8 * x + 56 * z ** 6 * x ** 3) / 2500.0
    L = oracle.laplacian(ndim, u, h)
    s = (slice(4, -4), slice(4, -4) if ndim == 3 else slice(None), slice(4, -4))
    assert np.abs(L[s] - ex[s]).max() <= 1e-12 * np.abs(ex[s]).max()


@pytest.mark.parametrize("ndim", [2, 3])
def test_laplacian_symmetric_with_zero_exterior(ndim):
    """Zero values outside the grid make L a symmetric matrix: <Lu,v> = <u,Lv>
    for arbitrary fields, boundary cells included."""
    rng = np.random.default_rng(3)
    shape = (9, 1, 11) if ndim == 2 else (7, 8, 9)
    u, v = rng.standard_normal(shape), rng.standard_normal(shape)
    a = (oracle.laplacian(ndim, u, 2.0) * v).sum()
    b = (u * oracle.laplacian(ndim, v, 2.0)).sum()
    assert abs(a - b) <= 1e-13 * abs(a)


def test_stencil_symbol_bounds_cfl():
    """The Nyquist symbol of the 3D operator (checkerboard eigenvector in the
    interior) is 3 * 6.50159.../h^2, which gives the CFL bound 2/sqrt(19.505)
    = 0.45286 used by the library's plan check."""
    n = 24
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    u = (-1.0) ** (x + y + z)
    L = oracle.laplacian(3, u, 1.0)
    s = (slice(4, -4),) * 3
    lam = -(L[s] / u[s])
    assert np.allclose(lam, lam.flat[0], rtol=1e-13)
    assert lam.flat[0] / 3 == pytest.approx(6.501587301587302, rel=1e-12)
    assert 2.0 / math.sqrt(lam.flat[0]) == pytest.approx(0.452856, abs=1e-6)


# ---------------------------------------------------------------------------
# damping
# ---------------------------------------------------------------------------
def test_damping_profile_closed_form():
    n, nb, h, c, R = 30, 6, 12.5, 3000.0, 1e-3
    eta = oracle.damping_profile(n, nb, h, c, R)
    top = 3.0 * math.log(1.0 / R) / (2.0 * nb * h * c)
    assert eta[0] == pytest.approx(top, rel=1e-14)
    assert eta[-1] == pytest.approx(top, rel=1e-14)
    assert np.all(eta[nb:n - nb] == 0.0)
    # quadratic in the normalised depth d = (nb - i)/nb
    for i in range(nb):
        assert eta[i] == pytest.approx(top * ((nb - i) / nb) ** 2, rel=1e-13)
        assert eta[n - 1 - i] == pytest.approx(eta[i], rel=1e-14)


# ---------------------------------------------------------------------------
# propagation against closed-form Green's functions
# ---------------------------------------------------------------------------
def test_green_function_3d():
    """Homogeneous 3D medium: u(r,t) = w(t - r/c) / (4 pi r) for a point
    source of signature w (injected as w/h^3).  Traces end before any
    boundary return reaches the receivers."""
    n, h, dt, nt, f0, c = 72, 10.0, 1e-3, 260, 8.0, 2000.0
    g = Grid(3, (n, n, n), h, dt, nt, 10, c, 1e-3)
    ctr = n // 2
    offs = [8, 10, 12]
    src = np.array([[ctr, ctr, ctr]], float)
    rec = np.array([[ctr, ctr, ctr + o] for o in offs], float)
    d = oracle.forward(g, np.full(g.N, 1.0 / c ** 2), src,
                       synth.source_signature(nt, dt, f0, h, 3), rec)["d"]
    t = (np.arange(nt) + 1) * dt          # d[n] samples u^{n+1}, i.e. t = (n+1) dt
    for j, o in enumerate(offs):
        r = o * h
        ex = np.array([_ricker(tt - r / c, f0) for tt in t]) / (4 * math.pi * r)
        err = np.linalg.norm(d[:, j] - ex) / np.linalg.norm(ex)
        assert err < 3e-3, (o, err)


def _green2d(r, c, f0, t):
    if c * t <= r:
        return 0.0
    v, _ = quad(lambda th: _ricker(t - (r / c) * math.cosh(th), f0), 0.0,
                math.acosh(c * t / r), limit=400)
    return v / (2 * math.pi)


def _trace2d(dt, nt, off=15, n=161, h=10.0, f0=8.0, c=2000.0):
    g = Grid(2, (n, 1, n), h, dt, nt, 10, c, 1e-3)
    ctr = n // 2
    d = oracle.forward(g, np.full(g.N, 1.0 / c ** 2), np.array([[ctr, 0, ctr]], float),
                       synth.source_signature(nt, dt, f0, h, 2),
                       np.array([[ctr, 0, ctr + off]], float))["d"][:, 0]
    t = (np.arange(nt) + 1) * dt
    ex = np.array([_green2d(off * h, c, f0, tt) for tt in t])
    return np.linalg.norm(d - ex) / np.linalg.norm(ex)


def test_green_function_2d_and_second_order_in_time():
    """2D: u = (1/2pi) int_0^{acosh(ct/r)} w(t - r cosh(th)/c) d th.  With the
    spatial error negligible (8th order, > 20 cells per wavelength) the error
    falls by ~4 when dt is halved (2nd-order time stepping)."""
    e1 = _trace2d(1e-3, 300)
    e2 = _trace2d(5e-4, 600)
    assert e1 < 2e-3
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["2d", "3d", "offgrid"])
def test_dot_product_test(which):
    """<F q, y> = <q, F^T y> for the map q -> d, where F^T samples the adjoint
    wavefield at the source (positions on and off the grid)."""
    rng = np.random.default_rng(7)
    if which == "3d":
        wl = synth.workload_small_3d(shape=(20, 18, 22), nt=60, dtype=np.float64)
    else:
        wl = synth.workload_small_2d(shape=(30, 34), nt=120)
    src, rec = wl.src_pos.copy(), wl.rec_pos.copy()
    if which == "offgrid":
        src = np.array([[10.3, 0.0, 15.6], [12.0, 0.0, 7.25]])
        rec = rec + np.array([0.4, 0.0, 0.35])
    g = Grid.of(wl)
    q = rng.standard_normal((g.nt, src.shape[0]))
    y = rng.standard_normal((g.nt, rec.shape[0]))
    d = oracle.forward(g, wl.m, src, q, rec)["d"]
    qa = oracle.adjoint(g, wl.m, rec, y, src_pos=src)["qadj"]
    a, b = (d * y).sum(), (q * qa).sum()
    assert abs(a - b) <= 1e-12 * abs(a)


def test_adjoint_is_explicit_transpose():
    """Column by column, the matrix of the adjoint recursion equals the
    transpose of the matrix of the forward recursion (tiny grid)."""
    wl = synth.workload_small_2d(shape=(12, 13), nt=14, nb=3)
    g = Grid.of(wl)
    src = np.array([[4.0, 0.0, 5.0], [6.5, 0.0, 8.25]])
    rec = np.array([[3.0, 0.0, 2.0], [4.0, 0.0, 9.5], [8.0, 0.0, 6.0]])
    ns, nr = 2, 3
    F = np.zeros((g.nt * nr, g.nt * ns))
    for k in range(g.nt * ns):
        e = np.zeros(g.nt * ns)
        e[k] = 1.0
        F[:, k] = oracle.forward(g, wl.m, src, e.reshape(g.nt, ns), rec)["d"].ravel()
    Ft = np.zeros((g.nt * ns, g.nt * nr))
    for k in range(g.nt * nr):
        e = np.zeros(g.nt * nr)
        e[k] = 1.0
        Ft[:, k] = oracle.adjoint(g, wl.m, rec, e.reshape(g.nt, nr), src_pos=src)["qadj"].ravel()
    assert np.abs(F).max() > 0
    assert np.abs(F.T - Ft).max() <= 1e-14 * np.abs(F).max()


# ---------------------------------------------------------------------------
# gradient (Eq. 2)
# ---------------------------------------------------------------------------
def _fwi_case():
    wl = synth.workload_small_2d(shape=(40, 44), nt=250)
    g = Grid.of(wl)
    m_true = wl.m
    m0 = gaussian_filter(m_true.reshape(40, 44), 3, mode="nearest").ravel()
    d_obs = oracle.forward(g, m_true, wl.src_pos, wl.q, wl.rec_pos)["d"]
    return wl, g, m0, d_obs


def test_taylor_second_order():
    """|J(m + e dm) - J(m) - e <g, dm>| = O(e^2) for the exact gradient
    -sum_n (d2u/dt2)^n lam^n of the discrete misfit."""
    wl, g, m0, d_obs = _fwi_case()
    J0, grad = oracle.exact_gradient(g, m0, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    dm = np.random.default_rng(1).standard_normal(m0.size) * m0 * 0.002
    e0, e1 = [], []
    for eps in (1.0, 0.5, 0.25, 0.125):
        J1, _ = oracle.misfit(oracle.forward(g, m0 + eps * dm, wl.src_pos, wl.q,
                                             wl.rec_pos)["d"], d_obs)
        e0.append(abs(J1 - J0))
        e1.append(abs(J1 - J0 - eps * grad @ dm))
    r1 = [e1[i] / e1[i + 1] for i in range(3)]
    assert all(3.6 < x < 4.4 for x in r1), r1
    assert e1[-1] < 0.5 * e0[-1]      # the first-order term is captured


def test_gradient_matches_central_differences_per_cell():
    """Every cell of a 10 x 11 grid: central difference of J vs the exact
    gradient (FP64, step 1e-4 m, truncation O(step^2))."""
    wl = synth.workload_small_2d(shape=(10, 11), nt=90, nb=2)
    g = Grid.of(wl)
    m_true = wl.m
    m0 = m_true * (1.0 + 0.02 * np.random.default_rng(2).standard_normal(m_true.size))
    src = np.array([[2.0, 0.0, 5.0]])
    rec = np.array([[2.0, 0.0, float(i)] for i in range(1, 10, 2)])
    d_obs = oracle.forward(g, m_true, src, wl.q, rec)["d"]
    _, grad = oracle.exact_gradient(g, m0, src, wl.q, rec, d_obs)
    fd = np.zeros_like(grad)
    for i in range(m0.size):
        step = 1e-4 * m0[i]
        mp, mm = m0.copy(), m0.copy()
        mp[i] += step
        mm[i] -= step
        Jp, _ = oracle.misfit(oracle.forward(g, mp, src, wl.q, rec)["d"], d_obs)
        Jm, _ = oracle.misfit(oracle.forward(g, mm, src, wl.q, rec)["d"], d_obs)
        fd[i] = (Jp - Jm) / (2 * step)
    assert np.linalg.norm(fd - grad) <= 1e-6 * np.linalg.norm(grad)


# ---------------------------------------------------------------------------
# probing (Eq. 1 and Eq. 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nt", [64, 128])
def test_orthogonal_probes_with_r_equal_nt_are_exact(nt):
    """With Z Z^T = r I (Sylvester Hadamard, r = nt) the probed imaging
    condition of Eq. 3 equals the full-history one of Eq. 2 to round-off.  A
    misaligned probe row (off by one step, or not reversed in the adjoint)
    breaks this."""
    wl = synth.workload_small_2d(shape=(30, 32), nt=nt)
    g = Grid.of(wl)
    d_obs = np.zeros((nt, wl.rec_pos.shape[0]))
    Z = synth.sylvester_hadamard(nt)
    _, gp, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, Z)
    _, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    assert np.linalg.norm(gp - ge) <= 1e-12 * np.linalg.norm(ge)


@pytest.mark.parametrize("what", ["u", "utt"])
def test_identity_probes_recover_history(what):
    """Z = I (r = nt) makes Ubar row n the probed field of step n: the second
    time difference of three stored levels, or the current level u^n."""
    wl = synth.workload_small_2d(shape=(20, 22), nt=40)
    g = Grid.of(wl)
    Z = np.eye(g.nt)
    f = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=Z, what=what)
    full = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, what=what, hist=True)
    np.testing.assert_array_equal(f["Ubar"], full["hist"])
    # levels: u^0 = 0; rebuild the wavefield level by level from d's final state
    lv = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, what="u", hist=True)["hist"]
    assert np.all(lv[0] == 0.0)
    if what == "utt":
        fin = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, final=True)["final"]
        levels = np.vstack([np.zeros((1, g.N)), lv[1:], fin[0][None]])  # u^0..u^nt
        prev = np.vstack([np.zeros((1, g.N)), levels[:-1]])                # u^-1..u^nt-1
        dd = (levels[1:] - 2 * levels[:-1] + prev[:-1]) / g.dt ** 2
        np.testing.assert_allclose(full["hist"], dd, rtol=0, atol=1e-12 * np.abs(dd).max())


def test_probed_estimator_unbiased_with_predicted_variance():
    """Eq. 1 with Rademacher probes: over many seeds the probed image's mean
    tends to the exact zero-lag image and its per-cell variance matches the
    closed form (|a|^2|b|^2 + (a.b)^2 - 2 sum a_t^2 b_t^2) / r, with a, b the
    forward and adjoint time series at the cell."""
    wl = synth.workload_small_2d(shape=(16, 18), nt=60, nb=3)
    g = Grid.of(wl)
    d_obs = np.zeros((g.nt, wl.rec_pos.shape[0]))
    f = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, what="utt", hist=True)
    _, res = oracle.misfit(f["d"], d_obs)
    a = oracle.adjoint(g, wl.m, wl.rec_pos, res, lam_hist=True)
    A, B = f["hist"], a["hist"]                     # [nt][N]
    exact = (A * B).sum(0)
    r, S = 4, 800
    imgs = np.empty((S, g.N))
    for s in range(S):
        Z = synth.rademacher(g.nt, r, 1000 + s)
        fz = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=Z, what="utt",
                            want_d=False)
        az = oracle.adjoint(g, wl.m, wl.rec_pos, res, Z=Z)
        imgs[s] = oracle.image(fz["Ubar"], az["Vbar"], 1.0 / r)
    var = ((A * A).sum(0) * (B * B).sum(0) + exact ** 2 - 2 * (A * A * B * B).sum(0)) / r
    keep = var > 1e-6 * var.max()
    z = (imgs.mean(0) - exact)[keep] / np.sqrt(var[keep] / S)
    # every cell shares the same probe draws, so the z-scores are correlated
    # across cells: check each cell, not their spread
    assert np.abs(z).max() < 4.5, np.abs(z).max()
    ratio = imgs.var(0, ddof=1)[keep] / var[keep]
    assert 0.85 < np.median(ratio) < 1.15, np.median(ratio)
    # a dropped cross term or a wrong 1/r would move the ratio by >= 2x
    assert np.percentile(ratio, 5) > 0.7 and np.percentile(ratio, 95) < 1.3


def test_sampled_cells_match_full_probing():
    """Probing a subset of cells gives exactly the matching columns."""
    wl = synth.workload_small_3d(shape=(14, 12, 16), nt=30, r=5, dtype=np.float64)
    g = Grid.of(wl)
    idx = np.array([0, 7, 100, 1234, g.N - 1])
    full = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z)["Ubar"]
    part = oracle.forward(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z, sample_idx=idx)["Ubar"]
    np.testing.assert_array_equal(part, full[:, idx])


def test_rejects_points_outside_grid():
    wl = synth.workload_small_2d(shape=(12, 13), nt=5, nb=2)
    with pytest.raises(ValueError):
        oracle.forward(Grid.of(wl), wl.m, np.array([[12.5, 0, 3.0]]), wl.q, wl.rec_pos)


def test_table1_fixture_is_consistent():
    """Table 1: the compressed memory is linear in r (r = 64 is twice r = 32)
    and each printed gain is standard / compressed, truncated."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_memory.txt"))
            if l.strip() and not l.startswith("#")]
    for name, full, sub, te64, te32, ghi, glo in rows:
        full, sub, te64, te32 = map(float, (full, sub, te64, te32))
        assert te64 / te32 == pytest.approx(2.0, rel=1e-12)
        assert int(full / te64) == int(ghi)
        assert int(sub / te32) == int(glo)
