"""Pins of the FP64 oracle's pseudo-acoustic TTI operator and sweeps.

The paper images a TTI model (Section "2007 BP TTI") but prints no equations;
the coupled p-q system used here is stated in oracle.c.  Its pins: exact
reduction to the acoustic operator when eps = delta = 0, agreement with the
continuous dispersion matrix on a resolved plane wave (rotated symmetry axis),
exact transposition of the operator and of the sweep (dot test), a
second-order Taylor test of the gradient, and exactness of probing with
orthogonal probes."""
import numpy as np
import pytest

import oracle
import synth
from oracle import Grid


def _aniso(shape, seed=0):
    rng = np.random.default_rng(seed)
    eps = 0.3 * rng.random(shape)
    dl = np.minimum(0.15 * rng.random(shape), eps)
    th = np.deg2rad(30) * rng.random(shape)
    ph = 2 * np.pi * rng.random(shape)
    return eps, dl, th, ph


def test_isotropic_limit_is_the_acoustic_laplacian():
    rng = np.random.default_rng(1)
    sh = (12, 11, 13)
    p = rng.standard_normal(sh)
    _, _, th, ph = _aniso(sh)
    op, oq = oracle.tti_apply(0.0, 0.0, th, ph, p, p, 7.0)
    L = oracle.laplacian(3, p, 7.0)
    assert np.abs(op - L).max() <= 1e-13 * np.abs(L).max()
    assert np.abs(oq - L).max() <= 1e-13 * np.abs(L).max()


def test_operator_transpose_is_exact():
    rng = np.random.default_rng(2)
    sh = (13, 12, 14)
    an = _aniso(sh, 3)
    p, q, a, b = (rng.standard_normal(sh) for _ in range(4))
    op, oq = oracle.tti_apply(*an, p, q, 10.0)
    ta, tb = oracle.tti_apply(*an, a, b, 10.0, transpose=True)
    lhs = (op * a).sum() + (oq * b).sum()
    rhs = (p * ta).sum() + (q * tb).sum()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("tilt,azim", [(25.0, 70.0), (0.0, 0.0), (40.0, 200.0)])
def test_plane_wave_matches_continuous_dispersion_matrix(tilt, azim):
    """Homogeneous medium, resolved plane wave u = cos(k.x): the operator acts
    as -[[c1 kh2, c2 ka2], [c2 kh2, ka2]] on (p, q) = (u, al u), with ka the
    wavenumber along the symmetry axis and kh2 = |k|^2 - ka^2 (8th-order
    accurate in the interior)."""
    n, h = 40, 10.0
    z, y, x = np.meshgrid(*(np.arange(n) * h,) * 3, indexing="ij")
    k = np.array([0.013, -0.009, 0.017])          # (z, y, x), kh ~ 0.2
    E, D = 0.25, 0.1
    TH, PH = np.deg2rad(tilt), np.deg2rad(azim)
    u = np.cos(k[0] * z + k[1] * y + k[2] * x)
    axis = np.array([np.cos(TH), np.sin(TH) * np.sin(PH), np.sin(TH) * np.cos(PH)])
    ka2 = (axis @ k) ** 2
    kh2 = k @ k - ka2
    c1, c2, al = 1 + 2 * E, np.sqrt(1 + 2 * D), 0.7
    op, oq = oracle.tti_apply(E, D, TH, PH, u, al * u, h)
    s = (slice(8, -8),) * 3
    ep = -(c1 * kh2 + c2 * ka2 * al) * u
    eq = -(c2 * kh2 + ka2 * al) * u
    assert np.abs(op - ep)[s].max() <= 1e-8 * np.abs(ep[s]).max()
    assert np.abs(oq - eq)[s].max() <= 1e-8 * np.abs(eq[s]).max()
    # the matrix's eigenvalues solve l^2 - l((1+2e)kh2 + ka2) + 2(e - d) kh2 ka2 = 0
    M = np.array([[c1 * kh2, c2 * ka2], [c2 * kh2, ka2]])
    lam = np.linalg.eigvals(M)
    for l in lam:
        assert abs(l * l - l * ((1 + 2 * E) * kh2 + ka2) + 2 * (E - D) * kh2 * ka2) \
            <= 1e-12 * (k @ k) ** 2


def _case(nt=40):
    sh = (14, 12, 16)
    g = Grid(3, sh, 10.0, 1e-3, nt, 3, 3500.0, 1e-3)
    m = np.full(np.prod(sh), 1 / 3000.0 ** 2)
    src = np.array([[6.0, 5.5, 7.25]])
    rec = np.array([[5.0, 4.0, 3.0], [7.0, 8.0, 12.0], [9.0, 6.0, 9.5]])
    return g, m, _aniso(sh, 4), src, rec


def test_sweep_dot_product_test():
    g, m, an, src, rec = _case()
    rng = np.random.default_rng(5)
    qv, yv = rng.standard_normal((g.nt, 1)), rng.standard_normal((g.nt, 3))
    d = oracle.tti_forward(g, m, an, src, qv, rec)["d"]
    qa = oracle.tti_adjoint(g, m, an, rec, yv, src_pos=src)["qadj"]
    a, b = (d * yv).sum(), (qv * qa).sum()
    assert abs(a - b) <= 1e-12 * abs(a)


def test_isotropic_sweep_equals_acoustic_sweep():
    g, m, an, src, rec = _case()
    rng = np.random.default_rng(6)
    qv = rng.standard_normal((g.nt, 1))
    iso = (np.zeros_like(an[0]), np.zeros_like(an[1]), an[2], an[3])
    d_tti = oracle.tti_forward(g, m, iso, src, qv, rec)["d"]
    d_ac = oracle.forward(g, m, src, qv, rec)["d"]
    assert np.abs(d_tti - d_ac).max() <= 1e-12 * np.abs(d_ac).max()


def test_tti_gradient_taylor_second_order():
    g, m, an, src, rec = _case()
    rng = np.random.default_rng(7)
    qv = rng.standard_normal((g.nt, 1))
    d_obs = oracle.tti_forward(g, m * 1.05, an, src, qv, rec)["d"]
    J0, grad = oracle.tti_exact_gradient(g, m, an, src, qv, rec, d_obs)
    dm = rng.standard_normal(m.size) * m * 0.002
    e1 = []
    for eps in (1.0, 0.5, 0.25):
        J1, _ = oracle.misfit(oracle.tti_forward(g, m + eps * dm, an, src, qv, rec)["d"], d_obs)
        e1.append(abs(J1 - J0 - eps * grad @ dm))
    assert 3.6 < e1[0] / e1[1] < 4.4 and 3.6 < e1[1] / e1[2] < 4.4, e1


def test_tti_orthogonal_probes_exact():
    g, m, an, src, rec = _case(nt=32)
    rng = np.random.default_rng(8)
    qv = rng.standard_normal((g.nt, 1))
    d_obs = np.zeros((g.nt, 3))
    H = synth.sylvester_hadamard(g.nt)
    _, gp, _, _ = oracle.tti_probed_gradient(g, m, an, src, qv, rec, d_obs, H)
    _, ge = oracle.tti_exact_gradient(g, m, an, src, qv, rec, d_obs)
    assert np.linalg.norm(gp - ge) <= 1e-12 * np.linalg.norm(ge)


def test_tti_sampled_cells_match_full_probing():
    """Probing a subset of cells in the TTI sweeps gives exactly the matching
    columns of both compressed fields."""
    wl, an = synth.workload_tti(shape=(14, 12, 16), nt=30, r=5, sigma=2.0, nb=3, f0=15.0,
                                rec_stride=5, dtype=np.float64)
    g = Grid.of(wl)
    idx = np.array([0, 7, 100, 1234, g.N - 1])
    full = oracle.tti_forward(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z)["bar"]
    part = oracle.tti_forward(g, wl.m, an, wl.src_pos, wl.q, wl.rec_pos, Z=wl.Z,
                              sample_idx=idx)["bar"]
    np.testing.assert_array_equal(part, full[:, :, idx])
    res = np.random.default_rng(1).standard_normal((g.nt, wl.rec_pos.shape[0]))
    fa = oracle.tti_adjoint(g, wl.m, an, wl.rec_pos, res, Z=wl.Z)["bar"]
    pa = oracle.tti_adjoint(g, wl.m, an, wl.rec_pos, res, Z=wl.Z, sample_idx=idx)["bar"]
    np.testing.assert_array_equal(pa, fa[:, :, idx])


def _tti_matrix(sh, h, m, eps, dl, th, ph):
    """Dense m^{-1} A of the oracle's TTI operator on a tiny grid, column by
    column (A applied to unit vectors of (p, q))."""
    N = int(np.prod(sh))
    M = np.zeros((2 * N, 2 * N))
    for j in range(2 * N):
        e = np.zeros(2 * N)
        e[j] = 1.0
        op, oq = oracle.tti_apply(eps, dl, th, ph, e[:N].reshape(sh), e[N:].reshape(sh), h)
        M[:N, j] = (op / m).ravel()
        M[N:, j] = (oq / m).ravel()
    return M


def test_spectrum_within_the_frozen_coefficient_bound_and_delta_above_eps_grows():
    """The library's TTI screen rests on a frozen-coefficient bound: with
    delta <= eps the coupled operator's symbol at a cell has real
    non-positive eigenvalues of magnitude at most max(1, 1 + 2 eps) / m times
    the acoustic symbol (3 S / h^2 at Nyquist, S = 6.50159).  On a tiny grid
    with cell-wise random m, eps, delta, tilt and azimuth, the dense operator
    m^{-1} A has no eigenvalue with a positive real part (no growing mode)
    and its spectral radius is below that bound; with delta > eps a positive
    real eigenvalue appears (growth for any dt), which is why the screen
    rejects such models."""
    sh, h = (6, 7, 8), 12.5
    rng = np.random.default_rng(9)
    m = 1.0 / (1500.0 + 3000.0 * rng.random(sh)) ** 2
    eps, dl, th, ph = _aniso(sh, 4)
    lam = np.linalg.eigvals(_tti_matrix(sh, h, m, eps, dl, th, ph))
    rho = np.abs(lam).max()
    S = 6.501587301587302
    bound = (np.maximum(1.0, 1.0 + 2.0 * eps) / m).max() * 3.0 * S / h ** 2
    assert lam.real.max() <= 1e-9 * rho
    assert rho <= bound and rho > 0.3 * bound, rho / bound
    dl_bad = eps + 0.3 * np.random.default_rng(5).random(sh)
    lam_bad = np.linalg.eigvals(_tti_matrix(sh, h, m, eps, dl_bad, th, ph))
    assert lam_bad.real.max() > 1e-2 * np.abs(lam_bad).max()
