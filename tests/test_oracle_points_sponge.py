"""Pins of the oracle's point operators and of its absorbing sponge.

Off-grid points (multilinear weights): sampling must return the exact value of
any field that is multilinear in (z, y, x), and a unit injection must spread
weights that are non-negative, sum to one and have the position as their
first moment.  Swapping f and 1 - f on an axis, or a wrong corner, fails both.

Sponge: the damped leapfrog m (u^{n+1} - 2 u^n + u^{n-1}) + a (u^{n+1} -
u^{n-1}) = dt^2 L u^n with a = eta dt / 2 has, once the source is off, the
discrete energy
    E^{n+1/2} = sum m ((u^{n+1} - u^n) / dt)^2 - sum u^{n+1} L u^n
whose change per step is exactly -sum (eta / (2 dt)) (u^{n+1} - u^{n-1})^2
(multiply the recursion by u^{n+1} - u^{n-1}; L is symmetric).  So E is
conserved without a sponge, falls with one, and rises if eta changes sign.  A
receiver near the edge of a sponged grid must also match the same trace on a
grid large enough that no boundary return arrives in the record.  Each check
is run against deliberately broken copies of the oracle (built here from its
source with one sign changed) to show that it catches that mistake.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import Grid

# ---------------------------------------------------------------------------
# multilinear point operators
# ---------------------------------------------------------------------------
def _multilinear(ndim, shape, coef):
    """f = c0 + c1 z + c2 y + c3 x + c4 zy + c5 zx + c6 yx + c7 zyx on the grid
    (y terms dropped in 2D), and the same function at arbitrary points."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")

    def f(z, y, x):
        if ndim == 2:
            y = 0.0 * z
        c = coef
        return (c[0] + c[1] * z + c[2] * y + c[3] * x + c[4] * z * y + c[5] * z * x
                + c[6] * y * x + c[7] * z * y * x)
    return f(z, y, x), f


def _points(ndim, shape, n, rng):
    nz, ny, nx = shape
    p = np.column_stack([rng.uniform(0, nz - 1, n), rng.uniform(0, ny - 1, n),
                         rng.uniform(0, nx - 1, n)])
    # on-grid coordinates on some axes, and the far faces (index n - 1)
    p[0] = [nz - 1, ny - 1, nx - 1]
    p[1] = [0.0, 0.0, 0.0]
    p[2, 0] = 3.0
    p[3, 2] = nx - 1
    p[4, 1] = float(ny - 1)
    if ndim == 2:
        p[:, 1] = 0.0
    return p


@pytest.mark.parametrize("ndim", [2, 3])
def test_sampling_is_exact_on_multilinear_fields(ndim):
    rng = np.random.default_rng(11)
    shape = (9, 7, 11) if ndim == 3 else (9, 1, 11)
    for trial in range(4):
        coef = rng.standard_normal(8)
        field, f = _multilinear(ndim, shape, coef)
        pos = _points(ndim, shape, 64, rng)
        got = oracle.sample_points(ndim, field, pos)
        want = f(pos[:, 0], pos[:, 1], pos[:, 2])
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_injection_weights_sum_to_one_with_the_position_as_first_moment(ndim):
    rng = np.random.default_rng(12)
    shape = (8, 6, 10) if ndim == 3 else (8, 1, 10)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(nx, dtype=float), indexing="ij")
    for p in _points(ndim, shape, 40, rng):
        w = oracle.inject_points(ndim, shape, p[None, :], [1.0])
        assert np.all(w >= 0.0)
        assert np.count_nonzero(w) <= (8 if ndim == 3 else 4)
        # every weight sits on a corner of the cell holding p
        nzidx = np.argwhere(w > 0)
        assert np.all(np.abs(nzidx - p[None, :]) < 1.0)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (w * z).sum() == pytest.approx(p[0], abs=1e-13)
        assert (w * x).sum() == pytest.approx(p[2], abs=1e-13)
        assert (w * z * x).sum() == pytest.approx(p[0] * p[2], abs=1e-12)
        if ndim == 3:
            assert (w * y).sum() == pytest.approx(p[1], abs=1e-13)
            assert (w * z * y * x).sum() == pytest.approx(p[0] * p[1] * p[2], abs=1e-11)


def test_injection_accumulates_and_points_outside_are_refused():
    shape = (5, 1, 6)
    two = oracle.inject_points(2, shape, [[1.5, 0, 2.25], [1.5, 0, 2.25]], [1.0, 2.0])
    one = oracle.inject_points(2, shape, [[1.5, 0, 2.25]], [3.0])
    np.testing.assert_allclose(two, one, rtol=1e-15)
    with pytest.raises(ValueError):
        oracle.inject_points(2, shape, [[4.01, 0, 1.0]], [1.0])
    with pytest.raises(ValueError):
        oracle.sample_points(2, np.zeros(shape), [[1.0, 0, -0.01]])


# ---------------------------------------------------------------------------
# sponge
# ---------------------------------------------------------------------------
N2 = 81           # physical-ish square 2D grid used by the energy checks
H, DT, C = 10.0, 1e-3, 2000.0


def _pulse(nt, n_on, f0=20.0):
    """Ricker source of 20 Hz switched off exactly after n_on steps."""
    t = np.arange(nt) * DT
    a = (np.pi * f0 * (t - 1.0 / f0)) ** 2
    w = (1 - 2 * a) * np.exp(-a)
    w[n_on:] = 0.0
    return (w / H ** 2)[:, None]


def _levels(g, m, src, q):
    """u^0 .. u^nt of the forward sweep (rows)."""
    f = oracle.forward(g, m, src, q, np.zeros((1, 3)), what="u", hist=True, final=True,
                       want_d=False)
    return np.vstack([f["hist"], f["final"][0][None]])


def _energy(g, m, lv):
    """E^{n+1/2} for n = 0..nt-1 and the damping loss predicted per step."""
    nz, ny, nx = g.shape
    eta = (oracle.damping_profile(nz, g.nb, g.h, g.c_ref, g.R)[:, None, None]
           + oracle.damping_profile(nx, g.nb, g.h, g.c_ref, g.R)[None, None, :]).ravel()
    E = np.empty(g.nt)
    for n in range(g.nt):
        Lu = oracle.laplacian(2, lv[n].reshape(g.shape), g.h).ravel()
        E[n] = (m * ((lv[n + 1] - lv[n]) / g.dt) ** 2).sum() - (lv[n + 1] * Lu).sum()
    loss = np.zeros(g.nt)
    for n in range(1, g.nt):
        loss[n] = (eta / (2 * g.dt) * (lv[n + 1] - lv[n - 1]) ** 2).sum()
    return E, loss


def _energy_case(nb, R=1e-3, nt=700, n_on=110):
    g = Grid(2, (N2, 1, N2), H, DT, nt, nb, C, R)
    m = np.full(g.N, 1.0 / C ** 2)
    src = np.array([[N2 // 2, 0, N2 // 2]], float)
    lv = _levels(g, m, src, _pulse(nt, n_on))
    E, loss = _energy(g, m, lv)
    return E, loss, n_on


def _check_energy_balance(E, loss, n_on):
    """E^{n+1/2} - E^{n-1/2} = -loss_n for every step after the source is off."""
    dE = E[n_on + 1:] - E[n_on:-1]
    scale = E[n_on:].max()
    np.testing.assert_allclose(dE, -loss[n_on + 1:], rtol=0, atol=1e-10 * scale)


def test_energy_is_conserved_without_a_sponge():
    E, loss, n_on = _energy_case(nb=0)
    assert np.all(loss == 0.0)
    tail = E[n_on:]
    assert tail.min() > 0.0
    assert (tail.max() - tail.min()) <= 1e-11 * tail.max()


def test_sponge_energy_balance_and_decay():
    E, loss, n_on = _energy_case(nb=10)
    _check_energy_balance(E, loss, n_on)
    tail = E[n_on:]
    assert np.all(np.diff(tail) <= 1e-12 * tail[0])    # never grows once the source is off
    # the wave crosses the 40-cell half-width in 0.2 s; after 0.59 s the
    # sponge has taken out almost all of it
    assert tail[-1] < 2e-2 * tail[0], tail[-1] / tail[0]


def _reflected_energy(nb, R=1e-3, nt=520, interior=61):
    """|trace - free-space trace|^2 / |free-space trace|^2 at a receiver 25
    cells from the source and 5 cells inside the sponge's inner edge, on a grid
    of `interior` cells plus nb sponge cells per face.  The free-space trace
    comes from a grid 90 cells wider on every side, from which no boundary
    return reaches the receiver within nt steps (1.07 s of travel needed)."""
    out = []
    for n, nbb, RR in ((interior + 2 * nb, nb, R), (interior + 180, 10, 1e-3)):
        g = Grid(2, (n, 1, n), H, DT, nt, nbb, C, RR)
        ctr = n // 2
        src = np.array([[ctr, 0, ctr]], float)
        rec = np.array([[ctr, 0, ctr + 25]], float)
        m = np.full(g.N, 1.0 / C ** 2)
        out.append(oracle.forward(g, m, src, _pulse(nt, nt), rec)["d"][:, 0])
    small, free = out
    return float(((small - free) ** 2).sum() / (free ** 2).sum())


def test_sponge_suppresses_boundary_returns():
    """With R = 1e-3 the reflected energy falls as the sponge thickens (10 cells
    is one wavelength of the 20 Hz pulse): below 5 % at 10 cells and 1e-4 at 40
    cells, against more than the direct wave's own energy for a hard
    (Dirichlet) edge, whose returns from all four faces add up."""
    e = {nb: _reflected_energy(nb) for nb in (0, 5, 10, 20, 40)}
    assert e[10] < 0.05, e
    assert e[40] < 1e-4, e
    assert e[0] > 1.0, e
    assert e[0] > e[5] > e[10] > e[20] > e[40], e


def test_a_flipped_eta_fails_the_sponge_checks():
    """eta with the wrong sign (R > 1 turns ln(1/R) negative) must fail both
    the decay check and the reflection bound."""
    E, loss, n_on = _energy_case(nb=10, R=1e3)
    assert not np.all(np.diff(E[n_on:]) <= 1e-12 * E[n_on])
    assert _reflected_energy(nb=10, R=1e3) > 0.05


# ---------------------------------------------------------------------------
# broken copies of the oracle: one sign changed in the damped update
# ---------------------------------------------------------------------------
MUTANTS = {
    "prev-coefficient": ("(m[i] - a) * prev[i]", "(m[i] + a) * prev[i]"),
    "denominator": ("/ (m[i] + a);", "/ (m[i] - a);"),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_energy_balance_catches_a_sign_slip_in_the_damped_update(name, mutant_dir,
                                                                 monkeypatch):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site {old!r} not found exactly once"
    cpath = mutant_dir / f"{name}.c"
    so = mutant_dir / f"{name}.so"
    cpath.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-ffp-contract=off", str(cpath), "-o", str(so), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load(str(so)))
    E, loss, n_on = _energy_case(nb=10, nt=400)
    with pytest.raises(AssertionError):
        _check_energy_balance(E, loss, n_on)
