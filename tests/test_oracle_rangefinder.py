"""Pins of the oracle's range-finder probes (Section "Randomized trace
estimation": probing vectors from a partial QR of A Z with Z Rademacher).

The sketch matrix comes from Philox4x64-10 (Salmon, Moraes, Dror, Shaw 2011),
pinned here against numpy's independent implementation through a transcription
of the published round function.  The sketch Y = H Omega is pinned through a
second route to the history (receivers at every cell and an explicit second
time difference); the range finder through orthonormality and range capture;
the probed gradient through two cases where the projector must reproduce the
exact gradient: r = nt, and a history whose rank (at most N cells) is <= r."""
import numpy as np
import pytest

import oracle
import synth
from oracle import Grid

_M0, _M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
_W0, _W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def _philox4x64(ctr, key, rounds=10):
    """Philox4x64-R: each round multiplies words 0 and 2 by M0, M1, swaps the
    high halves across with the key xored in; the key advances by the Weyl
    constants between rounds."""
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for rd in range(rounds):
        if rd:
            k0, k1 = (k0 + _W0) & _MASK, (k1 + _W1) & _MASK
        p0, p1 = _M0 * x0, _M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0), p1 & _MASK, ((p0 >> 64) ^ x3 ^ k1), p0 & _MASK
    return [x0, x1, x2, x3]


def test_philox_blocks_match_numpy_and_published_rounds():
    for seed in (0, 7, 123456789):
        bg = np.random.Philox(counter=[0, 0, 0, 0], key=[seed, 0])
        w = bg.random_raw(4 * 6).reshape(6, 4)
        for x in range(6):
            assert [int(v) for v in w[x]] == _philox4x64([x + 1, 0, 0, 0], [seed, 0])


@pytest.mark.parametrize("r", [1, 37, 64, 200, 256])
def test_sketch_signs_are_the_published_bits(r):
    N, seed = 50, 99
    om = oracle.sketch_signs(N, r, seed)
    assert om.shape == (N, r) and set(np.unique(om)) <= {-1.0, 1.0}
    for x in (0, 1, 17, 49):
        w = _philox4x64([x + 1, 0, 0, 0], [seed, 0])
        want = [1.0 - 2.0 * ((w[i // 64] >> (i % 64)) & 1) for i in range(r)]
        assert list(om[x]) == want
    if r == 256:   # balanced signs overall
        assert abs(om.mean()) < 0.02


def _all_cells(g):
    nz, ny, nx = g.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([z.ravel(), y.ravel(), x.ravel()], axis=1).astype(np.float64)


def test_sketch_equals_sampled_second_difference():
    """Y from the stored u_tt history equals Y from receivers at every cell
    (d[n] = u^{n+1}) and an explicit second difference with u^0 = u^-1 = 0."""
    wl = synth.workload_small_2d(shape=(14, 17), nt=45, r=8)
    g = Grid.of(wl)
    r, seed = 12, 3
    Y = oracle.sketch(g, wl.m, wl.src_pos, wl.q, seed, r)
    d = oracle.forward(g, wl.m, wl.src_pos, wl.q, _all_cells(g))["d"]   # [nt][N] = u^{n+1}
    u = np.vstack([np.zeros((2, g.N)), d])                               # u^-1, u^0, u^1 ...
    utt = (u[2:] - 2.0 * u[1:-1] + u[:-2]) / g.dt ** 2
    Y2 = utt @ oracle.sketch_signs(g.N, r, seed)
    assert np.abs(Y - Y2).max() <= 1e-11 * np.abs(Y2).max()


def test_range_finder_is_orthonormal_and_captures_the_range():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((90, 13)) @ np.diag(10.0 ** -np.arange(13) * 0.5)
    Q = oracle.range_finder(Y)
    assert np.abs(Q.T @ Q - np.eye(13)).max() < 1e-13
    assert np.abs(Q @ (Q.T @ Y) - Y).max() < 1e-13 * np.abs(Y).max()


def test_rf_gradient_exact_with_r_equal_nt():
    wl = synth.workload_small_2d(shape=(16, 18), nt=32, r=8)
    g = Grid.of(wl)
    d_obs = oracle.forward(g, wl.m * 1.02, wl.src_pos, wl.q, wl.rec_pos)["d"]
    J, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    Jr, gr, Q, _ = oracle.rf_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, 11, g.nt)
    assert abs(Jr - J) <= 1e-13 * J
    assert np.linalg.norm(gr - ge) <= 1e-11 * np.linalg.norm(ge)


def test_rf_gradient_exact_when_history_rank_is_at_most_r():
    """N = 6 x 5 = 30 cells <= r = 30 < nt = 80: H [nt][N] has rank <= 30, the
    sketch spans its column space, and the projector leaves every u_tt time
    series unchanged, so the probed gradient is the exact one although r < nt."""
    wl = synth.workload_small_2d(shape=(6, 5), nt=80, r=8, nb=1)
    wl.src_pos = np.array([[2.0, 0.0, 2.0]])
    wl.rec_pos = np.array([[1.0, 0.0, 1.0], [4.0, 0.0, 3.0]])
    g = Grid.of(wl)
    d_obs = np.zeros((g.nt, 2))
    J, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    _, gr, Q, Y = oracle.rf_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, 5, g.N)
    assert Q.shape == (g.nt, g.N)
    assert np.linalg.norm(gr - ge) <= 1e-9 * np.linalg.norm(ge)
    # with fewer probes than the rank it is no longer exact
    _, g2, _, _ = oracle.rf_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, 5, 10)
    assert np.linalg.norm(g2 - ge) > 1e-6 * np.linalg.norm(ge)


def test_rf_probes_beat_rademacher_at_equal_r():
    wl = synth.workload_small_2d(shape=(30, 34), nt=120, r=8)
    g = Grid.of(wl)
    d_obs = oracle.forward(g, wl.m * 1.03, wl.src_pos, wl.q, wl.rec_pos)["d"]
    _, ge = oracle.exact_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs)
    r = 8
    _, gz, _, _ = oracle.probed_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs,
                                         synth.rademacher(g.nt, r, 21))
    _, gq, _, _ = oracle.rf_gradient(g, wl.m, wl.src_pos, wl.q, wl.rec_pos, d_obs, 21, r)
    ez = np.linalg.norm(gz - ge) / np.linalg.norm(ge)
    eq = np.linalg.norm(gq - ge) / np.linalg.norm(ge)
    assert eq < 0.5 * ez, (eq, ez)
