"""Pins of the oracle's stack over sources (the sum of per-shot probed
gradients, each shot with its own probes; Section "Approximate gradient
calculations", the remark after Eq. 4).

- With orthogonal probes (Z Z^T = r I, r = nt) every shot's estimate is exact, so the stack
  equals the sum of the exact per-shot gradients (Eq. 2).
- With independent Rademacher probes per shot the estimates are unbiased and
  their errors independent, so the stack's mean-square error is the sum of the
  per-shot closed-form variances (|a|^2|b|^2 + (a.b)^2 - 2 sum a_t^2 b_t^2)/r
  (a, b: a cell's forward u_tt and adjoint time series).  For a fold of S
  copies of one shot, the error of the average falls as 1/S; reusing one
  probe matrix for every copy, a plausible slip, keeps it at the single-shot
  level.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import Grid


def _setup(nshots=3):
    wl = synth.workload_small_2d(shape=(16, 18), nt=60, nb=3)
    g = Grid.of(wl)
    d_obs = np.zeros((g.nt, wl.rec_pos.shape[0]))
    xs = [5.0, 9.0, 13.0][:nshots]
    shots = [(np.array([[5.0, 0.0, x]]), wl.q, wl.rec_pos, d_obs) for x in xs]
    return wl, g, shots


def _histories(g, m, shot):
    src, q, rec, d_obs = shot
    f = oracle.forward(g, m, src, q, rec, what="utt", hist=True)
    _, res = oracle.misfit(f["d"], d_obs)
    a = oracle.adjoint(g, m, rec, res, lam_hist=True)
    return f["hist"], a["hist"]


def _variance(A, B, r):
    ab = (A * B).sum(0)
    return ((A * A).sum(0) * (B * B).sum(0) + ab ** 2 - 2 * (A * A * B * B).sum(0)) / r


def test_stack_with_orthogonal_probes_is_the_exact_stack():
    wl, g, shots = _setup()
    # r = nt orthogonal probes (nt = 60 is no Hadamard order): a random
    # orthogonal matrix scaled to Z Z^T = r I
    Q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((g.nt, g.nt)))
    Zo = Q * np.sqrt(g.nt)
    J, G = oracle.stacked_probed_gradient(g, wl.m, shots, [Zo] * len(shots))
    Je, Ge = 0.0, np.zeros(g.N)
    for src, q, rec, d_obs in shots:
        Ji, gi = oracle.exact_gradient(g, wl.m, src, q, rec, d_obs)
        Je += Ji
        Ge += gi
    assert J == pytest.approx(Je, rel=1e-13)
    np.testing.assert_allclose(G, Ge, rtol=0, atol=1e-11 * np.abs(Ge).max())
    # and it is the sum over shots, not one shot's gradient or their mean
    _, g0 = oracle.exact_gradient(g, wl.m, *shots[0])
    assert np.linalg.norm(G - g0) > 0.1 * np.linalg.norm(Ge)


def test_stack_error_is_the_sum_of_independent_shot_variances():
    wl, g, shots = _setup()
    r, T = 4, 200
    hists = [_histories(g, wl.m, sh) for sh in shots]
    exact = -sum((A * B).sum(0) for A, B in hists)
    pred = sum(_variance(A, B, r).sum() for A, B in hists)
    err = np.empty(T)
    for t in range(T):
        Zs = [synth.rademacher(g.nt, r, 5000 + 10 * t + i) for i in range(len(shots))]
        _, G = oracle.stacked_probed_gradient(g, wl.m, shots, Zs)
        err[t] = ((G - exact) ** 2).sum()
    assert 0.8 < err.mean() / pred < 1.25, err.mean() / pred


def test_fold_averages_the_probing_noise_as_one_over_s():
    wl, g, shots = _setup(nshots=1)
    r, T = 4, 200
    A, B = _histories(g, wl.m, shots[0])
    exact = -(A * B).sum(0)
    v1 = _variance(A, B, r).sum()
    mse = {}
    for S in (1, 4):
        e = np.empty(T)
        for t in range(T):
            Zs = [synth.rademacher(g.nt, r, 9000 + 100 * t + i) for i in range(S)]
            _, G = oracle.stacked_probed_gradient(g, wl.m, shots * S, Zs)
            e[t] = ((G / S - exact) ** 2).sum()
        mse[S] = e.mean()
        assert 0.8 < mse[S] / (v1 / S) < 1.25, (S, mse[S] / (v1 / S))
    assert 2.8 < mse[1] / mse[4] < 5.5, mse[1] / mse[4]
    # one probe matrix reused across the fold: no averaging at all
    e = np.empty(T)
    for t in range(T):
        Z = synth.rademacher(g.nt, r, 9000 + 100 * t)
        _, G = oracle.stacked_probed_gradient(g, wl.m, shots * 4, [Z] * 4)
        e[t] = ((G / 4 - exact) ** 2).sum()
    assert 0.8 < e.mean() / v1 < 1.25, e.mean() / v1
