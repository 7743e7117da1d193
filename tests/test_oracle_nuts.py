"""Pins of the oracle's NUTS, its warm-up adaptation and nested R-hat
against what the mathematics and the published schedules fix:

- on Gaussian targets NUTS recovers the means and variances;
- the no-U-turn criterion ends trajectories: on a unit Gaussian with a small
  step the trajectory spans a bounded multiple of the half period pi, far
  below the depth cap (a sign error in the criterion runs to the cap);
- the leapfrog and the momentum draw use the inverse mass consistently: a
  badly scaled Gaussian sampled with inverse mass = its variances behaves
  like the unit Gaussian (same trajectory statistics);
- dual averaging brings the mean acceptance of its window to the target,
  mass adaptation recovers the target's variances, and the warm-up windows are Stan's published ones
  (75 / 25 / 50, doubling: ends at 100, 150, 250, 450, 950 of 1000);
- nested R-hat equals a hand-computed value, is invariant under shifts,
  scalings and permutations within super-chains, and when all super-chains
  sample one distribution nR^2 - 1 is near its expectation 1/n_within;
- on the prior-only cave posterior NUTS recovers the uniform marginals."""
import numpy as np
import pytest
from scipy import stats

from tests.helpers import make_scenario


def test_warmup_windows_are_stans(oracle_mod):
    assert oracle_mod.warmup_window_ends(1000) == [99, 149, 249, 449, 949]
    # too short for the defaults: 15 % / 75 % / 10 %
    assert oracle_mod.warmup_window_ends(100) == [89]
    assert oracle_mod.warmup_window_ends(10) == []


def test_nested_rhat_hand_value_and_invariances(oracle_mod):
    # super-chains {0, 2} and {4, 6}: means 1 and 5, B = 8, W = 2, nR = sqrt(5)
    x = np.array([[0.0], [2.0], [4.0], [6.0]])
    assert oracle_mod.nested_rhat(x, 2, 2)[0] == pytest.approx(np.sqrt(5.0), rel=1e-14)
    rng = np.random.default_rng(1)
    y = rng.standard_normal((6 * 4, 3))
    r = oracle_mod.nested_rhat(y, 6, 4)
    np.testing.assert_allclose(oracle_mod.nested_rhat(3.0 * y - 7.0, 6, 4), r, rtol=1e-12)
    perm = np.concatenate([rng.permutation(4) + 4 * k for k in range(6)])
    np.testing.assert_allclose(oracle_mod.nested_rhat(y[perm], 6, 4), r, rtol=1e-12)
    # every super-chain from one distribution: with one draw per chain the
    # super-chain means vary by sigma^2 / n_within, so nR^2 - 1 is near 1/n_within
    z = rng.standard_normal((64 * 32, 5))
    q = (oracle_mod.nested_rhat(z, 64, 32) ** 2 - 1.0) * 32
    assert np.all((q > 0.5) & (q < 1.6)), q
    # one shifted super-chain is detected
    z[:32] += 3.0
    assert np.all((oracle_mod.nested_rhat(z, 64, 32) ** 2 - 1.0) * 32 > 3.0)


def test_nuts_recovers_gaussian_moments(oracle_mod):
    sd = np.array([0.5, 1.0, 2.0, 1.0, 3.0, 0.7])
    rng = np.random.default_rng(2)
    n = 400
    r = oracle_mod.nuts_gauss(sd, rng.standard_normal((n, 6)) * sd, np.full(n, 0.25), n_steps=30, seed=5)
    x = r["x"]
    assert r["diverged"].sum() == 0
    # final draws of independent chains: means and variances
    assert np.all(np.abs(x.mean(axis=0)) < 4 * sd / np.sqrt(n))
    ratio = x.var(axis=0) / sd ** 2
    assert np.all((ratio > 0.8) & (ratio < 1.25)), ratio
    for i in range(6):
        assert stats.kstest(x[:, i] / sd[i], "norm").pvalue > 1e-3


def test_uturn_ends_trajectories(oracle_mod):
    n, eps = 200, 0.05
    rng = np.random.default_rng(3)
    r = oracle_mod.nuts_gauss(np.ones(1), rng.standard_normal((n, 1)), np.full(n, eps), max_depth=10, n_steps=5,
                              seed=7)
    span = r["n_leap"] * eps
    assert r["depth"].max() < 10
    assert 1.0 < np.median(span) < 8.0, np.median(span)
    # an inverse mass equal to the target's variances makes a badly scaled
    # Gaussian the unit one: identical trajectory lengths for the same draws
    s = np.array([40.0])
    r2 = oracle_mod.nuts_gauss(s, rng.standard_normal((n, 1)) * s, np.full(n, eps), inv_mass=np.full((n, 1), 1600.0),
                               max_depth=10, n_steps=5, seed=7)
    assert abs(np.median(r2["n_leap"]) - np.median(r["n_leap"])) <= 0.25 * np.median(r["n_leap"])


def test_dual_averaging_and_mass_adaptation(oracle_mod):
    sd = np.array([0.1, 0.3, 1.0, 3.0, 10.0, 0.5, 2.0, 5.0])
    n = 8
    rng = np.random.default_rng(4)
    r = oracle_mod.nuts_gauss(sd, rng.standard_normal((n, 8)) * sd, np.full(n, 0.01),
                              inv_mass=np.ones((n, 8)), n_warmup=1000, n_steps=300, seed=11)
    ratio = r["inv_mass"] / sd ** 2
    assert np.all((ratio > 0.6) & (ratio < 1.6)), ratio
    # dual averaging drives the mean acceptance of its own window to the
    # target: (t + t0) H_bar_t = sum (target - accept_s); the last window is
    # the terminal buffer, iterations 950..999
    acc_term = r["accept_stat"][:, 950:1000].mean()
    assert 0.74 < acc_term < 0.86, acc_term
    # sampling runs at the averaged step size, a little shorter than the iterates
    assert 0.75 < r["accept_stat"][:, 1000:].mean() < 0.97
    # step size alone (identity mass): one window over the whole warm-up
    r = oracle_mod.nuts_gauss(np.ones(10), rng.standard_normal((n, 10)), np.full(n, 2.0), n_warmup=400,
                              n_steps=300, seed=12)
    assert 0.74 < r["accept_stat"][:, :400].mean() < 0.86
    assert np.all(r["eps"] > 0.3) and np.all(r["eps"] < 3.0)


def test_nuts_prior_only_cave_marginals_are_uniform(oracle_mod):
    """No sensors: the posterior is the copula prior, whose marginal at every
    node is uniform between the floor and the top (one free surface)."""
    R, C = 3, 4
    top = np.full((R, C), 100.0)
    free = np.full((1, R, C), 50.0)
    sc = make_scenario(2, R, C, 30.0, 40.0, free, top, (1.8, 2.7), np.zeros((0, 3)), None, car_r=[0.5])
    orc = oracle_mod.OracleProblem(sc)
    n = 256
    rng = np.random.default_rng(5)
    x0 = rng.uniform(20.0, 80.0, size=(n, 1, R, C))
    r = orc.nuts(x0, np.full(n, np.nan), np.full(n, 2.0), inv_mass=np.ones((n, 1, R, C)), n_warmup=200,
                 n_steps=100, seed=13)
    u = r["x"].reshape(n, -1) / 100.0
    for i in range(R * C):
        assert stats.kstest(u[:, i], "uniform").pvalue > 1e-3
    assert stats.kstest(u.ravel(), "uniform").pvalue > 1e-4
