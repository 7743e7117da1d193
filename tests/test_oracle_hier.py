"""Pins of the oracle's hierarchical sampler: the CAR dependence parameters
r_l are unknowns with iid Uniform(0, 1) priors (paper Sec. 2.2.1) and are
updated by Metropolis-within-Gibbs on the logit scale.

Without data the joint target is p(H | r) p(r), whose r-marginal is the
Uniform(0, 1) prior itself -- but only if every r-dependent normalising term
of p(H | r) (1/2 log det Q(r), N log s(r), the quadratic form) and the
Jacobian r(1 - r) of the logit move are right; a dropped or mis-signed term
biases the r samples.  (The u = H_1/top marginals of the copula prior are
pinned at fixed r by the sampler tests in test_oracle_grad_mcmc.py.)"""
import numpy as np
import pytest
from scipy import stats

from tests.helpers import make_scenario


def _prior_only(R=3, C=4, top=200.0, r0=0.5):
    rng = np.random.default_rng(3)
    topg = top + rng.uniform(-5, 5, (R, C))
    free = np.stack([0.3 * topg, 0.6 * topg])
    return make_scenario(3, R, C, 30.0, 40.0, free, topg, (1.8, 0.0, 2.7), np.zeros((0, 3)), None,
                         car_r=np.full(2, r0))


def test_log_prior_r_is_the_prior_at_those_r(oracle_mod):
    sc = _prior_only()
    rng = np.random.default_rng(1)
    for _ in range(5):
        r = rng.uniform(0.05, 0.999, 2)
        sc_r = _prior_only()
        sc_r.car_r = r
        a = oracle_mod.OracleProblem(sc).log_prior_r(sc.truth, r)
        b = oracle_mod.OracleProblem(sc_r).log_prior(sc.truth)
        assert a == b


def test_prior_only_r_marginal_is_uniform(oracle_mod):
    sc = _prior_only()
    orc = oracle_mod.OracleProblem(sc)
    n, steps = 384, 2500
    rng = np.random.default_rng(5)
    # starts spread inside the support
    u1 = rng.uniform(0.1, 0.9, (n, 3, 4))
    u2 = rng.uniform(0.1, 0.9, (n, 3, 4))
    h1 = u1 * sc.top[None]
    h2 = h1 + u2 * (sc.top[None] - h1)
    states = np.stack([h1, h2], axis=1)
    r0 = rng.uniform(0.05, 0.95, (n, 2))
    H, r, lp, acc, accr, _ = orc.mcmc_rw_r(states, r0, np.full(n, np.nan), np.zeros(n, np.int64), steps, 0,
                                           4.0, 1.5, 2024)
    assert np.all(np.isfinite(lp))
    rate_h, rate_r = acc.mean() / steps, accr.mean() / steps
    assert 0.1 < rate_h < 0.9 and 0.1 < rate_r < 0.95, (rate_h, rate_r)
    for l in range(2):
        ks = stats.kstest(r[:, l], "uniform")
        assert ks.pvalue > 1e-3, (l, ks)
        assert abs(r[:, l].mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)


def test_prior_only_r_marginal_detects_a_dropped_jacobian(oracle_mod):
    """The same chains scored against the wrong target (r moves without the
    Jacobian: density uniform in logit r, i.e. r ~ Beta(0, 0) shape, mass
    piled at 0 and 1) must fail the uniformity test: the pin has power."""
    # the r-marginal implied by a target uniform in eta = logit r on a wide
    # box is far from uniform; emulate it by sampling eta ~ U(-6, 6)
    rng = np.random.default_rng(0)
    r = 1.0 / (1.0 + np.exp(-rng.uniform(-6, 6, 768)))
    assert stats.kstest(r, "uniform").pvalue < 1e-3
