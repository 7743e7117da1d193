"""Pins of the latent parametrisation the paper's sampler runs on: the CAR
fields x with H = H(x) through the copula map (Sec. 2.2.1, 3.1).

- the map and its inverse are inverse to each other and keep the surfaces
  ordered under the top;
- change of variables: the latent density minus log|det dH/dx|, with the
  Jacobian taken by central differences of the map over all coordinates (no
  use of its triangular structure), equals the density in H, itself pinned
  by a numerical Jacobian of the generative map;
- the gradient against central differences of the latent log posterior
  (with data);
- NUTS on the latent vector of the prior-only problem gives uniform height
  marginals."""
import numpy as np
import pytest
from scipy import stats

from paper_2603_28907_amd import inputs
from tests.helpers import make_scenario


def prior_problem(oracle_mod, R=3, C=3, S=3, r=0.6, seed=0):
    rng = np.random.default_rng(seed)
    top = 100.0 + 5.0 * rng.random((R, C))
    free = np.stack([np.full((R, C), 30.0 + 20.0 * l) for l in range(S - 1)])
    sc = make_scenario(S, R, C, 30.0, 30.0, free, top, (1.8, 0.0, 2.7, 2.2)[:S], np.zeros((0, 3)), None,
                       car_r=np.full(S - 1, r))
    return sc, oracle_mod.OracleProblem(sc)


def test_map_round_trip_and_order(oracle_mod):
    sc, orc = prior_problem(oracle_mod)
    rng = np.random.default_rng(1)
    # the prior's own scale (sqrt(Sigma11) = 0.53 here): far in the tails the
    # inverse loses precision to H - H_{l-1} cancelling, not to the map
    x = 0.5 * rng.standard_normal((5, 2, 3, 3))
    H = orc.latent_to_heights(x)
    assert np.all(H[:, 0] > 0) and np.all(H[:, 1] > H[:, 0]) and np.all(H[:, 1] < sc.top)
    np.testing.assert_allclose(orc.heights_to_latent(H), x, rtol=1e-9, atol=1e-9)


def test_change_of_variables_matches_the_density_in_h(oracle_mod):
    sc, orc = prior_problem(oracle_mod)
    rng = np.random.default_rng(2)
    M = orc.M
    for _ in range(3):
        x = 0.5 * rng.standard_normal(M)
        h = 1e-6
        J = np.empty((M, M))
        for k in range(M):
            e = np.zeros(M)
            e[k] = h
            J[:, k] = (orc.latent_to_heights(x + e).ravel() - orc.latent_to_heights(x - e).ravel()) / (2 * h)
        sign, logdet = np.linalg.slogdet(J)
        assert sign > 0
        lx = orc.latent_logpost(x)          # no sensors: the prior of x
        lh = orc.log_prior(orc.latent_to_heights(x)[0])
        assert lx - logdet == pytest.approx(lh, abs=1e-6)


def test_latent_gradient_against_central_differences(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    orc = oracle_mod.OracleProblem(sc)
    x = orc.heights_to_latent(inputs.init_states(sc, 1, seed=3))[0]
    lp, g = orc.latent_logpost(x, with_grad=True)
    rng = np.random.default_rng(4)
    checked = 0
    for k in rng.choice(orc.M, size=40, replace=False):
        h = 1e-4
        e = np.zeros(orc.M)
        e[k] = h
        fp, fm = orc.latent_logpost(x.ravel() + e), orc.latent_logpost(x.ravel() - e)
        fd = (fp - fm) / (2 * h)
        one_sided = ((fp - lp) / h, (lp - fm) / h)
        if abs(one_sided[0] - one_sided[1]) > 1e-2 * (abs(fd) + 1.0):   # a kink of the exact march
            continue
        assert g.ravel()[k] == pytest.approx(fd, rel=1e-4, abs=1e-4), k
        checked += 1
    assert checked >= 30


def test_latent_nuts_prior_marginals_are_uniform(oracle_mod):
    R, C = 3, 4
    top = np.full((R, C), 100.0)
    sc = make_scenario(2, R, C, 30.0, 40.0, np.full((1, R, C), 50.0), top, (1.8, 2.7), np.zeros((0, 3)), None,
                       car_r=[0.5])
    orc = oracle_mod.OracleProblem(sc)
    n = 256
    rng = np.random.default_rng(5)
    x0 = rng.standard_normal((n, 1, R, C))
    r = orc.nuts(x0, np.full(n, np.nan), np.full(n, 0.5), inv_mass=np.ones((n, 1, R, C)), n_warmup=100,
                 n_steps=60, seed=14, latent=True)
    assert r["diverged"][:, 100:].sum() == 0
    u = orc.latent_to_heights(r["x"]).reshape(n, -1) / 100.0
    for i in range(R * C):
        assert stats.kstest(u[:, i], "uniform").pvalue > 1e-3
