"""Pins of the sampler's latent vector with the hierarchical dependence:
z = (x, logit r), r_l ~ Uniform(0, 1) a priori (Sec. 2.2.1), sampled jointly
with the CAR fields (Sec. 3.1).

- at any r, the density minus the Jacobian log(r (1 - r)) equals the
  fixed-r latent density of a problem whose r is that r (itself pinned by
  the change of variables to the density in H);
- the gradient in x and in logit r against central differences, with data;
- NUTS on z for the prior-only problem, started from exact draws of the
  joint prior (r uniform, x ~ N(0, Q(r)^-1) by a dense Cholesky factor),
  keeps r uniform (KS) and x at its prior variance; with the Jacobian
  planted out of the oracle the same test fails."""
import copy

import numpy as np
import pytest
from scipy import stats

from paper_2603_28907_amd import inputs
from tests.helpers import make_scenario


def _with_r(sc, r):
    sc2 = copy.copy(sc)
    sc2.car_r = np.asarray(r, np.float64)
    return sc2


def test_density_reduces_to_the_fixed_r_latent_density(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    orc = oracle_mod.OracleProblem(sc)
    rng = np.random.default_rng(3)
    for _ in range(3):
        r = rng.uniform(0.05, 0.995, size=2)
        ref = oracle_mod.OracleProblem(_with_r(sc, r))
        x = ref.heights_to_latent(inputs.init_states(sc, 1, seed=int(rng.integers(100)))[0])[0]
        v = orc.latent_r_logpost(x, r)
        expect = ref.latent_logpost(x) + np.sum(np.log(r * (1.0 - r)))
        assert v == pytest.approx(expect, rel=1e-12)


def test_gradient_central_differences(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    orc = oracle_mod.OracleProblem(sc)
    r = np.array([0.7, 0.95])
    ref = oracle_mod.OracleProblem(_with_r(sc, r))
    x = ref.heights_to_latent(inputs.init_states(sc, 1, seed=5)[0])[0]
    v, gx, geta = orc.latent_r_logpost(x, r, with_grad=True)
    eta = np.log(r / (1.0 - r))
    h = 1e-5
    for l in range(2):
        ep, em = eta.copy(), eta.copy()
        ep[l] += h
        em[l] -= h
        fd = (orc.latent_r_logpost(x, 1.0 / (1.0 + np.exp(-ep))) -
              orc.latent_r_logpost(x, 1.0 / (1.0 + np.exp(-em)))) / (2 * h)
        assert geta[l] == pytest.approx(fd, rel=1e-5, abs=1e-4), (l, geta[l], fd)
    rng = np.random.default_rng(6)
    scale = np.abs(gx).max()
    kinks = 0
    for k in rng.choice(x.size, 24, replace=False):
        idx = np.unravel_index(k, x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fp, fm = orc.latent_r_logpost(xp, r), orc.latent_r_logpost(xm, r)
        fwd, bwd = (fp - v) / h, (v - fm) / h
        if abs(fwd - bwd) > 1e-3 * scale + 1e-2 * abs(fwd + bwd):
            kinks += 1   # a kink of the piecewise-smooth likelihood
            continue
        assert gx[idx] == pytest.approx((fp - fm) / (2 * h), rel=1e-4, abs=1e-4 * scale), (idx,)
    assert kinks <= 3


def _prior_problem(oracle_mod, R=3, C=4):
    rng = np.random.default_rng(0)
    top = 100.0 + 5.0 * rng.random((R, C))
    free = np.stack([np.full((R, C), 30.0), np.full((R, C), 60.0)])
    sc = make_scenario(3, R, C, 30.0, 40.0, free, top, (1.8, 0.0, 2.7), np.zeros((0, 3)), None,
                       car_r=np.full(2, 0.5))
    return sc, oracle_mod.OracleProblem(sc)


def _exact_prior_draws(R, C, n, seed):
    """r ~ U(0, 1) per free surface and x_l ~ N(0, Q(r_l)^-1), Q = 4 I - r A on
    the R x C torus, by a dense Cholesky factor of Q."""
    rng = np.random.default_rng(seed)
    N = R * C
    A = np.zeros((N, N))
    for i in range(R):
        for j in range(C):
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                A[i * C + j, ((i + di) % R) * C + (j + dj) % C] += 1.0
    r = rng.uniform(size=(n, 2))
    x = np.empty((n, 2, R, C))
    for c in range(n):
        for l in range(2):
            L = np.linalg.cholesky(4.0 * np.eye(N) - r[c, l] * A)
            x[c, l] = np.linalg.solve(L.T, rng.standard_normal(N)).reshape(R, C)
    return x, r


@pytest.mark.parametrize("fault", [0, 4])
def test_prior_only_nuts_keeps_r_uniform(oracle_mod, fault):
    sc, orc = _prior_problem(oracle_mod)
    n = 400
    x0, r0 = _exact_prior_draws(sc.n_rows, sc.n_cols, n, seed=7)
    try:
        oracle_mod.set_nuts_fault(fault)
        out = orc.nuts(x0, np.full(n, np.nan), np.full(n, 0.3), max_depth=6, n_steps=30, seed=9, latent=True, r=r0)
    finally:
        oracle_mod.set_nuts_fault(0)
    r = out["r"].ravel()
    p = stats.kstest(r, "uniform").pvalue
    moved = np.mean(np.abs(out["r"] - r0) > 1e-3)
    if fault == 0:
        assert out["diverged"].sum() == 0
        assert moved > 0.9
        assert p > 1e-3, p
    else:
        assert p < 1e-6, p
