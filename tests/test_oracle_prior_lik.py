"""Pins of the oracle's prior (Sec. 2.2.1: Gaussian copula over a periodic
proper CAR field per layer) and likelihood (eq. def_likelihood)."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special
import scipy.stats

from tests.helpers import make_scenario


def torus_adjacency(R, C):
    N = R * C
    A = np.zeros((N, N))
    for i in range(R):
        for j in range(C):
            n = i * C + j
            for di, dj in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                m = ((i + di) % R) * C + (j + dj) % C
                A[n, m] = 1.0
    return A


@pytest.mark.parametrize("R,C", [(3, 4), (5, 5), (6, 4)])
@pytest.mark.parametrize("r", [0.5, 0.99, 0.9999])
def test_car_constants_vs_dense_cholesky(oracle_mod, R, C, r):
    """log det Q and Sigma_11 from the torus eigenvalues agree with a dense
    Cholesky factorisation Q = L L^T and the forward solve L v = e_1,
    Sigma_11 = v^T v (eq. CAR_cdf_transform and the sentence after it)."""
    A = torus_adjacency(R, C)
    assert np.all(A.sum(1) == 4)                 # periodic grid: every degree is 4
    Q = np.diag(A.sum(1)) - r * A
    L = np.linalg.cholesky(Q)
    logdet_dense = 2.0 * np.sum(np.log(np.diag(L)))
    e1 = np.zeros(R * C)
    e1[0] = 1.0
    v = scipy.linalg.solve_triangular(L, e1, lower=True)
    s11_dense = float(v @ v)
    # the diagonal of Sigma is constant (translation invariance on the torus)
    assert np.allclose(np.diag(np.linalg.inv(Q)), s11_dense, rtol=1e-9)
    logdet, s11 = oracle_mod.car_consts(R, C, r)
    assert logdet == pytest.approx(logdet_dense, rel=1e-11, abs=1e-10)
    assert s11 == pytest.approx(s11_dense, rel=1e-9)


def test_ndtri_vs_scipy(oracle_mod):
    us = np.concatenate([np.logspace(-300, -1, 200), np.linspace(0.1, 0.5, 50)])
    for u in us:
        w = oracle_mod.ndtri_lower(u)
        ref = scipy.special.ndtri(u)
        assert w == pytest.approx(ref, rel=2e-14, abs=1e-15), u


def prior_scenario(R, C, free, top, r):
    S = free.shape[0] + 1
    return make_scenario(S, R, C, 30.0, 40.0, free, top, np.ones(S), np.zeros((0, 3)), None,
                         car_r=np.asarray(r, float))


def random_ordered_state(rng, R, C, S1, top):
    u = rng.uniform(0.05, 0.95, (S1, R, C))
    out, lo = [], np.zeros((R, C))
    for l in range(S1):
        h = lo + u[l] * (top - lo)
        out.append(h)
        lo = h
    return np.stack(out)


def test_prior_r0_is_independent_uniform_columns(oracle_mod):
    """At r = 0 the copula is independent and the prior reduces to eq.
    indep_columns: H_1 ~ U(0, H_top), H_l | H_{l-1} ~ U(H_{l-1}, H_top)."""
    rng = np.random.default_rng(0)
    R, C = 4, 5
    top = 50 + rng.uniform(0, 5, (R, C))
    free = random_ordered_state(rng, R, C, 2, top)
    sc = prior_scenario(R, C, free, top, [0.0, 0.0])
    prob = oracle_mod.OracleProblem(sc)
    expect = -np.sum(np.log(top)) - np.sum(np.log(top - free[0]))
    assert prob.log_prior(free) == pytest.approx(expect, rel=1e-13)


def generative_map(z, R, C, r, top):
    """The paper's prior sampler: x = L^-T z with Q = L L^T, u = Phi(x/sqrt(S11)),
    H_l = (1-u) H_{l-1} + u H_top (dense linear algebra, small grids only)."""
    N = R * C
    S1 = len(r)
    A = torus_adjacency(R, C)
    H, lo = [], np.zeros(N)
    for l in range(S1):
        Q = np.diag(A.sum(1)) - r[l] * A
        Lc = np.linalg.cholesky(Q)
        x = scipy.linalg.solve_triangular(Lc.T, z[l * N:(l + 1) * N], lower=False)
        e1 = np.zeros(N)
        e1[0] = 1
        v = scipy.linalg.solve_triangular(Lc, e1, lower=True)
        u = scipy.special.ndtr(x / math.sqrt(v @ v))
        h = (1 - u) * lo + u * top.reshape(-1)
        H.append(h)
        lo = h
    return np.concatenate(H)


def inverse_map(H, R, C, r, top):
    N = R * C
    A = torus_adjacency(R, C)
    z, lo = [], np.zeros(N)
    for l in range(len(r)):
        Q = np.diag(A.sum(1)) - r[l] * A
        Lc = np.linalg.cholesky(Q)
        e1 = np.zeros(N)
        e1[0] = 1
        v = scipy.linalg.solve_triangular(Lc, e1, lower=True)
        h = H[l * N:(l + 1) * N]
        u = (h - lo) / (top.reshape(-1) - lo)
        x = scipy.special.ndtri(u) * math.sqrt(v @ v)
        z.append(Lc.T @ x)
        lo = h
    return np.concatenate(z)


@pytest.mark.parametrize("r", [(0.5, 0.9), (0.99, 0.3)])
def test_prior_density_by_brute_force_jacobian(oracle_mod, r):
    """log p(H) = log N(z; 0, I) - log|det dH/dz| for the paper's generative
    map z -> H, with the Jacobian determinant taken numerically (central
    differences) on a 3x4 grid with two free surfaces."""
    R, C = 3, 4
    N = R * C
    rng = np.random.default_rng(2)
    top = 30 + rng.uniform(0, 4, (R, C))
    H = random_ordered_state(rng, R, C, 2, top)
    z = inverse_map(H.reshape(-1), R, C, r, top)
    assert np.allclose(generative_map(z, R, C, r, top), H.reshape(-1), atol=1e-9)
    J = np.empty((2 * N, 2 * N))
    h = 1e-6
    for k in range(2 * N):
        e = np.zeros(2 * N)
        e[k] = h
        J[:, k] = (generative_map(z + e, R, C, r, top) - generative_map(z - e, R, C, r, top)) / (2 * h)
    sign, logabsdet = np.linalg.slogdet(J)
    logp = -0.5 * z @ z - N * math.log(2 * math.pi) - logabsdet
    sc = prior_scenario(R, C, H, top, r)
    prob = oracle_mod.OracleProblem(sc)
    assert prob.log_prior(H) == pytest.approx(logp, abs=2e-6)


def test_prior_support(oracle_mod):
    R, C = 3, 3
    top = np.full((R, C), 10.0)
    good = np.stack([np.full((R, C), 3.0), np.full((R, C), 6.0)])
    sc = prior_scenario(R, C, good, top, [0.7, 0.7])
    prob = oracle_mod.OracleProblem(sc)
    assert np.isfinite(prob.log_prior(good))
    for bad_val, where in [(0.0, (0, 1, 1)), (-1.0, (0, 0, 0)), (6.5, (0, 2, 2)), (10.0, (1, 0, 1)),
                           (np.nan, (1, 1, 1))]:
        bad = good.copy()
        bad[where] = bad_val
        assert prob.log_prior(bad) == -math.inf


def test_loglik_vs_scipy_poisson(oracle_mod):
    """eq. def_likelihood: sum over pixels of the Poisson log-pmf, with
    lambda_p = E_p exp(-O_p / Lambda)."""
    rng = np.random.default_rng(4)
    n_s, n_pix = 3, 50
    E = rng.uniform(1e3, 1e5, (n_s, n_pix))
    O = rng.uniform(0, 2000, n_s * n_pix)
    counts = rng.integers(0, 20000, (n_s, n_pix)).astype(np.int32)
    counts[0, :5] = 0
    sc = make_scenario(2, 3, 3, 10, 10, np.ones((1, 3, 3)), np.full((3, 3), 5.0), (1, 1),
                       np.zeros((n_s, 3)), np.tile([0, 0, 1.0], (n_s, n_pix, 1)), exposure=E,
                       atten=400.0, counts=counts)
    prob = oracle_mod.OracleProblem(sc)
    lam = E.reshape(-1) * np.exp(-O / 400.0)
    ref = float(np.sum(scipy.stats.poisson.logpmf(counts.reshape(-1), lam)))
    assert prob.loglik(O) == pytest.approx(ref, rel=1e-12)
