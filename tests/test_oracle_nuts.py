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
- on the prior-only cave posterior NUTS recovers the uniform marginals;
- one transition preserves 2e5 exact draws of diagonal and correlated
  Gaussians (moments to 4.5 standard errors of 0.3 %, KS of the marginals and
  of the whitened radius), and the same pin fails by a wide margin when a
  mistake is planted in the oracle (U-turn checks inside subtrees skipped, or
  a subtree that turned merged);
- a plain recursive multinomial NUTS written in this file, fed the same
  random draws, reproduces the oracle's trees (depth, leapfrog count,
  divergence, turning, acceptance statistic, chosen state) exactly."""
import math

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


# ---------------------------------------------------------------------------
# Pins of the transition kernel itself, independent of the oracle's
# iterative block bookkeeping
# ---------------------------------------------------------------------------

def _exact_gaussian(cov, n, seed):
    L = np.linalg.cholesky(cov)
    return np.random.default_rng(seed).standard_normal((n, cov.shape[0])) @ L.T


def _stationarity_stats(x, cov):
    """z-scores of the sample means and (co)variances against N(0, cov), the
    smallest KS p-value of the marginals, and the KS p-value of the
    whitened squared radius against chi^2(dim)."""
    n, M = x.shape
    sd = np.sqrt(np.diag(cov))
    z_mean = np.abs(x.mean(axis=0)) / (sd / np.sqrt(n))
    S = (x.T @ x) / n
    # var(x_i x_j) = cov_ii cov_jj + cov_ij^2 for a centred Gaussian
    se = np.sqrt((np.outer(np.diag(cov), np.diag(cov)) + cov ** 2) / n)
    z_cov = np.abs(S - cov) / se
    p_marg = min(stats.kstest(x[:, i] / sd[i], "norm").pvalue for i in range(M))
    w = np.linalg.solve(np.linalg.cholesky(cov), x.T)
    p_rad = stats.kstest((w ** 2).sum(axis=0), stats.chi2(M).cdf).pvalue
    return z_mean.max(), z_cov.max(), p_marg, p_rad


STATIONARITY_CASES = [
    # (name, covariance, eps, inverse mass or None, max_depth)
    ("diag_unit_mass", np.diag([0.5, 1.0, 2.0, 4.0]) ** 2, 0.35, None, 10),
    ("diag_matched_mass", np.diag([0.5, 1.0, 2.0, 4.0]) ** 2, 0.6, np.array([0.25, 1.0, 4.0, 16.0]), 10),
    ("corr2d", np.array([[1.0, 0.95], [0.95, 1.0]]), 0.2, None, 10),
    ("corr2d_capped", np.array([[1.0, 0.95], [0.95, 1.0]]), 0.2, None, 3),
]


@pytest.mark.parametrize("case", STATIONARITY_CASES, ids=[c[0] for c in STATIONARITY_CASES])
def test_one_transition_preserves_exact_gaussian_draws(oracle_mod, case):
    """Any valid MCMC kernel leaves its target invariant: 2e5 exact draws
    of a Gaussian, each moved by one oracle NUTS transition (its own Philox
    chain), are again draws of that Gaussian.  The sample (co)variances have a
    standard error of 0.3 %, so a bias of ~1.5 % fails the 4.5-sigma bar; a
    missed U-turn check inside subtrees, or a merged subtree that turned,
    biases them by tens of percent (checked below)."""
    name, cov, eps, im, depth = case
    n = 200_000
    x0 = _exact_gaussian(cov, n, seed=hash(name) % 1000)
    r = oracle_mod.nuts_dense(np.linalg.inv(cov), x0, eps, inv_mass=im, max_depth=depth, seed=17)
    assert r["diverged"].sum() == 0
    if depth < 10:
        assert (r["depth"] == depth).mean() > 0.3   # the cap binds for many trees
    else:
        assert r["depth"].max() < depth and np.median(r["depth"]) >= 2   # sub-block checks are exercised
    zm, zc, pm, pr = _stationarity_stats(r["x"], cov)
    assert zm < 4.5 and zc < 4.5, (zm, zc)
    assert pm > 1e-4 and pr > 1e-4, (pm, pr)
    # the transition really moved the states
    assert np.mean(np.all(r["x"] == x0, axis=1)) < 0.05


@pytest.mark.parametrize("fault", [1, 2])
def test_stationarity_pin_sees_planted_mistakes(oracle_mod, fault):
    """Power of the pin above: with the U-turn checks inside subtrees
    skipped (fault 1), or a subtree that turned inside merged instead of
    dropped (fault 2), one transition no longer preserves the Gaussian."""
    cov = np.array([[1.0, 0.95], [0.95, 1.0]])
    x0 = _exact_gaussian(cov, 200_000, seed=5)
    try:
        oracle_mod.set_nuts_fault(fault)
        r = oracle_mod.nuts_dense(np.linalg.inv(cov), x0, 0.2, max_depth=10, seed=17)
    finally:
        oracle_mod.set_nuts_fault(0)
    zm, zc, pm, pr = _stationarity_stats(r["x"], cov)
    assert zc > 20 and min(pm, pr) < 1e-10, (zc, pm, pr)


# A plain recursive multinomial NUTS (Hoffman & Gelman 2014, Algorithm 6 in
# its multinomial form; Betancourt 2017 for the generalised criterion and the
# checks across the two halves of every subtree), written here independently
# of the oracle's iterative bookkeeping and fed the same random draws: the
# momentum normals (tag 5), the doubling sides (tag 6), the leaf proposals
# (tag 7, progressive within the subtree) and the merges (tag 8).
_TAG_MOM, _TAG_SIDE, _TAG_LEAF, _TAG_MERGE = 5, 6, 7, 8


def _exp(v):
    return math.exp(v) if v < 709.0 else math.inf


def _logaddexp(a, b):
    if a == -math.inf:
        return b
    if b == -math.inf:
        return a
    m = max(a, b)
    return m + math.log(_exp(a - m) + _exp(b - m))


def _dense_target(P, x):
    lp, g = 0.0, [0.0] * len(x)
    for i in range(len(x)):
        px = 0.0
        for j in range(len(x)):
            px += P[i][j] * x[j]
        g[i] = -px
        lp -= 0.5 * x[i] * px
    return lp, g


def _seqsum(moms):
    """Sum of the momenta of a span, leaf by leaf in build order."""
    s = [0.0] * len(moms[0])
    for p in moms:
        s = [a + b for a, b in zip(s, p)]
    return s


def _no_uturn(x, y, rho, im):
    dx = dy = 0.0
    for k in range(len(rho)):
        dx += x[k] * im[k] * rho[k]
    for k in range(len(rho)):
        dy += y[k] * im[k] * rho[k]
    return dx > 0.0 and dy > 0.0


def _turning(rho_a, a_far, a_near, rho_b, b_near, b_far, im):
    """The span A + B turns unless the generalised criterion holds for the
    whole span and for each half extended by the adjacent end of the other."""
    ok = _no_uturn(a_far, b_far, [u + v for u, v in zip(rho_a, rho_b)], im)
    ok &= _no_uturn(a_far, b_near, [u + v for u, v in zip(rho_a, b_near)], im)
    ok &= _no_uturn(a_near, b_far, [u + v for u, v in zip(a_near, rho_b)], im)
    return not ok


class _Transition:
    def __init__(self, oracle_mod, P, x, im, eps, max_dh, seed, chain, step):
        self.o, self.P, self.im, self.eps, self.max_dh = oracle_mod, P, im, eps, max_dh
        self.seed, self.chain, self.step = seed, chain, step
        M = len(x)
        lp, g = _dense_target(P, x)
        p = [0.0] * M
        kin = 0.0
        for i in range(0, M, 2):
            z = oracle_mod.normal_pair(seed, chain, step, _TAG_MOM, i // 2)
            for e in range(2):
                if i + e < M:
                    p[i + e] = z[e] / math.sqrt(im[i + e])
                    kin += im[i + e] * p[i + e] * p[i + e]
        self.H0 = -lp + 0.5 * kin
        self.p0 = list(p)
        self.ends = [[list(x), list(p), list(g)], [list(x), list(p), list(g)]]   # backward, forward
        self.prop = (list(x), lp)
        self.n_leap, self.sum_acc, self.diverged, self.leaf = 0, 0.0, False, 0

    def u(self, tag, j):
        return float(self.o.uniform_pair(self.seed, self.chain, self.step, tag, j)[0])

    def leaf_step(self, side):
        """One leapfrog step from the tree's end on `side`; returns whether the
        leaf is valid and its momentum."""
        x, p, g = self.ends[side]
        v, eps, im = (1.0 if side else -1.0), self.eps, self.im
        for k in range(len(x)):
            p[k] += 0.5 * v * eps * g[k]
            x[k] = x[k] + v * eps * im[k] * p[k]
        lp, g2 = _dense_target(self.P, x)
        g[:] = g2
        kin = 0.0
        for k in range(len(x)):
            p[k] += 0.5 * v * eps * g[k]
            kin += im[k] * p[k] * p[k]
        self.n_leap += 1
        dH = (-lp + 0.5 * kin) - self.H0
        if not dH <= self.max_dh:
            self.diverged = True
            if dH == dH:
                self.sum_acc += min(1.0, _exp(-dH))
            return False, list(p)
        self.sum_acc += min(1.0, _exp(-dH))
        new = _logaddexp(self.sub_logW, -dH)
        ul = self.u(_TAG_LEAF, self.leaf)
        self.leaf += 1
        if self.sub_prop is None or math.log(ul) < -dH - new:
            self.sub_prop = (list(x), lp)
        self.sub_logW = new
        return True, list(p)

    def build(self, side, j):
        """Subtree of 2^j leaves grown on `side`, recursively: (valid, the
        leaves' momenta in build order)."""
        if j == 0:
            ok, p = self.leaf_step(side)
            return ok, [p]
        ok, A = self.build(side, j - 1)
        if not ok:
            return False, A
        ok, B = self.build(side, j - 1)
        if not ok:
            return False, A + B
        if _turning(_seqsum(A), A[0], A[-1], _seqsum(B), B[0], B[-1], self.im):
            return False, A + B
        return True, A + B

    def run(self, max_depth):
        rho, logW, depth, turned = list(self.p0), 0.0, 0, False
        while depth < max_depth:
            side = 0 if self.u(_TAG_SIDE, depth) < 0.5 else 1
            p_near = list(self.ends[side][1])
            self.sub_logW, self.sub_prop = -math.inf, None
            ok, moms = self.build(side, depth)
            if not ok:
                break
            if math.log(self.u(_TAG_MERGE, depth)) < self.sub_logW - logW:
                self.prop = self.sub_prop
            logW = _logaddexp(logW, self.sub_logW)
            rho_b = _seqsum(moms)
            turned = _turning(rho, self.ends[1 - side][1], p_near, rho_b, moms[0], self.ends[side][1], self.im)
            rho = [a + b for a, b in zip(rho, rho_b)]
            depth += 1
            if turned:
                break
        return dict(x=self.prop[0], depth=depth, n_leap=self.n_leap, diverged=int(self.diverged),
                    turned=int(turned), accept_stat=self.sum_acc / self.n_leap if self.n_leap else 0.0)


TREE_CASES = [
    # (name, covariance, eps, inverse mass or None, max_depth, max_dh)
    ("diag_mass", np.diag([0.5, 1.0, 2.0]) ** 2, 0.3, np.array([0.5, 2.0, 3.0]), 8, 1000.0),
    ("corr2d", np.array([[1.0, 0.9], [0.9, 1.0]]), 0.25, None, 8, 1000.0),
    ("dense3d_capped", np.array([[2.0, 0.5, 0.3], [0.5, 1.0, -0.2], [0.3, -0.2, 0.5]]), 0.15, None, 3, 1000.0),
    ("divergent", np.diag([0.3, 1.0]) ** 2, 0.9, None, 8, 2.0),
]


@pytest.mark.parametrize("case", TREE_CASES, ids=[c[0] for c in TREE_CASES])
def test_oracle_trees_equal_a_recursive_reference(oracle_mod, case):
    """Every tree of the oracle (depth, leapfrog count, divergence, turning,
    acceptance statistic and the chosen state) equals the recursive
    reference's on the same draws, over two transitions of 40 chains."""
    name, cov, eps, im, max_depth, max_dh = case
    n, n_steps, seed = 40, 2, 23
    P = np.linalg.inv(cov)
    x0 = _exact_gaussian(cov, n, seed=7)
    r = oracle_mod.nuts_dense(P, x0, eps, inv_mass=im, max_depth=max_depth, max_dh=max_dh, n_steps=n_steps,
                              seed=seed)
    Pl = P.tolist()
    iml = [1.0] * cov.shape[0] if im is None else list(im)
    compared = 0
    for c in range(n):
        if r["margin"][c] < 1e-10:   # a near-tie: either decision is correct
            continue
        x = list(x0[c])
        for k in range(n_steps):
            t = _Transition(oracle_mod, Pl, x, iml, eps, max_dh, seed, c, k)
            ref = t.run(max_depth)
            for key in ("depth", "n_leap", "diverged", "turned"):
                assert ref[key] == r[key][c, k], (name, c, k, key, ref[key], r[key][c, k])
            assert ref["accept_stat"] == pytest.approx(r["accept_stat"][c, k], rel=1e-14, abs=1e-300)
            x = ref["x"]
        assert np.array_equal(np.array(x), r["x"][c]), (name, c)
        compared += 1
    assert compared >= 0.9 * n
    if name == "divergent":
        assert r["diverged"].sum() > 0
    if name == "dense3d_capped":
        assert (r["depth"] == max_depth).any()
    assert r["turned"].sum() > 0
