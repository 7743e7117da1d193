"""Pins of the oracle's smoothed voxel forward model (Sec. 2.1.2 and 2.1.4)
against what the paper and the mathematics fix, not against itself:

- the scaled sigmoid: value 1/2 at 0, symmetry, the Heaviside limit;
- the normalised weights: a partition of unity, non-negative, local to their
  column, and in the limit gamma -> 0 the hard-interface density (the unit
  that contains the voxel centre, found here by counting surfaces);
- ray-voxel lengths: brute-force midpoint sampling of the ray with an
  independent point-to-voxel map, and the total length to the box exit;
- flat layers on voxel boundaries at gamma -> 0: the closed form
  sum rho * thickness / cos(theta), and the exact march's opacity;
- the linearisation: exact at the reference, and its error against the
  unlinearised count E exp(-O/Lambda) is second order in the perturbation
  (a wrong sign or scale of G makes it first order);
- the likelihood against scipy's Poisson log-pmf at the reference state."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2603_28907_amd import inputs
from tests.helpers import box_exit, make_scenario, unit


def test_sigmoid_half_symmetry_and_heaviside_limit(oracle_mod):
    lib = oracle_mod._load()
    for g in (0.1, 1.0, 5.0):
        assert lib.orc_sigmoid(0.0, g) == 0.5
        for u in (0.3, 2.0, 17.0):
            assert lib.orc_sigmoid(u, g) + lib.orc_sigmoid(-u, g) == pytest.approx(1.0, abs=1e-15)
            assert lib.orc_sigmoid(u, g) > 0.5 > lib.orc_sigmoid(-u, g)
    assert lib.orc_sigmoid(0.05, 1e-3) == 1.0
    assert lib.orc_sigmoid(-0.05, 1e-3) < 1e-20


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    return sc


def test_weights_partition_of_unity_and_locality(oracle_mod, tiny):
    orc = oracle_mod.OracleProblem(tiny)
    n_z = 25
    W = orc.voxel_weights(tiny.truth, n_z, 1.0)
    assert W.shape == (tiny.n_rows, tiny.n_cols, n_z, tiny.n_surfaces + 1)
    assert np.all(W >= 0.0)
    np.testing.assert_allclose(W.sum(axis=-1), 1.0, atol=1e-14)
    # raising surface 1 at one node changes only that column: unit 1 gains, unit 2 loses
    up = tiny.truth.copy()
    up[0, 5, 7] += 3.0
    W2 = orc.voxel_weights(up, n_z, 1.0)
    diff = np.abs(W2 - W).sum(axis=(2, 3))
    assert diff[5, 7] > 1e-3
    diff[5, 7] = 0.0
    assert diff.max() == 0.0
    assert np.all(W2[5, 7, :, 0] >= W[5, 7, :, 0]) and np.all(W2[5, 7, :, 1] <= W[5, 7, :, 1])
    # the density lies between the smallest and largest unit density (air included)
    Rh = orc.voxel_density(tiny.truth, n_z, 1.0)
    assert Rh.min() >= 0.0 and Rh.max() <= max(tiny.density) + 1e-12


def test_gamma_to_zero_gives_the_hard_interface_density(oracle_mod, tiny):
    orc = oracle_mod.OracleProblem(tiny)
    n_z = 40
    Rh = orc.voxel_density(tiny.truth, n_z, 1e-4)
    surf = np.concatenate([tiny.truth, tiny.top[None]])          # [S, R, C]
    dz = tiny.top.max() / n_z
    z = (np.arange(n_z) + 0.5) * dz
    below = surf[:, :, :, None] <= z[None, None, None, :]          # surfaces at or below z
    unit_idx = below.sum(axis=0)                                   # 0 -> unit 1, ..., S -> air
    rho = np.concatenate([tiny.density, [0.0]])
    hard = rho[unit_idx]
    gap = np.min(np.abs(surf[:, :, :, None] - z[None, None, None, :]), axis=0)
    far = gap > 0.02
    assert far.mean() > 0.95
    np.testing.assert_allclose(Rh[far], hard[far], atol=1e-12)


def _voxel_of_points(x, y, z, R, C, n_z, X, Y, ztop):
    dx, dy, dz = X / (R - 1), Y / (C - 1), ztop / n_z
    i = np.clip(np.rint(x / dx).astype(int), 0, R - 1)      # nearest node column
    j = np.clip(np.rint(y / dy).astype(int), 0, C - 1)
    k = np.clip((z / dz).astype(int), 0, n_z - 1)
    return (i * C + j) * n_z + k


def test_voxel_pieces_match_brute_force_sampling(oracle_mod, tiny):
    orc = oracle_mod.OracleProblem(tiny)
    n_z = 30
    ztop = tiny.top.max()
    rng = np.random.default_rng(5)
    for ray in rng.choice(tiny.n_rays, size=12, replace=False):
        s = ray // tiny.n_pix
        q, d = tiny.sensor_pos[s], tiny.dirs[s, ray % tiny.n_pix]
        vox, ln = orc.voxel_pieces(int(ray), n_z)
        T = box_exit(q, d, tiny.extent_x, tiny.extent_y, ztop)
        assert ln.sum() == pytest.approx(T, rel=1e-12)
        assert np.all(ln > 0)
        delta = T / 200000
        tm = (np.arange(200000) + 0.5) * delta
        v = _voxel_of_points(q[0] + tm * d[0], q[1] + tm * d[1], q[2] + tm * d[2], tiny.n_rows, tiny.n_cols, n_z,
                             tiny.extent_x, tiny.extent_y, ztop)
        bf = np.bincount(v, minlength=tiny.n_rows * tiny.n_cols * n_z) * delta
        ex = np.bincount(vox, weights=ln, minlength=bf.size)
        assert set(np.nonzero(ex)[0]) >= set(np.nonzero(bf > 2 * delta)[0])
        assert np.max(np.abs(ex - bf)) <= 2 * delta + 1e-12


def _flat_problem(oracle_mod, n_grid=9, extent=80.0):
    dirs = np.array([unit([0.0, 0.0, 1.0]), unit([0.1, 0.05, 1.0]), unit([-0.2, 0.1, 1.0]),
                     unit([0.05, -0.15, 1.0])])
    free = np.stack([np.full((n_grid, n_grid), 60.0), np.full((n_grid, n_grid), 80.0)])
    top = np.full((n_grid, n_grid), 200.0)
    sc = make_scenario(3, n_grid, n_grid, extent, extent, free, top, (1.8, 0.0, 2.7),
                       [[40.0, 40.0, 0.0]], dirs[None])
    sc.counts = np.full((1, 4), 100, np.int32)
    return sc


def test_flat_layers_hard_limit_equals_closed_form(oracle_mod):
    sc = _flat_problem(oracle_mod)
    orc = oracle_mod.OracleProblem(sc)
    n_z = 100                                     # dz = 2 m: 60 and 80 lie on voxel boundaries
    orc.set_voxel_model(n_z, 1e-4, sc.truth)
    _, O = orc.voxel_loglik(sc.truth, with_opacity=True)
    d = sc.dirs.reshape(-1, 3)
    closed = (1.8 * 60.0 + 0.0 * 20.0 + 2.7 * 120.0) / d[:, 2]
    np.testing.assert_allclose(O, closed, rtol=1e-12)
    orc_exact = oracle_mod.OracleProblem(sc)
    np.testing.assert_allclose(O, orc_exact.opacity(sc.truth), rtol=1e-12)


def test_linearisation_exact_at_reference_and_second_order(oracle_mod, tiny):
    orc = oracle_mod.OracleProblem(tiny)
    n_z = 50
    ref = tiny.truth
    orc.set_voxel_model(n_z, 1.0, ref)
    ll0, O0 = orc.voxel_loglik(ref, with_opacity=True)
    lam0 = tiny.exposure.reshape(-1) * np.exp(-O0 / tiny.atten_len)
    c = tiny.counts.reshape(-1)
    assert ll0 == pytest.approx(stats.poisson.logpmf(c, lam0).sum(), rel=1e-12)
    # a smooth bump on surface 1, small against gamma so that the voxel
    # opacity change is linear in its height t
    R, C = tiny.n_rows, tiny.n_cols
    xs = np.linspace(-1, 1, R)[:, None]
    ys = np.linspace(-1, 1, C)[None, :]
    bump = np.exp(-4 * (xs ** 2 + ys ** 2))
    errs = []
    for t in (0.1, 0.05, 0.025):
        h = ref.copy()
        h[0] -= t * bump
        ll_lin, O = orc.voxel_loglik(h, with_opacity=True)
        ll_exact = stats.poisson.logpmf(c, tiny.exposure.reshape(-1) * np.exp(-O / tiny.atten_len)).sum()
        errs.append(abs(ll_lin - ll_exact))
        assert abs(O - O0).max() > 1e-2 * t
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(3.2 < r < 4.8 for r in ratios), (errs, ratios)


def test_logpost_and_nonpositive_counts(oracle_mod, tiny):
    orc = oracle_mod.OracleProblem(tiny)
    orc.set_voxel_model(30, 1.0, tiny.truth)
    st = inputs.init_states(tiny, 3, seed=4)
    for s in st:
        assert orc.logpost(s) == pytest.approx(orc.log_prior(s) + orc.voxel_loglik(s), rel=1e-13)
    bad = st[0].copy()
    bad[1] = bad[0] - 1.0
    assert orc.logpost(bad) == -np.inf
    # a short attenuation length: lowering the cave back by 30 m adds rock on
    # the way and drives the linearised count of some pixel below zero
    o2 = oracle_mod.OracleProblem(tiny, atten_len=5.0)
    o2.set_voxel_model(30, 1.0, tiny.truth)
    assert math.isfinite(o2.voxel_loglik(tiny.truth))
    low = tiny.truth.copy()
    low[1] = low[0] + 0.5
    assert o2.voxel_loglik(low) == -np.inf
    # the gradient of the voxel model: finite, and zero where some linearised
    # count is not positive (log posterior -inf)
    lp, g = orc.grad(st[0])
    assert lp == pytest.approx(orc.logpost(st[0]), rel=1e-13) and np.all(np.isfinite(g))
    lpl, gl = o2.grad(low)
    assert lpl == -np.inf and np.all(gl == 0.0)
    orc.set_voxel_model(0)
    assert math.isfinite(orc.logpost(st[0]))


def test_voxel_gradient_central_differences(oracle_mod, tiny):
    """The voxel model is smooth in the heights: the oracle's gradient
    (chain rule through the linearised counts, G and the sigmoid
    derivatives) equals central differences of its log posterior on 48
    free and 16 top coordinates (R0 kept fixed)."""
    import copy
    n_z, gamma = 25, 2.0
    tiny = copy.copy(tiny)   # a terrain with one highest node, so the box lid stays put
    xs = np.linspace(0.0, 1.0, tiny.n_rows)[:, None] + np.linspace(0.0, 0.7, tiny.n_cols)[None, :]
    tiny.top = 200.0 - 4.0 * xs
    tiny.counts = oracle_mod.make_counts(tiny, seed=1)
    orc = oracle_mod.OracleProblem(tiny)
    orc.set_voxel_model(n_z, gamma, tiny.truth)
    x0 = inputs.init_states(tiny, 1, seed=21, jitter=1.0)[0]
    lp, g = orc.grad(x0)
    assert np.isfinite(lp) and lp == pytest.approx(orc.logpost(x0), rel=1e-13)
    assert np.abs(g[2]).max() > 0.0   # the top surface has a gradient too
    rng = np.random.default_rng(22)
    h = 1e-4
    scale = np.abs(g).max()
    free = [np.unravel_index(k, x0.shape) for k in rng.choice(x0.size, 48, replace=False)]
    for idx in free:
        xp, xm = x0.copy(), x0.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (orc.logpost(xp) - orc.logpost(xm)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * scale + 1e-5, (idx, fd, g[idx])
    argmax = np.unravel_index(np.argmax(tiny.top), tiny.top.shape)
    tops = [np.unravel_index(k, tiny.top.shape) for k in rng.choice(tiny.top.size, 17, replace=False)]
    tops = [t for t in tops if t != argmax][:16]
    for t in tops:
        vals = []
        for sgn in (1.0, -1.0):
            sc2 = copy.copy(tiny)
            sc2.top = tiny.top.copy()
            sc2.top[t] += sgn * h
            o2 = oracle_mod.OracleProblem(sc2)
            o2.set_voxel_model(n_z, gamma, tiny.truth)
            o2._vox_ref[...] = orc._vox_ref   # the same linearisation point R0
            vals.append(o2.logpost(x0))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[2][t]) <= 1e-6 * scale + 1e-5, (t, fd, g[2][t])


def test_voxel_gradient_uniform_lift_sum_rule(oracle_mod):
    """Flat layers crossed inside the box by one ray: lifting a surface
    uniformly moves every smoothed interface by the same amount, and the
    ray's length per level is dz / d_z, so the node gradients of the
    opacity sum to (rho_l - rho_{l+1}) / d_z (the exact march's sum rule)
    up to the midpoint sum of the sigmoid's derivative over the levels,
    which is below 1e-6 for gamma = dz."""
    R, C, X, Y = 6, 5, 100.0, 80.0
    levels = [30.0, 45.0, 90.0]
    dens = np.array([1.8, 0.0, 2.7])
    free = np.stack([np.full((R, C), c) for c in levels[:2]])
    d = unit([0.2, 0.1, 1.0])
    q = np.array([40.0, 30.0, 0.0])
    sc = make_scenario(3, R, C, X, Y, free, np.full((R, C), levels[2]), dens, q[None], d[None, None],
                       exposure=np.array([[1e4]]), counts=np.array([[100]], np.int32), car_r=np.array([0.5, 0.5]))
    orc = oracle_mod.OracleProblem(sc)
    n_z = 45                              # dz = 2 m
    orc.set_voxel_model(n_z, 2.0, free)   # at the reference, lambda-hat = lambda(R0)
    lp, g = orc.grad(free)
    _, gprior = orc.log_prior_grad(free)
    _, O = orc.voxel_loglik(free, with_opacity=True)
    lam0 = 1e4 * math.exp(-O[0] / 400.0)
    dll_do = (100.0 / lam0 - 1.0) * (-lam0 / 400.0)
    dOdH = (g - gprior) / dll_do
    for l in range(2):
        expect = (dens[l] - dens[l + 1]) / d[2]
        assert dOdH[l].sum() == pytest.approx(expect, rel=1e-5), (l, dOdH[l].sum(), expect)
