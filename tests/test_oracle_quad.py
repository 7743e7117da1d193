"""Pins of the oracle's solid-angle pixel integral (eq. expected_counts):

- one sub-ray per pixel with weight E_p and log I = -O/Lambda reproduces the
  one-ray-per-pixel model exactly;
- on flat layers, where O = c / cos(zenith) in closed form, the midpoint
  quadrature converges to the pixel integral computed by scipy's adaptive
  quadrature, with the error falling about 4x when the sub-cells halve;
- the intensity table is exact at its nodes, linear in log I between them
  and continues its last segment beyond o_max;
- the gradient (each sub-ray's dLL/dO = (C/lambda - 1) w I(O) dlogI/dO
  through the crossing form) reduces to the one-ray model's gradient with
  one sub-ray per pixel and log I = -O/Lambda, and matches central
  differences with 2 x 2 sub-rays and the synthetic table."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2603_28907_amd import inputs
from tests.helpers import make_scenario


def test_one_subray_reduces_to_the_one_ray_model(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    ref = oracle_mod.OracleProblem(sc)
    orc = oracle_mod.OracleProblem(sc)
    o_max = 2000.0
    tab = -np.linspace(0.0, o_max, 64) / sc.atten_len
    orc.set_pixel_quadrature(1, sc.exposure.reshape(-1), tab, o_max, sc.counts.reshape(-1))
    st = inputs.init_states(sc, 3, seed=2)
    for s in st:
        assert orc.logpost(s) == pytest.approx(ref.logpost(s), rel=1e-12)
    lam = orc.pixel_lambda(st[0])
    np.testing.assert_allclose(lam, ref.expected_counts(st[0]), rtol=1e-12)


def _flat(oracle_mod, q, n_zen=3, n_az=4):
    R = C = 5
    X = Y = 2000.0       # wide enough that no ray leaves through a side
    free = np.stack([np.full((R, C), 60.0), np.full((R, C), 80.0)])
    top = np.full((R, C), 200.0)
    dirs, w = inputs.pixel_subrays(n_zen, n_az, q, max_zenith_deg=45.0, exposure=1.0)
    sc = make_scenario(3, R, C, X, Y, free, top, (1.8, 0.0, 2.7), [[X / 2, Y / 2, 0.0]], dirs[None])
    orc = oracle_mod.OracleProblem(sc)
    o_max = 3000.0
    tab = inputs.intensity_table(513, o_max, 400.0)
    orc.set_pixel_quadrature(q * q, w, tab, o_max, np.zeros(n_zen * n_az, np.int32))
    return sc, orc, tab, o_max


def test_quadrature_converges_to_the_pixel_integral(oracle_mod):
    n_zen, n_az = 3, 4
    c = 1.8 * 60.0 + 2.7 * 120.0       # vertical opacity of the flat layers
    sc1, orc1, tab, o_max = _flat(oracle_mod, 1)
    logI = lambda O: np.interp(O, np.linspace(0.0, o_max, tab.size), tab)   # noqa: E731
    dth = math.radians(45.0) / n_zen
    dph = 2.0 * math.pi / n_az
    exact = []
    for k in range(n_zen):
        pix_sa = dph * (math.cos(k * dth) - math.cos((k + 1) * dth))
        f = lambda th: (0.9 - 0.3 * math.sin(th) ** 2) * math.exp(logI(c / math.cos(th))) * math.sin(th)  # noqa
        val, _ = integrate.quad(f, k * dth, (k + 1) * dth, epsabs=1e-13, epsrel=1e-11, limit=200)
        exact += [val * dph / pix_sa] * n_az
    exact = np.array(exact)
    errs, lams = [], []
    for q in (1, 2, 4, 8):
        sc, orc, _, _ = _flat(oracle_mod, q)
        lams.append(orc.pixel_lambda(sc.truth))
        errs.append(np.max(np.abs(lams[-1] - exact) / exact))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.5 < r < 4.5 for r in ratios), (errs, ratios)      # second order
    # Richardson extrapolation of the last two removes the h^2 term
    rich = (4.0 * lams[-1] - lams[-2]) / 3.0
    assert np.max(np.abs(rich - exact) / exact) < 0.05 * errs[-1]


def test_intensity_table_interpolation(oracle_mod):
    sc, orc, tab, o_max = _flat(oracle_mod, 1)
    nodes = np.linspace(0.0, o_max, tab.size)
    np.testing.assert_allclose(orc.log_intensity(nodes[::37]), tab[::37], rtol=0, atol=1e-12)
    mid = 0.5 * (nodes[10] + nodes[11])
    assert orc.log_intensity([mid])[0] == pytest.approx(0.5 * (tab[10] + tab[11]), abs=1e-12)
    beyond = o_max + 100.0
    slope = (tab[-1] - tab[-2]) / (nodes[-1] - nodes[-2])
    assert orc.log_intensity([beyond])[0] == pytest.approx(tab[-1] + slope * 100.0, abs=1e-9)


def test_quadrature_likelihood_is_poisson(oracle_mod):
    sc, orc, _, _ = _flat(oracle_mod, 2)
    lam = orc.pixel_lambda(sc.truth)
    counts = np.random.default_rng(3).poisson(lam * 5e3)
    dirs, wq = inputs.pixel_subrays(3, 4, 2, exposure=5e3)
    orc.set_pixel_quadrature(4, wq, inputs.intensity_table(513, 3000.0, 400.0), 3000.0, counts)
    lam5 = orc.pixel_lambda(sc.truth)
    np.testing.assert_allclose(lam5, 5e3 * lam, rtol=1e-12)
    ll = orc.logpost(sc.truth) - orc.log_prior(sc.truth)
    assert ll == pytest.approx(stats.poisson.logpmf(counts, lam5).sum(), rel=1e-12)


def test_gradient_one_subray_reduces_to_the_one_ray_model(oracle_mod):
    """One sub-ray per pixel with weight E_p and log I = -O/Lambda: the
    quadrature's gradient, (C/lambda - 1) w I(O) dlogI/dO through the crossing
    form, is the one-ray model's (lambda - C)/Lambda, to rounding."""
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    ref = oracle_mod.OracleProblem(sc)
    orc = oracle_mod.OracleProblem(sc)
    o_max = 2000.0
    tab = -np.linspace(0.0, o_max, 64) / sc.atten_len
    orc.set_pixel_quadrature(1, sc.exposure.reshape(-1), tab, o_max, sc.counts.reshape(-1))
    for s in inputs.init_states(sc, 2, seed=3):
        lp, g = orc.grad(s)
        lpr, gr = ref.grad(s)
        assert lp == pytest.approx(lpr, rel=1e-12)
        np.testing.assert_allclose(g, gr, rtol=1e-9, atol=1e-9 * np.abs(gr).max())


def test_gradient_central_differences_with_subrays(oracle_mod):
    """2 x 2 sub-rays per pixel and the synthetic intensity table: the
    gradient against central differences (h = 1e-3 m) of the quadrature's log
    posterior on 48 coordinates; kinks (a crossing over a cell edge, an
    opacity over a table node) detected and skipped."""
    from tests.helpers import is_kink
    sc = inputs.tiny_bumps(seed=0, pix_side=16)
    q = 2
    dirs, w = inputs.pixel_subrays(16, 16, q, max_zenith_deg=45.0, exposure=1e4)
    sc.dirs = np.broadcast_to(dirs, (sc.n_sensors,) + dirs.shape).copy()
    sc.exposure = np.full((sc.n_sensors, dirs.shape[0]), 1e4)
    n_sub = q * q
    o_max = 2000.0
    tab = inputs.intensity_table(256, o_max, sc.atten_len)
    probe = oracle_mod.OracleProblem(sc, counts=np.zeros((sc.n_sensors, dirs.shape[0]), np.int32))
    probe.set_pixel_quadrature(n_sub, np.tile(w, sc.n_sensors), tab, o_max,
                               np.zeros(sc.n_sensors * dirs.shape[0] // n_sub, np.int32))
    lam = probe.pixel_lambda(sc.truth)
    counts = np.random.default_rng(4).poisson(lam).astype(np.int32)
    orc = oracle_mod.OracleProblem(sc, counts=np.zeros((sc.n_sensors, dirs.shape[0]), np.int32))
    orc.set_pixel_quadrature(n_sub, np.tile(w, sc.n_sensors), tab, o_max, counts)
    x0 = inputs.init_states(sc, 1, seed=5)[0]
    lp, g = orc.grad(x0)
    assert np.isfinite(lp) and lp == pytest.approx(orc.logpost(x0), rel=1e-12)
    rng = np.random.default_rng(6)
    h, scale, kinks = 1e-3, np.abs(g).max(), 0
    for k in rng.choice(x0.size, 48, replace=False):
        idx = np.unravel_index(k, x0.shape)
        xp, xm = x0.copy(), x0.copy()
        xp[idx] += h
        xm[idx] -= h
        fp, fm = orc.logpost(xp), orc.logpost(xm)
        fwd, bwd = (fp - lp) / h, (lp - fm) / h
        tol = 1e-4 * scale + 1e-3
        if is_kink(fwd, bwd, tol):
            kinks += 1
            continue
        assert abs((fp - fm) / (2 * h) - g[idx]) <= tol, (idx, (fp - fm) / (2 * h), g[idx])
    assert kinks <= 6
