"""GPU parity of the solid-angle pixel integral (eq. expected_counts as a
quadrature over sub-rays with tabulated log-intensity) against the oracle.

Tolerances: float64 sub-ray opacities to 1e-11 and log posteriors to 1e-11
relative.  float32: sub-ray opacities within the exact march's 1e-5
relative; the log posterior within sum_p |C_p - lambda_p| max_q |dO_q| |d
log I/dO|_max + 1e-6 n_pixels, first order in the opacity error (the
synthetic table's log-slope is at most 1/Lambda + 1/200).

Gradient: every coordinate within the oracle's conditioning bound at the
run's precision (tests.gpu_common), with each sub-ray's dLL/dO =
(C_p/lambda_p - 1) w_q I(O_q) dlog I/dO and its error taken from the
measured sub-ray opacities (the change of that expression between the
oracle's and the GPU's opacities, plus 1e-6 relative for a float32 store);
float64 also within 1e-8 relative in the L2 norm per chain (a small
gradient near the truth amplifies rounding in C_p/lambda_p - 1).  MALA and
NUTS chains in float64 equal the oracle's: the same decisions, and states
within (eps^2/2) n_steps 1e-8 max|grad| (the gradient's own agreement,
carried by every drift term)."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, rounded_states, say, to_dev
from tests.helpers import make_scenario

pytestmark = pytest.mark.gpu

O_MAX = 2500.0


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


@pytest.fixture(scope="module")
def quad(oracle_mod):
    base = inputs.tiny_bumps(seed=0, pix_side=16)
    dirs, w = inputs.pixel_subrays(16, 16, 2, exposure=1e4)
    n_s = base.n_sensors
    sc = make_scenario(3, base.n_rows, base.n_cols, base.extent_x, base.extent_y, base.truth, base.top,
                       base.density, base.sensor_pos, np.broadcast_to(dirs, (n_s,) + dirs.shape),
                       car_r=base.car_r)
    tab = inputs.intensity_table(257, O_MAX, 400.0)
    weights = np.tile(w, n_s)
    orc = oracle_mod.OracleProblem(sc, counts=np.zeros(sc.n_rays, np.int32))
    orc.set_pixel_quadrature(4, weights, tab, O_MAX, np.zeros(sc.n_rays // 4, np.int32))
    lam = orc.pixel_lambda(sc.truth)
    counts = np.random.default_rng(7).poisson(lam).astype(np.int32)
    return sc, weights, tab, counts


def oracle_for(oracle_mod, quad):
    sc, weights, tab, counts = quad
    orc = oracle_mod.OracleProblem(sc, counts=np.zeros(sc.n_rays, np.int32))
    orc.set_pixel_quadrature(4, weights, tab, O_MAX, counts)
    return orc


def gpu_problem(quad, precision):
    from paper_2603_28907_amd.binding import Problem
    sc, weights, tab, counts = quad
    prob = Problem.from_scenario(sc, counts=np.zeros(sc.n_rays, np.int32), precision=precision)
    prob.set_pixel_quadrature(4, weights, tab, O_MAX)
    prob.set_counts(counts)
    return prob


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quad_logpost_matches_oracle(torch_mod, oracle_mod, quad, precision):
    torch = torch_mod
    sc, weights, tab, counts = quad
    prob = gpu_problem(quad, precision)
    orc = oracle_for(oracle_mod, quad)
    states = inputs.init_states(sc, 5, seed=3)
    states[4, 1] = states[4, 0] - 1.0
    dt = torch.float64 if precision == "f64" else torch.float32
    O = torch.empty((5, sc.n_rays), dtype=dt, device="cuda:0")
    lp = prob.logpost_batch(to_dev(states, dt), opacity=O).cpu().numpy()
    O = O.double().cpu().numpy()
    st = rounded_states(states, precision)
    assert lp[4] == -np.inf
    for c in range(4):
        O_ref = orc.opacity(st[c])
        lp_ref = orc.logpost(st[c])
        if precision == "f64":
            np.testing.assert_allclose(O[c], O_ref, rtol=1e-11, atol=1e-9)
            assert lp[c] == pytest.approx(lp_ref, rel=1e-11)
        else:
            err = np.abs(O[c] - O_ref)
            assert np.all(err <= 1e-5 * np.abs(O_ref) + 1e-6), err.max()
            lam = orc.pixel_lambda(st[c])
            bound = np.sum(np.abs(counts - lam) * err.reshape(-1, 4).max(axis=1)) * (1 / 400 + 1 / 200)
            assert abs(lp[c] - lp_ref) <= 1.5 * bound + 1e-6 * counts.size, (lp[c], lp_ref, bound)


def test_quad_rw_matches_oracle(torch_mod, oracle_mod, quad):
    torch = torch_mod
    sc = quad[0]
    prob = gpu_problem(quad, "f64")
    orc = oracle_for(oracle_mod, quad)
    n, n_steps, sigma, seed = 4, 40, 0.05, 919
    states = inputs.init_states(sc, n, seed=8)
    H = to_dev(states, torch.float64)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    acc = to_dev(np.zeros(n, np.int64), torch.int64)
    prob.mcmc_run(H, lp, acc, n_steps, sigma, seed, graph_steps=8)
    torch.cuda.synchronize()
    Ho, lpo, acco, marg = orc.mcmc_rw(states, np.full(n, np.nan), np.zeros(n, np.int64), n_steps, 0, sigma, seed,
                                      want_margins=True)
    say("quad rw margins", np.nanmin(marg), acco)
    assert np.nanmin(marg) > 1e-6 and 0 < acco.sum() < n * n_steps
    assert np.array_equal(acc.cpu().numpy(), acco)
    np.testing.assert_allclose(H.cpu().numpy(), Ho, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(lp.cpu().numpy(), lpo, rtol=1e-11)


def test_quad_errors_and_switching_off(torch_mod, quad):
    from paper_2603_28907_amd.binding import MuonCaveError, Problem
    torch = torch_mod
    sc, weights, tab, counts = quad
    prob = gpu_problem(quad, "f32")
    H = to_dev(inputs.init_states(sc, 2, seed=1), torch.float32)
    with pytest.raises(MuonCaveError, match="pixel quadrature"):
        prob.set_voxel_model(10, 1.0, sc.truth)
    with pytest.raises(MuonCaveError, match="n_sub"):
        prob.set_pixel_quadrature(3, weights, tab, O_MAX)
    # switching off needs the per-ray counts again; then the one-ray model runs
    prob.set_pixel_quadrature(0)
    with pytest.raises(MuonCaveError, match="set_counts"):
        prob.logpost_batch(H)
    prob.set_counts(np.zeros(sc.n_rays, np.int32))
    fresh = Problem.from_scenario(sc, counts=np.zeros(sc.n_rays, np.int32), precision="f32")
    assert np.array_equal(prob.logpost_batch(H).cpu().numpy(), fresh.logpost_batch(H).cpu().numpy())


def subray_dll_do(tab, weights, counts, O):
    """dLL/dO of every sub-ray from opacities O [n_rays] (for the float32
    tolerance only): (C_p / lambda_p - 1) w_q I(O_q) dlog I/dO on O_q's table
    segment, 4 sub-rays per pixel."""
    inv = (tab.size - 1) / O_MAX
    t = O * inv
    j = np.clip(np.floor(t).astype(np.int64), 0, tab.size - 2)
    dl = tab[j + 1] - tab[j]
    wi = weights * np.exp(tab[j] + (t - j) * dl)
    lam = wi.reshape(-1, 4).sum(axis=1)
    return np.repeat(counts / lam - 1.0, 4) * wi * dl * inv


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_quad_gradient_matches_oracle(torch_mod, oracle_mod, quad, precision):
    from tests.gpu_common import f32_gradient_tolerance, f64_gradient_tolerance
    torch = torch_mod
    sc, weights, tab, counts = quad
    prob = gpu_problem(quad, precision)
    orc = oracle_for(oracle_mod, quad)
    n = 4
    states = np.concatenate([sc.truth[None], inputs.init_states(sc, n - 1, seed=5)])
    dt = torch.float64 if precision == "f64" else torch.float32
    H = to_dev(states, dt)
    lp, g = prob.logpost_grad_batch(H)
    O = torch.empty((n, sc.n_rays), dtype=dt, device="cuda:0")
    lp_fwd = prob.logpost_batch(H, opacity=O)
    torch.cuda.synchronize()
    lp, g, lp_fwd, O = (a.double().cpu().numpy() for a in (lp, g, lp_fwd, O))
    st = rounded_states(states, precision)
    lpo, go = orc.grad_batch(st)
    for c in range(n):
        rel = np.linalg.norm(g[c] - go[c]) / np.linalg.norm(go[c])
        say(f"quad grad {precision} chain {c}: relative L2 error {rel:.2e}")
        O_ref = orc.opacity(st[c])
        gp_ref = subray_dll_do(tab, weights, counts, O_ref)
        g_err = np.abs(subray_dll_do(tab, weights, counts, O[c]) - gp_ref) + 1e-6 * np.abs(gp_ref)
        _, gpr = orc.log_prior_grad(st[c])
        err = np.abs(g[c] - go[c])
        if precision == "f64":
            tol = f64_gradient_tolerance(orc, st[c], O[c] - O_ref, gpr, g=gp_ref, g_err=g_err)
            k = np.unravel_index(np.argmax(err / tol), tol.shape)
            say(f"  worst error / bound {err[k] / tol[k]:.3f} at node {k}")
            assert np.all(err <= tol), (c, k, g[c][k], go[c][k], tol[k])
            assert rel < 1e-8
            assert lp[c] == pytest.approx(lpo[c], rel=1e-11)
            assert lp[c] == pytest.approx(lp_fwd[c], rel=1e-13)
            continue
        # the gradient's log posterior: the forward bar, with two float32 ulps
        # of room for the gradient march's own opacities
        lam = orc.pixel_lambda(st[c])
        dO = np.abs(O[c] - O_ref) + 2 * np.spacing(np.abs(O_ref).astype(np.float32)).astype(np.float64)
        bound = np.sum(np.abs(counts - lam) * dO.reshape(-1, 4).max(axis=1)) * (1 / 400 + 1 / 200)
        assert abs(lp[c] - lpo[c]) <= 1.5 * bound + 1e-6 * counts.size, (lp[c], lpo[c], bound)
        tol = f32_gradient_tolerance(orc, st[c], O[c] - O_ref, gpr, g=gp_ref, g_err=g_err)
        k = np.unravel_index(np.argmax(err / tol), tol.shape)
        say(f"  worst error / bound {err[k] / tol[k]:.3f} at node {k}")
        assert np.all(err <= tol), (c, k, g[c][k], go[c][k], tol[k])
        assert rel < 1e-3


def test_quad_mala_f64_matches_oracle(torch_mod, oracle_mod, quad):
    from paper_2603_28907_amd.binding import KERNEL_MALA
    torch = torch_mod
    sc = quad[0]
    prob = gpu_problem(quad, "f64")
    orc = oracle_for(oracle_mod, quad)
    n, n_steps, eps, seed = 4, 20, 0.3, 77
    states = inputs.init_states(sc, n, seed=9)
    Ho, lpo, acco, marg = orc.mcmc_mala(states, np.full(n, np.nan), np.zeros(n, np.int64), n_steps, 0, eps, seed,
                                        want_margins=True)
    say("quad mala acceptances", acco, "min margin", np.nanmin(marg))
    assert np.nanmin(marg) > 1e-6, "a near-tie decision; choose another seed"
    assert 0 < acco.sum() < n * n_steps
    H = to_dev(states, torch.float64)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    acc = to_dev(np.zeros(n, np.int64), torch.int64)
    prob.mcmc_run(H, lp, acc, n_steps, eps, seed, kernel=KERNEL_MALA, graph_steps=5)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), acco)
    _, g0 = orc.grad_batch(states)
    atol = 0.5 * eps ** 2 * n_steps * 1e-8 * np.abs(g0).max()
    say(f"quad mala state tolerance {atol:.2e}")
    np.testing.assert_allclose(H.cpu().numpy(), Ho, rtol=1e-12, atol=atol)
    np.testing.assert_allclose(lp.cpu().numpy(), lpo, rtol=1e-11, atol=1e-6)


@pytest.mark.parametrize("latent", [False, True])
def test_quad_nuts_f64_matches_oracle(torch_mod, oracle_mod, quad, latent):
    """NUTS under the solid-angle pixel integral (heights, or the latent CAR
    fields): f64 trees equal the oracle's."""
    torch = torch_mod
    sc = quad[0]
    prob = gpu_problem(quad, "f64")
    orc = oracle_for(oracle_mod, quad)
    n = 4
    states = inputs.init_states(sc, n, seed=13)
    x = orc.heights_to_latent(states) if latent else states
    eps = np.full(n, 0.01) if latent else np.array([0.01, 0.02, 0.015, 0.01])
    H = to_dev(x, torch.float64)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    st = prob.nuts_run(H, lp, to_dev(eps, torch.float64), n_steps=3, seed=29, max_depth=5, latent=latent)
    torch.cuda.synchronize()
    o = orc.nuts(x, np.full(n, np.nan), eps, max_depth=5, n_steps=3, seed=29, latent=latent)
    say("quad nuts depths", o["depth"].tolist(), "margins", o["margin"])
    ok = [c for c in range(n) if o["margin"][c] > 1e-7]
    assert len(ok) >= 3
    assert o["n_leap"].sum() > 20
    for c in ok:
        assert np.array_equal(st["tree_depth"].cpu().numpy()[c], o["depth"][c])
        assert np.array_equal(st["n_leapfrog"].cpu().numpy()[c], o["n_leap"][c])
        np.testing.assert_allclose(H.cpu().numpy()[c], o["x"][c], rtol=1e-9, atol=1e-9)
