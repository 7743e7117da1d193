"""GPU parity of the solid-angle pixel integral (eq. expected_counts as a
quadrature over sub-rays with tabulated log-intensity) against the oracle.

Tolerances: float64 sub-ray opacities to 1e-11 and log posteriors to 1e-11
relative.  float32: sub-ray opacities within the exact march's 1e-5
relative; the log posterior within sum_p |C_p - lambda_p| max_q |dO_q| |d
log I/dO|_max + 1e-6 n_pixels, first order in the opacity error (the
synthetic table's log-slope is at most 1/Lambda + 1/200)."""
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
    from paper_2603_28907_amd.binding import KERNEL_MALA, MuonCaveError, Problem
    torch = torch_mod
    sc, weights, tab, counts = quad
    prob = gpu_problem(quad, "f32")
    H = to_dev(inputs.init_states(sc, 2, seed=1), torch.float32)
    lp = to_dev(np.full(2, np.nan), torch.float64)
    acc = to_dev(np.zeros(2, np.int64), torch.int64)
    g = torch.empty((2, 3, sc.n_rows, sc.n_cols), dtype=torch.float32, device="cuda:0")
    with pytest.raises(MuonCaveError, match="pixel"):
        prob.logpost_grad_batch(H, lp, g)
    with pytest.raises(MuonCaveError, match="MALA"):
        prob.mcmc_run(H, lp, acc, 2, 0.01, 1, kernel=KERNEL_MALA)
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
