"""GPU parity of the paper's smoothed voxel forward model (linearised around
R0 = R-hat(H_ref)) against the oracle.

Tolerances.  float64 mode: voxel opacities O_p(R-hat) within 1e-11
relative and log posteriors within 1e-11 relative.  float32 mode: the
smoothed densities carry the float32 rounding of the indicator argument
(z - H)/gamma (|dz| <= 2^-24 z_max), which moves each sigma by at most a
quarter of that; summed along a ray this stays far below 1e-5 O_p, the bar
of the exact march, which is used here too.  The float32 log posterior is
then held to sum_p (C_p/lambda-hat_p + 1) lambda_p(R0) |dO_p| / Lambda
(first order in the opacity error) + 1e-6 n_ray."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, rounded_states, say, to_dev
from tests.helpers import make_scenario

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    return sc


def gpu_vox(torch, sc, states, precision, n_z, gamma, ref, export=True):
    from paper_2603_28907_amd.binding import Problem
    prob = Problem.from_scenario(sc, precision=precision)
    prob.set_voxel_model(n_z, gamma, ref)
    dt = torch.float64 if precision == "f64" else torch.float32
    H = to_dev(states, dt)
    n = H.shape[0]
    O = torch.empty((n, sc.n_rays), dtype=dt, device="cuda:0") if export else None
    lp = prob.logpost_batch(H, opacity=O)
    torch.cuda.synchronize()
    return lp.cpu().numpy(), (O.double().cpu().numpy() if export else None), prob


def oracle_vox(oracle_mod, sc, n_z, gamma, ref, atten=None):
    orc = oracle_mod.OracleProblem(sc, atten_len=atten)
    orc.set_voxel_model(n_z, gamma, ref)
    return orc


def check(oracle_mod, sc, states, lp, O, precision, n_z, gamma, ref, label):
    orc = oracle_vox(oracle_mod, sc, n_z, gamma, ref)
    st = rounded_states(states, precision)
    _, O0 = orc.voxel_loglik(ref, with_opacity=True)
    lam0 = sc.exposure.reshape(-1) * np.exp(-O0 / sc.atten_len)
    cnt = sc.counts.reshape(-1)
    for c in range(st.shape[0]):
        lp_ref = orc.logpost(st[c])
        if not np.isfinite(lp_ref):
            assert lp[c] == lp_ref, (label, c, lp[c], lp_ref)
            continue
        _, O_ref = orc.voxel_loglik(st[c], with_opacity=True)
        if precision == "f64":
            np.testing.assert_allclose(O[c], O_ref, rtol=1e-11, atol=1e-9, err_msg=label)
            assert lp[c] == pytest.approx(lp_ref, rel=1e-11, abs=1e-6), (label, c)
        else:
            err = np.abs(O[c] - O_ref)
            assert np.all(err <= 1e-5 * np.abs(O_ref) + 1e-6), (label, c, err.max())
            lam = lam0 * (1.0 - (O_ref - O0) / sc.atten_len)
            bound = np.sum((cnt / lam + 1.0) * lam0 * err) / sc.atten_len
            assert abs(lp[c] - lp_ref) <= 1.5 * bound + 1e-6 * sc.n_rays, (label, c, lp[c], lp_ref, bound)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tiny_voxel_parity(torch_mod, oracle_mod, tiny, precision):
    states = inputs.init_states(tiny, 5, seed=2)
    states[4, 1] = states[4, 0] - 1.0        # outside the support
    ref = tiny.truth
    say(f"voxel {precision}: tiny, n_z 50")
    lp, O, _ = gpu_vox(torch_mod, tiny, states, precision, 50, 1.0, ref)
    assert lp[4] == -np.inf
    check(oracle_mod, tiny, states, lp, O, precision, 50, 1.0, ref, f"tiny-{precision}")


@pytest.mark.parametrize("S,R,C,n_pix,n_chains,n_z,gamma", [
    (2, 3, 3, 5, 1, 1, 1.0),          # minimum grid, one level, one chain
    (3, 7, 5, 9, 70, 17, 0.5),        # non-square, ragged tile and chain group
    (4, 12, 9, 11, 3, 40, 2.0),       # four surfaces
])
def test_shapes_chains_and_levels(torch_mod, oracle_mod, S, R, C, n_pix, n_chains, n_z, gamma):
    rng = np.random.default_rng(100 + S * R)
    X, Y = 60.0, 45.0
    base = 30.0 + 5.0 * rng.standard_normal((R, C))
    free = np.stack([base + 12.0 * l + 2.0 * rng.random((R, C)) for l in range(S - 1)])
    top = 120.0 + rng.random((R, C))
    dens = (1.8, 0.0, 2.7, 2.2)[:S]
    pos = np.array([[X * 0.4, Y * 0.55, 0.0], [X * 0.7, Y * 0.3, 2.0]])
    th = np.radians(rng.uniform(2, 40, n_pix))
    ph = rng.uniform(0, 2 * np.pi, n_pix)
    d1 = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    sc = make_scenario(S, R, C, X, Y, free, top, dens, pos, np.stack([d1, d1[::-1]]), car_r=np.full(S - 1, 0.7))
    sc.counts = oracle_mod.make_counts(sc, seed=3)
    states = np.stack([free + 0.3 * rng.standard_normal(free.shape) for _ in range(n_chains)])
    states = np.sort(states, axis=1)
    ref = free
    for precision in ("f64", "f32"):
        lp, O, _ = gpu_vox(torch_mod, sc, states, precision, n_z, gamma, ref)
        pick = sorted({0, n_chains - 1, n_chains // 2, min(64, n_chains - 1)})
        check(oracle_mod, sc, states[pick], lp[pick], O[pick], precision, n_z, gamma, ref,
              f"S{S} {R}x{C} n{n_chains} {precision}")


def test_nonpositive_linearised_counts_give_minus_inf(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.tiny_bumps(seed=0)
    sc.atten_len = 5.0
    sc.counts = tiny.counts
    low = tiny.truth.copy()
    low[1] = low[0] + 0.5
    states = np.stack([tiny.truth, low])
    prob = Problem.from_scenario(sc, precision="f64")
    prob.set_voxel_model(30, 1.0, tiny.truth)
    lp = prob.logpost_batch(to_dev(states, torch.float64)).cpu().numpy()
    orc = oracle_vox(oracle_mod, sc, 30, 1.0, tiny.truth, atten=5.0)
    assert np.isfinite(lp[0]) and lp[0] == pytest.approx(orc.logpost(states[0]), rel=1e-11)
    assert lp[1] == -np.inf and orc.logpost(states[1]) == -np.inf


def test_rw_with_voxel_model_matches_oracle(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    n, n_steps, sigma, seed = 4, 60, 0.05, 515
    states = inputs.init_states(tiny, n, seed=7)
    prob = Problem.from_scenario(tiny, precision="f64")
    prob.set_voxel_model(40, 1.0, tiny.truth)
    H = to_dev(states, torch.float64)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    acc = to_dev(np.zeros(n, np.int64), torch.int64)
    prob.mcmc_run(H, lp, acc, n_steps, sigma, seed, graph_steps=10)
    torch.cuda.synchronize()
    orc = oracle_vox(oracle_mod, tiny, 40, 1.0, tiny.truth)
    Ho, lpo, acco, marg = orc.mcmc_rw(states, np.full(n, np.nan), np.zeros(n, np.int64), n_steps, 0, sigma, seed,
                                      want_margins=True)
    say("voxel rw: margins", np.nanmin(marg), "accepts", acco)
    assert np.nanmin(marg) > 1e-6
    assert 0 < acco.sum() < n * n_steps
    assert np.array_equal(acc.cpu().numpy(), acco)
    np.testing.assert_allclose(H.cpu().numpy(), Ho, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(lp.cpu().numpy(), lpo, rtol=1e-11, atol=1e-6)


def test_graph_eager_repeat_bitwise_and_switching_back(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    states = inputs.init_states(tiny, 6, seed=9)
    outs = []
    for G in (8, 1):
        prob = Problem.from_scenario(tiny, precision="f32")
        prob.set_voxel_model(40, 1.0, tiny.truth)
        H = to_dev(states, torch.float32)
        lp = to_dev(np.full(6, np.nan), torch.float64)
        acc = to_dev(np.zeros(6, np.int64), torch.int64)
        prob.mcmc_run(H, lp, acc, 32, 0.05, 3, graph_steps=G)
        torch.cuda.synchronize()
        outs.append((H.cpu().numpy(), lp.cpu().numpy(), acc.cpu().numpy()))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    assert outs[0][2].sum() > 0
    # n_z = 0: back to the exact march, identical to a problem that never had the voxel model
    prob.set_voxel_model(0)
    H = to_dev(states, torch.float32)
    lp_back = prob.logpost_batch(H).cpu().numpy()
    fresh = Problem.from_scenario(tiny, precision="f32")
    lp_fresh = fresh.logpost_batch(H).cpu().numpy()
    assert np.array_equal(lp_back, lp_fresh)


def test_voxel_model_errors(torch_mod, tiny):
    from paper_2603_28907_amd.binding import MuonCaveError, Problem, mcmc_run_multi, time_march
    torch = torch_mod
    prob = Problem.from_scenario(tiny, precision="f32")
    with pytest.raises(MuonCaveError, match="n_z"):
        prob.set_voxel_model(5000, 1.0, tiny.truth)
    with pytest.raises(MuonCaveError, match="gamma"):
        prob.set_voxel_model(10, -1.0, tiny.truth)
    prob.set_voxel_model(10, 1.0, tiny.truth)
    n = 2
    H = to_dev(inputs.init_states(tiny, n, seed=1), torch.float32)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    acc = to_dev(np.zeros(n, np.int64), torch.int64)
    with pytest.raises(MuonCaveError, match="exact march"):
        mcmc_run_multi([prob], [H], [lp], [acc], 2, [0.01], [1])
    with pytest.raises(MuonCaveError, match="mc_time_voxel"):
        time_march(prob, H)
    # new sensors switch the model off
    prob.set_sensors(tiny.sensor_pos, tiny.dirs, tiny.exposure, tiny.atten_len)
    prob.set_counts(tiny.counts)
    fresh = Problem.from_scenario(tiny, precision="f32")
    assert np.array_equal(prob.logpost_batch(H).cpu().numpy(), fresh.logpost_batch(H).cpu().numpy())


def test_paper_scale_sampled_chains(torch_mod, oracle_mod):
    """The 64x64 paper-scale geometry (32768 rays) with 100 levels of 2.1 m,
    at the benchmark's launch configuration (1024 chains); a sample of chains
    is compared with the oracle."""
    from paper_2603_28907_amd.binding import time_voxel
    torch = torch_mod
    sc = inputs.grf_cave(seed=10)
    sc.counts = oracle_mod.make_counts(sc, seed=11)
    n = 1024
    states = inputs.init_states(sc, n, seed=12)
    say("voxel paper scale: 1024 chains")
    lp, O, prob = gpu_vox(torch, sc, states, "f32", 100, 1.0, sc.truth, export=False)
    assert np.all(np.isfinite(lp))
    pick = [0, 333, 777, 1023]
    H = to_dev(states[pick], torch.float32)
    Op = torch.empty((len(pick), sc.n_rays), dtype=torch.float32, device="cuda:0")
    lp_small = prob.logpost_batch(H, opacity=Op).cpu().numpy()
    assert np.array_equal(lp_small, lp[pick])     # a chain's value does not depend on the batch
    check(oracle_mod, sc, states[pick], lp[pick], Op.double().cpu().numpy(), "f32", 100, 1.0, sc.truth,
          "grf64")
    Hf = to_dev(states, torch.float32)
    ms_d, ms_l = time_voxel(prob, Hf, iters=3)
    say("ms density", ms_d, "ms likelihood", ms_l)
    assert ms_d > 0 and ms_l > 0


def test_close_after_graph_capture_with_voxel_model(torch_mod, tiny):
    """Destroying a problem that holds both a captured graph and the voxel
    model releases each once (regression: the graph was destroyed twice)."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    states = inputs.init_states(tiny, 4, seed=11)
    for _ in range(3):
        prob = Problem.from_scenario(tiny, precision="f32")
        prob.set_voxel_model(20, 1.0, tiny.truth)
        H = to_dev(states, torch.float32)
        lp = to_dev(np.full(4, np.nan), torch.float64)
        acc = to_dev(np.zeros(4, np.int64), torch.int64)
        prob.mcmc_run(H, lp, acc, 8, 0.05, 5, graph_steps=4)
        torch.cuda.synchronize()
        prob.close()
    assert np.all(np.isfinite(lp.cpu().numpy()))


# ---------------------------------------------------------------------------
# The voxel model's gradient (the reason the paper smooths the density)
# ---------------------------------------------------------------------------

VOX_NZ, VOX_GAMMA = 25, 2.0


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_voxel_gradient_matches_oracle(torch_mod, oracle_mod, tiny, precision):
    """logpost_grad_batch under the voxel model: the back-projection of
    dLL/dO through G's transposed pattern and the sigmoid derivatives, against
    the oracle's chain rule.  float64: relative 1e-9 (L2 per chain); float32:
    relative 1e-4 and every coordinate within 1e-4 max|g|."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    states = np.concatenate([tiny.truth[None], inputs.init_states(tiny, 3, seed=4, jitter=1.0)])
    prob = Problem.from_scenario(tiny, precision=precision)
    prob.set_voxel_model(VOX_NZ, VOX_GAMMA, tiny.truth)
    dt = torch.float64 if precision == "f64" else torch.float32
    lp, g = prob.logpost_grad_batch(to_dev(states, dt))
    torch.cuda.synchronize()
    lp, g = lp.cpu().numpy(), g.double().cpu().numpy()
    orc = oracle_vox(oracle_mod, tiny, VOX_NZ, VOX_GAMMA, tiny.truth)
    st = rounded_states(states, precision)
    for c in range(states.shape[0]):
        lpo, go = orc.grad(st[c])
        rel = np.linalg.norm(g[c] - go) / np.linalg.norm(go)
        worst = np.abs(g[c] - go).max() / np.abs(go).max()
        say(f"voxel grad {precision} chain {c}: relative L2 {rel:.2e}, worst coordinate / max|g| {worst:.2e}")
        assert np.abs(go[2]).max() > 0.0
        if precision == "f64":
            assert rel < 1e-9
            assert lp[c] == pytest.approx(lpo, rel=1e-11, abs=1e-6)
        else:
            assert rel < 1e-4 and worst < 1e-4


VOX_ITEM = 1024   # entries per gradient work item (kVoxItemEntries in voxel.h)


def test_voxel_gradient_long_column_lists(torch_mod, oracle_mod):
    """Columns whose transposed lists run to several work items, with item
    cuts inside a level (two items each add part of that level's sum), and
    more than one 64-chain group: gradient against the oracle, same bars as
    the gradient test above."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    rng = np.random.default_rng(41)
    S, R, C, X, Y, n_pix, n_z, gamma = 3, 8, 8, 40.0, 40.0, 1600, 40, 1.5
    base = 30.0 + 3.0 * rng.standard_normal((R, C))
    free = np.stack([base + 10.0 * l + rng.random((R, C)) for l in range(S - 1)])
    top = 70.0 + rng.random((R, C))
    pos = np.array([[X * 0.45, Y * 0.5, 0.0], [X * 0.6, Y * 0.35, 1.0]])
    th = np.radians(rng.uniform(1, 35, n_pix))
    ph = rng.uniform(0, 2 * np.pi, n_pix)
    d1 = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    sc = make_scenario(S, R, C, X, Y, free, top, (1.8, 0.0, 2.7), pos, np.stack([d1, d1[::-1]]),
                       car_r=np.full(S - 1, 0.7))
    sc.counts = oracle_mod.make_counts(sc, seed=5)
    orc = oracle_vox(oracle_mod, sc, n_z, gamma, free)
    # the lists really are long and cut inside levels
    per_voxel = np.zeros(R * C * n_z, np.int64)
    for r in range(sc.n_rays):
        v, _ = orc.voxel_pieces(r, n_z)
        np.add.at(per_voxel, v, 1)
    toff = np.concatenate([[0], np.cumsum(per_voxel)])
    inside = 0
    for col in range(R * C):
        e0, e1 = toff[col * n_z], toff[(col + 1) * n_z]
        for cut in range(e0 + VOX_ITEM, e1, VOX_ITEM):
            inside += int(cut not in set(toff[col * n_z:(col + 1) * n_z + 1]))
    say(f"longest column list {int(np.diff(toff[::n_z]).max())} entries, {inside} item cuts inside a level")
    assert np.diff(toff[::n_z]).max() > 3 * VOX_ITEM and inside > 0
    n_chains = 70
    states = np.sort(np.stack([free + 0.4 * rng.standard_normal(free.shape) for _ in range(n_chains)]), axis=1)
    for precision in ("f64", "f32"):
        prob = Problem.from_scenario(sc, precision=precision)
        prob.set_voxel_model(n_z, gamma, free)
        dt = torch.float64 if precision == "f64" else torch.float32
        lp, g = prob.logpost_grad_batch(to_dev(states, dt))
        torch.cuda.synchronize()
        lp, g = lp.cpu().numpy(), g.double().cpu().numpy()
        st = rounded_states(states, precision)
        for c in (0, 63, 64, 69):
            lpo, go = orc.grad(st[c])
            rel = np.linalg.norm(g[c] - go) / np.linalg.norm(go)
            worst = np.abs(g[c] - go).max() / np.abs(go).max()
            say(f"long lists {precision} chain {c}: relative L2 {rel:.2e}, worst coordinate / max|g| {worst:.2e}")
            if precision == "f64":
                assert rel < 1e-9
                assert lp[c] == pytest.approx(lpo, rel=1e-11, abs=1e-6)
            else:
                assert rel < 1e-4 and worst < 1e-4


def test_voxel_gradient_zero_where_counts_nonpositive(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.tiny_bumps(seed=0)
    sc.atten_len = 5.0
    sc.counts = tiny.counts
    prob = Problem.from_scenario(sc, precision="f64")
    prob.set_voxel_model(30, 1.0, tiny.truth)
    low = tiny.truth.copy()
    low[1] = low[0] + 0.5
    lp, g = prob.logpost_grad_batch(to_dev(np.stack([tiny.truth, low]), torch.float64))
    torch.cuda.synchronize()
    assert np.isfinite(lp[0].item()) and lp[1].item() == -np.inf
    assert torch.all(g[1] == 0.0) and torch.any(g[0] != 0.0)


def test_voxel_mala_f64_matches_oracle(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import KERNEL_MALA, Problem
    torch = torch_mod
    states = inputs.init_states(tiny, 4, seed=6)
    n_steps, eps, seed = 20, 0.2, 33
    orc = oracle_vox(oracle_mod, tiny, VOX_NZ, VOX_GAMMA, tiny.truth)
    Ho, lpo, acco, marg = orc.mcmc_mala(states, np.full(4, np.nan), np.zeros(4, np.int64), n_steps, 0, eps, seed,
                                        want_margins=True)
    say("voxel mala acceptances", acco, "min margin", np.nanmin(marg))
    assert np.nanmin(marg) > 1e-6, "a near-tie decision; choose another seed"
    assert 0 < acco.sum() < 4 * n_steps
    prob = Problem.from_scenario(tiny, precision="f64")
    prob.set_voxel_model(VOX_NZ, VOX_GAMMA, tiny.truth)
    H = to_dev(states, torch.float64)
    lp = to_dev(np.full(4, np.nan), torch.float64)
    acc = to_dev(np.zeros(4, np.int64), torch.int64)
    prob.mcmc_run(H, lp, acc, n_steps, eps, seed, kernel=KERNEL_MALA, graph_steps=5)
    torch.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), acco)
    np.testing.assert_allclose(H.cpu().numpy(), Ho, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(lp.cpu().numpy(), lpo, rtol=1e-11, atol=1e-6)


@pytest.mark.parametrize("latent", [0, 1])
def test_voxel_nuts_f64_matches_oracle(torch_mod, oracle_mod, tiny, latent):
    """NUTS on the voxel model (heights, or the latent CAR fields as the
    paper's sampler runs): f64 trees equal the oracle's."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    n = 4
    states = inputs.init_states(tiny, n, seed=7)
    orc = oracle_vox(oracle_mod, tiny, VOX_NZ, VOX_GAMMA, tiny.truth)
    prob = Problem.from_scenario(tiny, precision="f64")
    prob.set_voxel_model(VOX_NZ, VOX_GAMMA, tiny.truth)
    if latent:
        x = orc.heights_to_latent(states)
        eps = np.full(n, 0.01)
    else:
        x = states
        eps = np.array([0.01, 0.02, 0.015, 0.01])
    H = to_dev(x, torch.float64)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    e = to_dev(eps, torch.float64)
    st = prob.nuts_run(H, lp, e, n_steps=4, seed=51, max_depth=5, latent=latent)
    torch.cuda.synchronize()
    o = orc.nuts(x, np.full(n, np.nan), eps, max_depth=5, n_steps=4, seed=51, latent=bool(latent))
    say("voxel nuts depths", o["depth"].tolist(), "margins", o["margin"])
    ok = [c for c in range(n) if o["margin"][c] > 1e-7]
    assert len(ok) >= 3
    assert o["n_leap"].sum() > 20
    for c in ok:
        assert np.array_equal(st["tree_depth"].cpu().numpy()[c], o["depth"][c])
        assert np.array_equal(st["n_leapfrog"].cpu().numpy()[c], o["n_leap"][c])
        np.testing.assert_allclose(H.cpu().numpy()[c], o["x"][c], rtol=1e-9, atol=1e-9)
