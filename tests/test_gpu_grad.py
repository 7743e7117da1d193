"""GPU parity of the hand-written adjoint (gradient of the log posterior with
respect to every surface height) and of the MALA sampler that uses it.

Tolerances: float64, relative 1e-9 in the L2 norm per chain.  float32:
every coordinate within its own conditioning bound (tests.gpu_common.
f32_gradient_tolerance: a crossing contributes w_n/|f'|, so float32 rounding
of z - h moves it by eps_z/|f'| and its weight by about eps_z/f'^2; pairs
near tangency may vanish; dLL/dO carries the ray's measured opacity error),
with no coordinate exempt, and relative 1e-4 (small cave) or 1e-3 (128x128)
in the L2 norm per chain.  Central differences of float64 log posteriors
(h = 1e-3 m, 64 seeded coordinates, kinks of the piecewise-smooth lp
detected and skipped) on the small cave and on the 128x128 geometry."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import f32_gradient_tolerance, require_gpu, rounded_states, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    return sc


def gpu_grad(torch, sc, states, precision):
    from paper_2603_28907_amd.binding import Problem
    prob = Problem.from_scenario(sc, precision=precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    H = to_dev(states, dt)
    lp, g = prob.logpost_grad_batch(H)
    torch.cuda.synchronize()
    return lp.cpu().numpy(), g.double().cpu().numpy(), prob


def gpu_opacities(torch, prob, states):
    """The float32 forward opacities of `states` (the ones the gradient uses:
    the march is the same kernel, and a chain's results do not depend on the
    batch)."""
    H = to_dev(states, torch.float32)
    O = torch.empty((states.shape[0], prob.n_rays), dtype=torch.float32, device="cuda:0")
    prob.logpost_batch(H, opacity=O)
    torch.cuda.synchronize()
    return O.double().cpu().numpy()


def check_f32_gradient(orc, state, g_gpu, g_ref, O_gpu, label):
    """Every coordinate within its conditioning bound."""
    _, gpr = orc.log_prior_grad(state)
    dO = O_gpu - orc.opacity(state)
    tol = f32_gradient_tolerance(orc, state, dO, gpr)
    err = np.abs(g_gpu - g_ref)
    ratio = err / tol
    k = np.unravel_index(np.argmax(ratio), ratio.shape)
    say(f"{label}: worst error / bound {ratio[k]:.3f} at node {k} (error {err[k]:.3g}, bound {tol[k]:.3g}); "
        f"median bound / max|g| {np.median(tol) / np.abs(g_ref).max():.2e}")
    assert np.all(err <= tol), (label, k, g_gpu[k], g_ref[k], tol[k])
    return tol


def test_prior_gradient_without_sensors(torch_mod, oracle_mod):
    from tests.helpers import make_scenario
    sc = inputs.tiny_bumps(seed=3)
    sc0 = make_scenario(3, sc.n_rows, sc.n_cols, sc.extent_x, sc.extent_y, sc.truth, sc.top, sc.density,
                        np.zeros((0, 3)), None, car_r=sc.car_r)
    states = inputs.init_states(sc, 2, seed=1)
    lp, g, _ = gpu_grad(torch_mod, sc0, states, "f64")
    orc = oracle_mod.OracleProblem(sc0)
    for c in range(2):
        v, go = orc.log_prior_grad(states[c])
        for l in range(3):
            say(f"prior grad surface {l}: rel {np.linalg.norm(g[c, l] - go[l]) / np.linalg.norm(go[l]):.2e}")
        assert lp[c] == pytest.approx(v, rel=1e-11)
        np.testing.assert_allclose(g[c], go, rtol=1e-9, atol=1e-9 * np.abs(go).max())


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gradient_matches_oracle(torch_mod, oracle_mod, tiny, precision):
    states = np.concatenate([tiny.truth[None], inputs.init_states(tiny, 3, seed=2)])
    lp, g, prob = gpu_grad(torch_mod, tiny, states, precision)
    st = rounded_states(states, precision)
    orc = oracle_mod.OracleProblem(tiny)
    lpo, go = orc.grad_batch(st)
    for c in range(states.shape[0]):
        rel = np.linalg.norm(g[c] - go[c]) / np.linalg.norm(go[c])
        say(f"grad {precision} chain {c}: relative L2 error {rel:.2e}; lp {lp[c]:.9f} vs {lpo[c]:.9f}")
        _, gpr = orc.log_prior_grad(st[c])
        for l in range(3):
            gl, ol = g[c, l] - gpr[l], go[c, l] - gpr[l]
            ratio = float(np.dot(gl.ravel(), ol.ravel()) / max(np.dot(ol.ravel(), ol.ravel()), 1e-300))
            say(f"  surface {l}: likelihood-part rel {np.linalg.norm(gl - ol) / np.linalg.norm(ol):.2e}, "
                f"projection ratio {ratio:.4f}")
        if precision == "f64":
            assert rel < 1e-9
            assert lp[c] == pytest.approx(lpo[c], rel=1e-11, abs=1e-6)
        else:
            assert rel < 1e-4
            O = gpu_opacities(torch_mod, prob, st[c:c + 1])[0]
            check_f32_gradient(orc, st[c], g[c], go[c], O, f"grad f32 chain {c}")


def test_gradient_finite_differences_on_gpu(torch_mod, tiny):
    """Central differences of the GPU's own float64 log posterior (h = 1e-3 m)
    on 64 seeded coordinates, skipping kinks of the piecewise-smooth lp."""
    from paper_2603_28907_amd.binding import Problem
    prob = Problem.from_scenario(tiny, precision="f64")
    x0 = inputs.init_states(tiny, 1, seed=3)
    lp, g = prob.logpost_grad_batch(to_dev(x0, torch_mod.float64))
    g = g.cpu().numpy()[0]
    rng = np.random.default_rng(9)
    idx = [np.unravel_index(k, x0.shape[1:]) for k in rng.choice(x0[0].size, 64, replace=False)]
    h = 1e-3
    batch = [x0[0]]
    for i in idx:
        xp, xm = x0[0].copy(), x0[0].copy()
        xp[i] += h
        xm[i] -= h
        batch += [xp, xm]
    lps = prob.logpost_batch(to_dev(np.stack(batch), torch_mod.float64)).cpu().numpy()
    scale = np.abs(g).max()
    kinks = 0
    for k, i in enumerate(idx):
        f0, fp, fm = lps[0], lps[1 + 2 * k], lps[2 + 2 * k]
        fwd, bwd = (fp - f0) / h, (f0 - fm) / h
        tol = 1e-4 * scale + 1e-3
        if abs(fwd - bwd) > 10 * tol + 1e-2 * abs(fwd + bwd):
            kinks += 1
            continue
        assert abs((fp - fm) / (2 * h) - g[i]) <= tol, (i, (fp - fm) / (2 * h), g[i])
    assert kinks <= 8


def test_gradient_paper_scale_128(torch_mod, oracle_mod):
    """128x128 grid, 8 sensors x 64x64 pixels, 512 chains on the GPU; two
    sampled chains against the oracle gradient."""
    sc = inputs.grf_cave(seed=10, n_grid=128)
    sc.counts = oracle_mod.make_counts(sc, seed=11)
    states = inputs.init_states(sc, 512, seed=12)
    say("gradient at 128x128 x 512 chains")
    lp, g, prob = gpu_grad(torch_mod, sc, states, "f32")
    assert np.all(np.isfinite(lp)) and np.all(np.isfinite(g))
    st = rounded_states(states, "f32")
    orc = oracle_mod.OracleProblem(sc)
    O = gpu_opacities(torch_mod, prob, st[[0, 511]])
    tol0 = None
    for k_c, c in enumerate((0, 511)):
        lpo, go = orc.grad(st[c])
        rel = np.linalg.norm(g[c] - go) / np.linalg.norm(go)
        say(f"128x128 chain {c}: relative L2 error {rel:.2e}")
        for l in range(3):
            e = np.abs(g[c, l] - go[l])
            k = np.unravel_index(np.argmax(e), e.shape)
            say(f"  surface {l}: rel {np.linalg.norm(g[c, l] - go[l]) / np.linalg.norm(go[l]):.2e}, worst node {k} "
                f"gpu {g[c, l][k]:.6g} oracle {go[l][k]:.6g}")
        assert rel < 1e-3
        tol = check_f32_gradient(orc, st[c], g[c], go, O[k_c], f"128x128 chain {c}")
        if c == 0:
            tol0, scale = tol, np.abs(go).max()
    # central differences of the oracle's float64 log posterior (h = 1e-3 m)
    # on 64 seeded coordinates of all three surfaces, against the GPU's
    # float32 gradient of chain 0
    from tests.helpers import central_differences, is_kink
    fd = central_differences(oracle_mod, sc, st[0], 64, 1e-3, seed=13)
    kinks = 0
    for (l, i, j, fwd, bwd, cd) in fd:
        t_fd = 1e-4 * scale + 1e-3
        if is_kink(fwd, bwd, t_fd):
            kinks += 1
            continue
        assert abs(cd - g[0, l, i, j]) <= t_fd + tol0[l, i, j], (l, i, j, cd, g[0, l, i, j])
    say(f"128x128 finite differences: {len(fd) - kinks} coordinates compared, {kinks} kinks")
    assert kinks <= 8


def test_gradient_repeat_bitwise_and_out_of_support(torch_mod, tiny):
    states = inputs.init_states(tiny, 3, seed=4)
    states[2, 0, 2, 2] = states[2, 1, 2, 2] + 1.0
    lp1, g1, _ = gpu_grad(torch_mod, tiny, states, "f32")
    lp2, g2, _ = gpu_grad(torch_mod, tiny, states, "f32")
    assert np.array_equal(g1, g2) and np.array_equal(lp1, lp2)
    assert lp1[2] == -np.inf and np.all(g1[2] == 0.0)


def test_autograd_function(torch_mod, tiny):
    from paper_2603_28907_amd.autograd import log_posterior
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    prob = Problem.from_scenario(tiny, precision="f64")
    H = to_dev(inputs.init_states(tiny, 2, seed=5), torch.float64).requires_grad_(True)
    lp = log_posterior(H, prob)
    w = torch.tensor([1.0, -2.0], dtype=torch.float64, device="cuda:0")
    (lp * w).sum().backward()
    lp2, g = prob.logpost_grad_batch(H.detach())
    expect = g[:, :2] * w.view(-1, 1, 1, 1)
    assert torch.equal(lp.detach(), lp2)
    assert torch.allclose(H.grad, expect, rtol=0, atol=0)


def test_mala_f64_matches_oracle(torch_mod, oracle_mod, tiny):
    from paper_2603_28907_amd.binding import KERNEL_MALA, Problem
    states = inputs.init_states(tiny, 4, seed=6)
    n_steps, eps, seed = 25, 0.15, 31
    orc = oracle_mod.OracleProblem(tiny)
    Ho, lpo, acco, marg = orc.mcmc_mala(states, np.full(4, np.nan), np.zeros(4, np.int64), n_steps, 0, eps, seed,
                                        want_margins=True)
    say("mala acceptances", acco, "min margin", np.nanmin(marg))
    assert np.nanmin(marg) > 1e-6, "a near-tie decision; choose another seed"
    assert 0 < acco.sum() < 4 * n_steps
    prob = Problem.from_scenario(tiny, precision="f64")
    H = to_dev(states, torch_mod.float64)
    lp = to_dev(np.full(4, np.nan), torch_mod.float64)
    acc = to_dev(np.zeros(4, np.int64), torch_mod.int64)
    prob.mcmc_run(H, lp, acc, n_steps, eps, seed, kernel=KERNEL_MALA, graph_steps=5)
    torch_mod.cuda.synchronize()
    assert np.array_equal(acc.cpu().numpy(), acco)
    np.testing.assert_allclose(H.cpu().numpy(), Ho, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(lp.cpu().numpy(), lpo, rtol=1e-11, atol=1e-6)


def test_adjoint_paths_agree_bitwise(torch_mod, oracle_mod):
    """float32: the record adjoint (one window of node rows, or several) and
    the re-walk of the rays (every chain, with one or several windows; or
    only the chains whose record slots overflow) give the same gradient bit
    for bit: they add the same fixed-point contributions, computed from the
    same walk.  The gradient also meets the oracle within its conditioning
    bound."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.grf_cave(seed=14, n_grid=32, n_sensors=4, pix_side=32)
    sc.counts = oracle_mod.make_counts(sc, seed=15)
    states = inputs.init_states(sc, 24, seed=16)
    prob = Problem.from_scenario(sc, precision="f32")
    base = prob.get_tuning()
    H = to_dev(states, torch.float32)
    lp0, g0 = prob.logpost_grad_batch(H)
    torch.cuda.synchronize()
    variants = [dict(adjoint_rows=5), dict(adjoint_rows=1), dict(grad_slots=-1), dict(grad_slots=-1, adjoint_rows=7),
                dict(grad_slots=1), dict(grad_slots=6), dict(grad_slots=9), dict(grad_slots=12, adjoint_rows=3)]
    for v in variants:
        t = dict(base)
        t.update(v)
        prob.set_tuning(**t)
        lp, g = prob.logpost_grad_batch(H)
        torch.cuda.synchronize()
        say(f"adjoint variant {v}: bitwise {torch.equal(g, g0)}")
        assert torch.equal(lp, lp0) and torch.equal(g, g0), v
    prob.set_tuning(**base)
    st = rounded_states(states, "f32")
    orc = oracle_mod.OracleProblem(sc)
    O = gpu_opacities(torch, prob, st[:2])
    gn = g0.double().cpu().numpy()
    for c in range(2):
        _, go = orc.grad(st[c])
        check_f32_gradient(orc, st[c], gn[c], go, O[c], f"32x32 chain {c}")


def test_gradient_equal_across_launch_shapes(torch_mod, oracle_mod):
    """float32: the gradient march and its record adjoint at every block size
    (256, 512 and 1024 threads, 8 or 16 rays per thread) give the same
    gradient bit for bit: each ray's walk does not depend on the launch
    shape, and the contributions are summed in fixed point.  Checks the
    records written by every instance of the gradient march, including the
    register-bound 512-thread one."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.grf_cave(seed=14, n_grid=32, n_sensors=4, pix_side=32)
    sc.counts = oracle_mod.make_counts(sc, seed=15)
    states = inputs.init_states(sc, 24, seed=17)
    prob = Problem.from_scenario(sc, precision="f32")
    H = to_dev(states, torch.float32)
    ref = None
    for block, rpt in [(256, 8), (512, 16), (1024, 16), (512, 8), (256, 16)]:
        prob.set_tuning(march_variant=4, block=block, rays_per_thread=rpt, top_in_lds=0)
        _, g = prob.logpost_grad_batch(H)
        torch.cuda.synchronize()
        if ref is None:
            ref = g.clone()
        say(f"gradient at block {block} x {rpt}: bitwise {torch.equal(g, ref)}")
        assert torch.equal(g, ref), (block, rpt)


@pytest.mark.gpu
def test_gradient_autotune_keeps_the_gradient(torch_mod, oracle_mod):
    """The gradient tuner times every candidate shape, leaves the fastest one
    set, and the gradient at that shape equals the one at the default shape
    bit for bit (launch shape changes performance only)."""
    from paper_2603_28907_amd import autotune
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.grf_cave(seed=14, n_grid=32, n_sensors=4, pix_side=32)
    sc.counts = oracle_mod.make_counts(sc, seed=15)
    prob = Problem.from_scenario(sc, precision="f32")
    H = to_dev(inputs.init_states(sc, 24, seed=17), torch.float32)
    _, g0 = prob.logpost_grad_batch(H)
    torch.cuda.synchronize()
    res = autotune.tune_gradient(prob, H, iters=2)
    shapes = [(t["block"], t["rays_per_thread"]) for t, _ in res["trials"]]
    say(f"trials {[(b, r, round(ms, 4)) for (b, r), (_, ms) in zip(shapes, res['trials'])]}")
    assert len(res["trials"]) == len(autotune.GRAD_SHAPES)
    assert all(ms > 0 for _, ms in res["trials"])
    best = min(res["trials"], key=lambda x: x[1])[0]
    t = prob.get_tuning()
    assert (t["block"], t["rays_per_thread"]) == (best["block"], best["rays_per_thread"])
    _, g1 = prob.logpost_grad_batch(H)
    torch.cuda.synchronize()
    assert torch.equal(g0, g1)
