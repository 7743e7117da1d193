"""GPU parity of the hierarchical sampler: random-walk Metropolis on H with a
Metropolis-within-Gibbs update of every surface's CAR dependence r_l (logit
scale, step tau) after each H decision, against the oracle's sampler.

As for the fixed-r samplers, a chain is compared only while every decision
margin |log U - log alpha| (the H decision and each r decision) is above the
log-posterior error bound."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    return sc


def r_starts(n, S1, seed):
    return np.random.default_rng(seed).uniform(0.15, 0.9, size=(n, S1))


def gpu_run_r(torch, sc, states, r0, precision, n_steps, sigma, tau, seed, offset=0, graph_steps=1, lp=None,
              acc=None, acc_r=None, prob=None):
    from paper_2603_28907_amd.binding import Problem
    prob = prob or Problem.from_scenario(sc, precision=precision)
    dt = torch.float64 if precision == "f64" else torch.float32
    H = to_dev(states, dt)
    n = H.shape[0]
    r = to_dev(r0, torch.float64)
    lpt = to_dev(np.full(n, np.nan) if lp is None else lp, torch.float64)
    acct = to_dev(np.zeros(n, np.int64) if acc is None else acc, torch.int64)
    accr = to_dev(np.zeros(r0.shape, np.int64) if acc_r is None else acc_r, torch.int64)
    prob.mcmc_run(H, lpt, acct, n_steps, sigma, seed, step_offset=offset, graph_steps=graph_steps,
                  r_state=r, r_step=tau, n_accept_r=accr)
    torch.cuda.synchronize()
    return (H.double().cpu().numpy(), r.cpu().numpy(), lpt.cpu().numpy(), acct.cpu().numpy(),
            accr.cpu().numpy())


def test_entry_logpost_uses_each_chains_r(torch_mod, oracle_mod, tiny):
    """n_steps = 0: the entry pass alone, log p(H | r_c) + log L for every chain,
    including one outside the support (-inf)."""
    orc = oracle_mod.OracleProblem(tiny)
    states = inputs.init_states(tiny, 5, seed=21)
    states[4, 1] = states[4, 0] - 1.0   # crossed surfaces: outside the support
    r0 = r_starts(5, tiny.n_surfaces - 1, 22)
    _, r1, lp, acc, accr = gpu_run_r(torch_mod, tiny, states, r0, "f64", 0, 0.05, 0.5, 1, lp=np.zeros(5))
    assert np.array_equal(r1, r0) and not acc.any() and not accr.any()
    ref = []
    for c in range(5):
        pr = orc.log_prior_r(states[c], r0[c])
        # log L = logpost - log prior at the problem's fixed r
        ref.append(pr + (orc.logpost(states[c]) - orc.log_prior(states[c]) if np.isfinite(pr) else 0.0))
    say("entry lp", lp, "oracle", ref)
    assert lp[4] == -np.inf and ref[4] == -np.inf
    np.testing.assert_allclose(lp[:4], ref[:4], rtol=1e-12, atol=1e-8)
    # r enters: the same states at the problem's fixed r give another value
    lp_fixed = orc.logpost_batch(states[:4])
    assert np.all(np.abs(lp_fixed - lp[:4]) > 1e-3)


def test_hier_f64_matches_oracle(torch_mod, oracle_mod, tiny):
    n, n_steps, sigma, tau, seed = 4, 100, 0.05, 0.7, 4242
    states = inputs.init_states(tiny, n, seed=2)
    r0 = r_starts(n, tiny.n_surfaces - 1, 3)
    say("hier f64: GPU run")
    Hg, rg, lpg, accg, accrg = gpu_run_r(torch_mod, tiny, states, r0, "f64", n_steps, sigma, tau, seed,
                                         graph_steps=10)
    orc = oracle_mod.OracleProblem(tiny)
    Ho, ro, lpo, acco, accro, marg = orc.mcmc_rw_r(states, r0, np.full(n, np.nan), np.zeros(n, np.int64), n_steps,
                                                   0, sigma, tau, seed, want_margins=True)
    say("min margin", np.nanmin(marg), "H accepts", acco, "r accepts", accro.tolist())
    assert np.nanmin(marg) > 1e-6, "a near-tie decision; choose another seed"
    assert 0 < acco.sum() < n * n_steps and 0 < accro.sum() < n * n_steps * (tiny.n_surfaces - 1)
    assert np.array_equal(accg, acco) and np.array_equal(accrg, accro)
    np.testing.assert_allclose(Hg, Ho, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(rg, ro, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(lpg, lpo, rtol=1e-11, atol=1e-6)


def test_hier_chain_outside_support_moves_r_under_its_prior(torch_mod, oracle_mod, tiny):
    """A chain whose H lies outside the support keeps lp = -inf and rejects
    every H proposal that stays outside; its r moves exactly as the oracle's."""
    n, n_steps, sigma, tau, seed = 2, 40, 1e-3, 1.0, 77
    states = inputs.init_states(tiny, n, seed=8)
    states[1, 1] = states[1, 0] - 5.0
    r0 = r_starts(n, tiny.n_surfaces - 1, 9)
    Hg, rg, lpg, accg, accrg = gpu_run_r(torch_mod, tiny, states, r0, "f64", n_steps, sigma, tau, seed)
    orc = oracle_mod.OracleProblem(tiny)
    Ho, ro, lpo, acco, accro, marg = orc.mcmc_rw_r(states, r0, np.full(n, np.nan), np.zeros(n, np.int64), n_steps,
                                                   0, sigma, tau, seed, want_margins=True)
    assert np.nanmin(marg[1, :, 1:]) > 1e-9
    assert lpo[1] == -np.inf and lpg[1] == -np.inf and acco[1] == 0 and accg[1] == 0
    assert np.array_equal(accrg[1], accro[1]) and accro[1].sum() > 0
    np.testing.assert_allclose(rg[1], ro[1], rtol=1e-12, atol=1e-14)
    assert np.array_equal(Hg[1], states[1])


def test_hier_graph_eager_and_resume_are_bitwise(torch_mod, tiny):
    states = inputs.init_states(tiny, 6, seed=3)
    r0 = r_starts(6, tiny.n_surfaces - 1, 4)
    a = gpu_run_r(torch_mod, tiny, states, r0, "f32", 40, 0.05, 0.6, 7, graph_steps=8)
    b = gpu_run_r(torch_mod, tiny, states, r0, "f32", 40, 0.05, 0.6, 7, graph_steps=1)
    h1, r1, lp1, acc1, accr1 = gpu_run_r(torch_mod, tiny, states, r0, "f32", 25, 0.05, 0.6, 7, graph_steps=5)
    c = gpu_run_r(torch_mod, tiny, h1, r1, "f32", 15, 0.05, 0.6, 7, offset=25, graph_steps=5, lp=lp1, acc=acc1,
                  acc_r=accr1)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)
    assert a[4].sum() > 0


def test_hier_request_errors(torch_mod, tiny):
    from paper_2603_28907_amd.binding import KERNEL_MALA, MuonCaveError, Problem
    torch = torch_mod
    prob = Problem.from_scenario(tiny, precision="f32")
    n, S1 = 2, tiny.n_surfaces - 1
    H = to_dev(inputs.init_states(tiny, n, seed=1), torch.float32)
    lp = to_dev(np.full(n, np.nan), torch.float64)
    acc = to_dev(np.zeros(n, np.int64), torch.int64)
    r = to_dev(np.full((n, S1), 0.5), torch.float64)
    accr = to_dev(np.zeros((n, S1), np.int64), torch.int64)
    with pytest.raises(MuonCaveError, match="random-walk"):
        prob.mcmc_run(H, lp, acc, 2, 0.01, 1, kernel=KERNEL_MALA, r_state=r, r_step=0.5)
    with pytest.raises(MuonCaveError, match="r_step"):
        prob.mcmc_run(H, lp, acc, 2, 0.01, 1, r_state=r, r_step=-1.0)
    with pytest.raises(MuonCaveError, match="n_accept_r"):
        prob.mcmc_run(H, lp, acc, 2, 0.01, 1, n_accept_r=accr)
    # the same problem still samples at fixed r afterwards
    prob.mcmc_run(H, lp, acc, 2, 0.01, 1)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(lp.cpu().numpy()))
