"""Many heterogeneous problems in shared launches (mcmc_run_multi).

Each chain runs the same device code as in a single-problem mcmc_run with the
default launch shape, so states, log posteriors and acceptance counts must be
bit-identical to running every problem on its own."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


def _batch(oracle_mod, ids, max_chains=16, scale_pixels=0.25, with_empty=False):
    out = []
    for i in ids:
        sc, n = inputs.heterogeneous_problem(i, scale_pixels=scale_pixels)
        sc.counts = oracle_mod.make_counts(sc, seed=100 + i)
        out.append((sc, min(n, max_chains), 0.02 + 0.005 * (i % 4), 1000 + i))
    if with_empty:
        from tests.helpers import make_scenario
        t = inputs.tiny_bumps(seed=2)
        sc0 = make_scenario(3, t.n_rows, t.n_cols, t.extent_x, t.extent_y, t.truth, t.top, t.density,
                            np.zeros((0, 3)), None, car_r=t.car_r)
        out.append((sc0, 8, 0.05, 77))
    return out


def _states(torch, batch, dtype):
    H, lp, acc = [], [], []
    for k, (sc, n, _, _) in enumerate(batch):
        H.append(to_dev(inputs.init_states(sc, n, seed=500 + k), dtype))
        lp.append(to_dev(np.full(n, np.nan), torch.float64))
        acc.append(to_dev(np.zeros(n, np.int64), torch.int64))
    return H, lp, acc


def _clone(ts):
    return [t.clone() for t in ts]


@pytest.mark.parametrize("precision,ids", [("f32", [0, 1, 2, 3, 4, 5]), ("f64", [1, 3, 4, 5])])
def test_multi_equals_single(torch_mod, oracle_mod, precision, ids):
    from paper_2603_28907_amd.binding import Problem, mcmc_run_multi
    torch = torch_mod
    batch = _batch(oracle_mod, ids, with_empty=True)
    probs = [Problem.from_scenario(sc, precision=precision) for sc, _, _, _ in batch]
    dt = probs[0].torch_dtype
    H, lp, acc = _states(torch, batch, dt)
    H1, lp1, acc1 = _clone(H), _clone(lp), _clone(acc)
    n_steps, G = 12, 5
    for k, (pr, (sc, n, sig, seed)) in enumerate(zip(probs, batch)):
        say(f"single {precision} problem {k}: grid {sc.n_rows}, rays {pr.n_rays}, chains {n}")
        pr.mcmc_run(H1[k], lp1[k], acc1[k], n_steps, sig, seed, graph_steps=G)
    torch.cuda.synchronize()
    say(f"multi {precision}: {len(probs)} problems")
    mcmc_run_multi(probs, H, lp, acc, n_steps, [b[2] for b in batch], [b[3] for b in batch], graph_steps=G)
    torch.cuda.synchronize()
    tot = 0
    for k in range(len(probs)):
        assert torch.equal(H[k], H1[k]), k
        assert torch.equal(lp[k], lp1[k]), k
        assert torch.equal(acc[k], acc1[k]), k
        tot += int(acc[k].sum())
    say("accepted", tot)
    assert tot > 0


def test_multi_resume_and_plan_reuse(torch_mod, oracle_mod):
    """7 + 5 steps (second call resumes at step 7 and reuses the cached plan)
    equal 12 steps in one call, and a repeated call is deterministic."""
    from paper_2603_28907_amd.binding import Problem, mcmc_run_multi
    torch = torch_mod
    batch = _batch(oracle_mod, [3, 4, 5])
    probs = [Problem.from_scenario(sc, precision="f32") for sc, _, _, _ in batch]
    H, lp, acc = _states(torch, batch, torch.float32)
    H1, lp1, acc1 = _clone(H), _clone(lp), _clone(acc)
    sig, seeds = [b[2] for b in batch], [b[3] for b in batch]
    mcmc_run_multi(probs, H1, lp1, acc1, 12, sig, seeds, graph_steps=4)
    mcmc_run_multi(probs, H, lp, acc, 7, sig, seeds, graph_steps=4)
    mcmc_run_multi(probs, H, lp, acc, 5, sig, seeds, step_offsets=[7, 7, 7], graph_steps=4)
    torch.cuda.synchronize()
    for k in range(len(probs)):
        assert torch.equal(H[k], H1[k]) and torch.equal(lp[k], lp1[k]) and torch.equal(acc[k], acc1[k])


def test_multi_persistent_grid(torch_mod, oracle_mod):
    """A persistent march grid (2 blocks per compute unit) gives the same bits
    as one block per work item."""
    from paper_2603_28907_amd.binding import Problem, mcmc_run_multi
    torch = torch_mod
    batch = _batch(oracle_mod, [0, 3, 5], max_chains=32)
    probs = [Problem.from_scenario(sc, precision="f32") for sc, _, _, _ in batch]
    H, lp, acc = _states(torch, batch, torch.float32)
    H1, lp1, acc1 = _clone(H), _clone(lp), _clone(acc)
    sig, seeds = [b[2] for b in batch], [b[3] for b in batch]
    mcmc_run_multi(probs, H1, lp1, acc1, 6, sig, seeds, graph_steps=3)
    t = probs[0].get_tuning()
    t["multi_blocks_per_cu"] = 2
    probs[0].set_tuning(**t)
    mcmc_run_multi(probs, H, lp, acc, 6, sig, seeds, graph_steps=3)
    torch.cuda.synchronize()
    for k in range(len(probs)):
        assert torch.equal(H[k], H1[k]) and torch.equal(lp[k], lp1[k]) and torch.equal(acc[k], acc1[k])


def test_multi_argument_errors(torch_mod, oracle_mod):
    from paper_2603_28907_amd.binding import MuonCaveError, Problem, mcmc_run_multi
    torch = torch_mod
    batch = _batch(oracle_mod, [3, 4])
    p32 = Problem.from_scenario(batch[0][0], precision="f32")
    p64 = Problem.from_scenario(batch[1][0], precision="f64")
    Ha = to_dev(inputs.init_states(batch[0][0], 2, seed=1), torch.float32)
    Hb = to_dev(inputs.init_states(batch[1][0], 2, seed=1), torch.float64)
    lp = [to_dev(np.full(2, np.nan), torch.float64) for _ in range(2)]
    acc = [to_dev(np.zeros(2, np.int64), torch.int64) for _ in range(2)]
    with pytest.raises(MuonCaveError, match="precision"):
        mcmc_run_multi([p32, p64], [Ha, Hb], lp, acc, 2, [0.1, 0.1], [1, 2])
    with pytest.raises(MuonCaveError, match="repeats"):
        mcmc_run_multi([p32, p32], [Ha, Ha.clone()], lp, acc, 2, [0.1, 0.1], [1, 2])


def test_autotune_per_class(torch_mod, oracle_mod, tmp_path):
    """The tuner picks one launch shape per grid class, applies it to every
    problem of the class, caches it on disk, and leaves the log posterior
    unchanged up to float32 rounding."""
    from paper_2603_28907_amd import autotune
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    batch = _batch(oracle_mod, [0, 3, 5, 10], max_chains=8)   # grids 128, 16, 64, 16
    probs = [Problem.from_scenario(sc, precision="f32") for sc, _, _, _ in batch]
    H, _, _ = _states(torch, batch, torch.float32)
    before = [p.logpost_batch(h).cpu().numpy() for p, h in zip(probs, H)]
    cache = str(tmp_path / "tune.json")
    autotune._memo.clear()
    res = autotune.tune_batch(probs, H, cache_path=cache, iters=2)
    say("tuned", res)
    assert len(res) == 3
    for p in probs:
        t = res[autotune.class_key(p, torch.cuda.get_device_name(0))]
        got = p.get_tuning()
        assert all(got[k] == t[k] for k in ("march_variant", "block", "rays_per_thread"))
    after = [p.logpost_batch(h).cpu().numpy() for p, h in zip(probs, H)]
    for a, b in zip(before, after):
        np.testing.assert_allclose(b, a, rtol=1e-6)
    autotune._memo.clear()
    again = autotune.tune_batch(probs, H, cache_path=cache, iters=2)
    assert again == res


@pytest.mark.parametrize("precision,ids", [("f32", [0, 2, 3, 5]), ("f64", [1, 4])])
def test_multi_with_sampled_r_equals_single(torch_mod, oracle_mod, precision, ids):
    """Every chain's r sampled too (logit-scale Metropolis-within-Gibbs after
    each H decision): each problem in the shared launches gives the states,
    r values, log posteriors and acceptance counts of mcmc_run on its own,
    bit for bit, across a resumed second call."""
    from paper_2603_28907_amd.binding import Problem, mcmc_run_multi
    torch = torch_mod
    batch = _batch(oracle_mod, ids)
    probs = [Problem.from_scenario(sc, precision=precision) for sc, _, _, _ in batch]
    dt = probs[0].torch_dtype
    H, lp, acc = _states(torch, batch, dt)
    H1, lp1, acc1 = _clone(H), _clone(lp), _clone(acc)
    rng = np.random.default_rng(9)
    r = [to_dev(rng.uniform(0.3, 0.95, size=(n, sc.n_surfaces - 1)), torch.float64) for sc, n, _, _ in batch]
    ar = [torch.zeros((n, sc.n_surfaces - 1), dtype=torch.int64, device="cuda:0") for sc, n, _, _ in batch]
    r1, ar1 = _clone(r), _clone(ar)
    tau, G = 0.4, 4
    for k, (pr, (sc, n, sig, seed)) in enumerate(zip(probs, batch)):
        pr.mcmc_run(H1[k], lp1[k], acc1[k], 8, sig, seed, graph_steps=G, r_state=r1[k], r_step=tau,
                    n_accept_r=ar1[k])
        pr.mcmc_run(H1[k], lp1[k], acc1[k], 5, sig, seed, step_offset=8, graph_steps=G, r_state=r1[k], r_step=tau,
                    n_accept_r=ar1[k])
    sig, seeds = [b[2] for b in batch], [b[3] for b in batch]
    mcmc_run_multi(probs, H, lp, acc, 8, sig, seeds, graph_steps=G, r_states=r, r_step=tau, n_accept_r=ar)
    mcmc_run_multi(probs, H, lp, acc, 5, sig, seeds, step_offsets=[8] * len(probs), graph_steps=G, r_states=r,
                   r_step=tau, n_accept_r=ar)
    torch.cuda.synchronize()
    moved = 0
    for k in range(len(probs)):
        assert torch.equal(H[k], H1[k]) and torch.equal(lp[k], lp1[k]) and torch.equal(acc[k], acc1[k]), k
        assert torch.equal(r[k], r1[k]) and torch.equal(ar[k], ar1[k]), k
        moved += int(ar[k].sum())
    say("r accepted", moved)
    assert moved > 0
    with pytest.raises(Exception, match="every problem or for none"):
        mcmc_run_multi(probs, H, lp, acc, 2, sig, seeds, r_states=[r[0]] + [None] * (len(probs) - 1), r_step=tau)
