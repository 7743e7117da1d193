"""The allocation-free entry point, logpost_batch_noalloc, against
logpost_batch (the same kernels, so results must be equal bit for bit) and
the FP64 oracle, on two calls in a row with the second call smaller; plus
its refusal of a request beyond its fixed workspace."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, rounded_states, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    return sc


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_equals_logpost_batch(torch_mod, oracle_mod, tiny, precision):
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    dt = torch.float64 if precision == "f64" else torch.float32
    prob = Problem.from_scenario(tiny, precision=precision)
    orc = oracle_mod.OracleProblem(tiny)
    states = inputs.init_states(tiny, 8, seed=31)
    for n in (8, 3):   # the second call is smaller and follows the first
        say(f"noalloc {precision} n={n}")
        H = to_dev(states[:n], dt)
        O_ref = torch.empty((n, tiny.n_rays), dtype=dt, device="cuda:0")
        lp_ref = prob.logpost_batch(H, opacity=O_ref)
        O = torch.full((n, tiny.n_rays), float("nan"), dtype=dt, device="cuda:0")
        lp = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        prob.logpost_batch_noalloc(H, lp, opacity=O)
        torch.cuda.synchronize()
        assert torch.equal(lp, lp_ref), (lp, lp_ref)
        assert torch.equal(O, O_ref)
        lp_orc = orc.logpost_batch(rounded_states(states[:n], precision))
        if precision == "f64":
            assert np.allclose(lp.cpu().numpy(), lp_orc, rtol=1e-11, atol=1e-6)
        else:
            assert np.all(np.abs(lp.cpu().numpy() - lp_orc) < 1.0)
    # without the opacity output
    lp2 = torch.empty((3,), dtype=torch.float64, device="cuda:0")
    prob.logpost_batch_noalloc(to_dev(states[:3], dt), lp2)
    torch.cuda.synchronize()
    assert torch.equal(lp2, lp)


def test_noalloc_paper_scale_grid(torch_mod, oracle_mod):
    """A 64x64 grid with 8 sensors of 32x32 pixels, in the production float32
    launch shape, against logpost_batch (bitwise) and the oracle on two
    sampled chains."""
    from paper_2603_28907_amd.binding import Problem
    torch = torch_mod
    sc = inputs.grf_cave(seed=10, n_grid=64, n_sensors=8, pix_side=32)
    sc.counts = oracle_mod.make_counts(sc, seed=11)
    prob = Problem.from_scenario(sc, precision="f32")
    states = inputs.init_states(sc, 64, seed=12)
    for n in (64, 17):
        say(f"noalloc grf64 n={n}")
        H = to_dev(states[:n], torch.float32)
        lp_ref = prob.logpost_batch(H)
        lp = torch.empty((n,), dtype=torch.float64, device="cuda:0")
        prob.logpost_batch_noalloc(H, lp)
        torch.cuda.synchronize()
        assert torch.equal(lp, lp_ref)
    orc = oracle_mod.OracleProblem(sc)
    st = rounded_states(states[:2], "f32")
    lp_orc = orc.logpost_batch(st)
    assert np.all(np.abs(lp[:2].cpu().numpy() - lp_orc) < 5.0), (lp[:2], lp_orc)


def test_noalloc_rejects_requests_beyond_its_workspace(torch_mod, tiny):
    from paper_2603_28907_amd.binding import MuonCaveError, Problem
    torch = torch_mod
    prob = Problem.from_scenario(tiny, precision="f32")
    prob.set_tuning(march_variant=4, block=256, rays_per_thread=1, top_in_lds=0)
    tiles = -(-tiny.n_rays // 256)
    n = 131072 // tiles + 1
    H = torch.zeros((n, tiny.n_surfaces - 1, tiny.n_rows, tiny.n_cols), dtype=torch.float32, device="cuda:0")
    lp = torch.empty((n,), dtype=torch.float64, device="cuda:0")
    with pytest.raises(MuonCaveError, match="MC_ERR_ARG"):
        prob.logpost_batch_noalloc(H, lp)
    # the largest request that fits still runs
    m = 131072 // tiles
    lp_ok = prob.logpost_batch_noalloc(H[:m], lp[:m])
    torch.cuda.synchronize()
    assert lp_ok.shape == (m,)
