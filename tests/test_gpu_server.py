"""The serving loop (mc_server_*): continuous batching of heterogeneous jobs.

A job's result must be the same alone and in a mix (bit for bit: its random
numbers and launch shape depend only on its own description), equal to the
plain sampler run on the same inputs, and -- in float64 on the small cave --
to the oracle's sampler up to rounding.  Admission must respect the slot
and memory limits, and jobs arriving while others run must be admitted
before those finish."""
import time

import numpy as np
import pytest

from paper_2603_28907_amd import inputs
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    return require_gpu()


def _jobs(oracle_mod, ids, max_chains=16, scale_pixels=0.25):
    out = []
    for i in ids:
        sc, n = inputs.heterogeneous_problem(i, scale_pixels=scale_pixels)
        sc.counts = oracle_mod.make_counts(sc, seed=100 + i)
        out.append((sc, min(n, max_chains), 3000 + i))
    return out


def _wait_status(srv, jid, status, timeout=60.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        if srv.poll(jid, arrays=False)["status"] >= status:
            return
        time.sleep(0.002)
    raise AssertionError(f"job {jid} did not reach status {status}")


def _same(a, b):
    for k in ("mean", "std", "map_state"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("accept_rate", "map_logpost", "map_chain", "steps_done"):
        assert a[k] == b[k], k


def test_job_alone_equals_mix_and_plain_sampler(torch_mod, oracle_mod):
    from paper_2603_28907_amd.binding import JOB_DONE, JOB_RUNNING, Problem, Server
    torch = torch_mod
    jobs = _jobs(oracle_mod, [0, 1, 3, 5])
    x_sc, x_n, x_seed = jobs[2]
    steps, sigma = 60, 0.005
    say("server: job alone")
    srv = Server(precision="f32", max_jobs=1, steps_per_round=20)
    jx = srv.submit(x_sc, x_n, steps, sigma, x_seed)
    srv.wait_idle(120)
    alone = srv.poll(jx)
    srv.close()
    assert alone["status"] == JOB_DONE and alone["steps_done"] == steps
    say("server: job in a mix")
    srv = Server(precision="f32", max_jobs=8, steps_per_round=20)
    ids = [srv.submit(sc, n, 100, sigma, seed) for sc, n, seed in (jobs[0], jobs[1])]
    _wait_status(srv, ids[0], JOB_RUNNING)
    jx2 = srv.submit(x_sc, x_n, steps, sigma, x_seed)
    ids.append(srv.submit(jobs[3][0], jobs[3][1], 40, sigma, jobs[3][2]))
    srv.wait_idle(120)
    mixed = srv.poll(jx2)
    st = srv.stats()
    say("stats", st)
    assert all(srv.poll(j, arrays=False)["status"] == JOB_DONE for j in ids)
    srv.close()
    assert st["max_resident"] >= 2
    _same(alone, mixed)
    # the plain sampler on the same inputs: every chain starts at the truth
    say("plain sampler")
    prob = Problem.from_scenario(x_sc, precision="f32")
    H = to_dev(np.broadcast_to(x_sc.truth, (x_n,) + x_sc.truth.shape), torch.float32)
    lp = to_dev(np.full(x_n, np.nan), torch.float64)
    acc = to_dev(np.zeros(x_n, np.int64), torch.int64)
    prob.mcmc_run(H, lp, acc, steps, sigma, x_seed, graph_steps=20)
    torch.cuda.synchronize()
    Hh, lph, acch = H.double().cpu().numpy(), lp.cpu().numpy(), acc.cpu().numpy()
    best = int(np.argmax(lph))
    assert alone["map_chain"] == best and alone["map_logpost"] == lph[best]
    assert np.array_equal(alone["map_state"], Hh[best])
    assert alone["accept_rate"] == acch.sum() / (x_n * steps)
    np.testing.assert_allclose(alone["mean"], Hh.mean(axis=0), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(alone["std"], Hh.std(axis=0), rtol=1e-9, atol=1e-12)


def test_f64_job_matches_oracle_sampler(torch_mod, oracle_mod):
    from paper_2603_28907_amd.binding import JOB_DONE, Server
    sc = inputs.tiny_bumps(seed=0)
    sc.counts = oracle_mod.make_counts(sc, seed=1)
    n, steps, sigma, seed = 4, 40, 0.05, 2024
    srv = Server(precision="f64", max_jobs=2, steps_per_round=16)
    j = srv.submit(sc, n, steps, sigma, seed)
    srv.wait_idle(60)
    r = srv.poll(j)
    srv.close()
    assert r["status"] == JOB_DONE
    orc = oracle_mod.OracleProblem(sc)
    states = np.broadcast_to(sc.truth, (n,) + sc.truth.shape).copy()
    Ho, lpo, acco, marg = orc.mcmc_rw(states, np.full(n, np.nan), np.zeros(n, np.int64), steps, 0, sigma, seed,
                                      want_margins=True)
    assert np.nanmin(marg) > 1e-6, "a near-tie decision; choose another seed"
    say("oracle acceptances", acco)
    assert r["accept_rate"] == acco.sum() / (n * steps)
    np.testing.assert_allclose(r["mean"], Ho.mean(axis=0), rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(r["std"], Ho.std(axis=0), rtol=1e-7, atol=1e-10)
    best = int(np.argmax(lpo))
    assert r["map_chain"] == best
    np.testing.assert_allclose(r["map_state"], Ho[best], rtol=1e-12, atol=1e-10)
    assert r["map_logpost"] == pytest.approx(lpo[best], rel=1e-11, abs=1e-6)


def test_admission_by_slots_and_memory(torch_mod, oracle_mod):
    from paper_2603_28907_amd.binding import JOB_DONE, MuonCaveError, Server
    jobs = _jobs(oracle_mod, [3, 4, 5, 7, 10], max_chains=8)
    srv = Server(precision="f32", max_jobs=2, steps_per_round=10)
    ids = [srv.submit(sc, n, 30, 0.005, seed) for sc, n, seed in jobs]
    srv.wait_idle(120)
    st = srv.stats()
    infos = [srv.poll(j, arrays=False) for j in ids]
    srv.close()
    say("slots", st)
    assert st["max_resident"] <= 2 and st["done"] == len(jobs) and st["bytes_in_use"] == 0
    for inf in infos:
        assert inf["status"] == JOB_DONE
        assert 0 < inf["t_submit"] <= inf["t_admit"] <= inf["t_done"]
    # a budget that holds the largest job but not two of them
    big = max(inf["footprint"] for inf in infos)
    srv = Server(precision="f32", memory_budget=big + big // 2, max_jobs=8, steps_per_round=10)
    ids = [srv.submit(sc, n, 30, 0.005, seed) for sc, n, seed in jobs]
    srv.wait_idle(120)
    st = srv.stats()
    say("memory", st)
    assert st["done"] == len(jobs) and st["peak_bytes"] <= big + big // 2
    sc, n, seed = jobs[0]
    with pytest.raises(MuonCaveError, match="budget"):
        srv.submit(sc, 4096, 30, 0.005, seed)
    srv.close()


def test_arrivals_join_running_jobs(torch_mod, oracle_mod):
    """Continuous batching: a short job submitted while a long one runs is
    admitted and finishes before the long one."""
    from paper_2603_28907_amd.binding import JOB_DONE, JOB_RUNNING, Server
    jobs = _jobs(oracle_mod, [5, 3], max_chains=16)
    srv = Server(precision="f32", max_jobs=4, steps_per_round=10)
    long_id = srv.submit(jobs[0][0], jobs[0][1], 400, 0.005, 1)
    _wait_status(srv, long_id, JOB_RUNNING)
    short_id = srv.submit(jobs[1][0], jobs[1][1], 20, 0.005, 2)
    srv.wait_idle(120)
    a, b = srv.poll(long_id, arrays=False), srv.poll(short_id, arrays=False)
    srv.close()
    say("long", a, "short", b)
    assert a["status"] == JOB_DONE and b["status"] == JOB_DONE
    assert b["t_admit"] < a["t_done"] and b["t_done"] < a["t_done"]


def test_mixed_surface_counts_and_request_errors(torch_mod, oracle_mod):
    """Jobs with 2 and 3 surfaces share a server (one batched launch group per
    surface count); each equals its run alone.  Invalid requests are refused
    at submission, unknown ids and early releases are errors."""
    from paper_2603_28907_amd.binding import JOB_DONE, MuonCaveError, Server
    from tests.helpers import make_scenario
    t = inputs.tiny_bumps(seed=4)
    s2 = make_scenario(2, t.n_rows, t.n_cols, t.extent_x, t.extent_y, t.truth[:1], t.top, (1.8, 2.7),
                       t.sensor_pos, t.dirs, car_r=t.car_r[:1])
    s2.counts = oracle_mod.make_counts(s2, seed=5)
    s3 = inputs.tiny_bumps(seed=6)
    s3.counts = oracle_mod.make_counts(s3, seed=7)
    from paper_2603_28907_amd.binding import JOB_RUNNING
    runs = []
    for mix in (False, True):
        srv = Server(precision="f32", max_jobs=4, steps_per_round=10)
        b = None
        if mix:   # a long 3-surface job is running when the 2-surface one arrives
            b = srv.submit(s3, 8, 600, 0.05, 12)
            _wait_status(srv, b, JOB_RUNNING)
        a = srv.submit(s2, 8, 30, 0.05, 11)
        srv.wait_idle(120)
        ra = srv.poll(a)
        rb = srv.poll(b) if mix else None
        if mix:
            with pytest.raises(MuonCaveError, match="n_chains"):
                srv.submit(s3, 0, 30, 0.05, 1)
            with pytest.raises(MuonCaveError, match="unknown"):
                srv.release(10 ** 9)
            st = srv.stats()
            assert st["max_resident"] == 2
        srv.close()
        assert ra["status"] == JOB_DONE and (rb is None or rb["status"] == JOB_DONE)
        runs.append(ra)
    for k in ("mean", "std", "map_state"):
        assert np.array_equal(runs[0][k], runs[1][k]), k
    assert runs[0]["accept_rate"] == runs[1]["accept_rate"] and 0 < runs[0]["accept_rate"] < 1


def test_release_before_done_is_refused(torch_mod, oracle_mod):
    from paper_2603_28907_amd.binding import JOB_DONE, MuonCaveError, Server
    sc = inputs.tiny_bumps(seed=8)
    sc.counts = oracle_mod.make_counts(sc, seed=9)
    srv = Server(precision="f32", max_jobs=1, steps_per_round=10)
    j = srv.submit(sc, 8, 2000, 0.05, 3)
    with pytest.raises(MuonCaveError, match="not finished"):
        srv.release(j)
    srv.wait_idle(120)
    assert srv.poll(j, arrays=False)["status"] == JOB_DONE
    srv.release(j)
    srv.close()


def test_job_with_sampled_r_alone_mix_and_plain(torch_mod, oracle_mod):
    """A served job whose chains sample r too (r_step > 0): the same bits alone,
    in a mix with fixed-r jobs and another r job, and as the plain sampler
    mcmc_run with r_state started at the job's r."""
    from paper_2603_28907_amd.binding import JOB_DONE, Problem, Server
    torch = torch_mod
    jobs = _jobs(oracle_mod, [0, 2, 3, 4])
    x_sc, x_n, x_seed = jobs[2]
    steps, sigma, tau = 60, 0.005, 0.4
    srv = Server(precision="f32", max_jobs=1, steps_per_round=20)
    jx = srv.submit(x_sc, x_n, steps, sigma, x_seed, r_step=tau)
    srv.wait_idle(120)
    alone = srv.poll(jx)
    srv.close()
    assert alone["status"] == JOB_DONE
    srv = Server(precision="f32", max_jobs=8, steps_per_round=20)
    others = [srv.submit(jobs[0][0], jobs[0][1], 80, sigma, jobs[0][2]),
              srv.submit(jobs[1][0], jobs[1][1], 40, sigma, jobs[1][2], r_step=0.3)]
    jx2 = srv.submit(x_sc, x_n, steps, sigma, x_seed, r_step=tau)
    others.append(srv.submit(jobs[3][0], jobs[3][1], 60, sigma, jobs[3][2]))
    srv.wait_idle(120)
    mixed = srv.poll(jx2)
    assert all(srv.poll(j, arrays=False)["status"] == JOB_DONE for j in others)
    srv.close()
    _same(alone, mixed)
    assert alone["r_mean"] == mixed["r_mean"] and alone["r_accept_rate"] == mixed["r_accept_rate"]
    # the plain sampler with r
    prob = Problem.from_scenario(x_sc, precision="f32")
    H = to_dev(np.broadcast_to(x_sc.truth, (x_n,) + x_sc.truth.shape), torch.float32)
    lp = to_dev(np.full(x_n, np.nan), torch.float64)
    acc = to_dev(np.zeros(x_n, np.int64), torch.int64)
    S1 = x_sc.n_surfaces - 1
    r = to_dev(np.broadcast_to(x_sc.car_r, (x_n, S1)), torch.float64)
    ar = torch.zeros((x_n, S1), dtype=torch.int64, device="cuda:0")
    prob.mcmc_run(H, lp, acc, steps, sigma, x_seed, graph_steps=20, r_state=r, r_step=tau, n_accept_r=ar)
    torch.cuda.synchronize()
    Hh, lph = H.double().cpu().numpy(), lp.cpu().numpy()
    best = int(np.argmax(lph))
    assert alone["map_chain"] == best and alone["map_logpost"] == lph[best]
    assert np.array_equal(alone["map_state"], Hh[best])
    rh = r.cpu().numpy()
    want = [float(v) for v in sum(rh[c] / x_n for c in range(x_n))]
    np.testing.assert_allclose(alone["r_mean"][:S1], want, rtol=1e-14)
    assert alone["r_accept_rate"] == ar.sum().item() / (x_n * S1 * steps)
    assert 0.0 < alone["r_accept_rate"] < 1.0
