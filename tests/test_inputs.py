"""CPU checks of the seeded input generators: reproducibility, the documented
ranges of the heterogeneous batch, the Poisson arrival process and the
ordering of chain starts.  The generators hold none of the method's
arithmetic; these tests only pin what the benchmarks and parity tests feed
both sides."""
import numpy as np
import pytest

from paper_2603_28907_amd import inputs


def test_generators_are_seeded():
    a, b = inputs.grf_cave(seed=10, n_grid=32), inputs.grf_cave(seed=10, n_grid=32)
    assert np.array_equal(a.truth, b.truth) and np.array_equal(a.dirs, b.dirs)
    c = inputs.grf_cave(seed=11, n_grid=32)
    assert not np.array_equal(a.truth, c.truth)
    s1 = inputs.init_states(a, 5, seed=3)
    s2 = inputs.init_states(a, 5, seed=3)
    assert np.array_equal(s1, s2)


def test_heterogeneous_batch_ranges():
    grids, sensors, pix, chains = set(), [], [], set()
    for i in range(256):
        sp = inputs.heterogeneous_problem_spec(i)
        grids.add(sp["n_grid"])
        sensors.append(sp["n_sensors"])
        pix.append(sp["pix_side"])
        chains.add(sp["n_chains"])
    assert grids == {16, 32, 64, 128}
    assert min(sensors) >= 2 and max(sensors) <= 16
    assert min(pix) >= 32 and max(pix) <= 64
    assert chains == {64, 128, 256, 512}
    sc, n = inputs.heterogeneous_problem(3, scale_pixels=0.25)
    sp = inputs.heterogeneous_problem_spec(3)
    assert sc.n_rows == sp["n_grid"] and sc.sensor_pos.shape[0] == sp["n_sensors"] and n == sp["n_chains"]
    assert sc.extent_x == pytest.approx(400.0)


def test_poisson_arrivals():
    t = inputs.poisson_arrivals(20.0, 200.0, seed=40)
    assert np.all(np.diff(t) > 0) and t[0] >= 0 and t[-1] < 200.0
    # mean rate and exponential gaps
    assert len(t) / 200.0 == pytest.approx(20.0, rel=0.05)
    gaps = np.diff(t)
    assert gaps.mean() == pytest.approx(1 / 20.0, rel=0.05)
    assert np.std(gaps) / gaps.mean() == pytest.approx(1.0, rel=0.1)


def test_chain_starts_are_ordered_inside_the_box():
    sc = inputs.grf_cave(seed=10, n_grid=32)
    st = inputs.init_states(sc, 64, seed=12, jitter=5.0)
    assert np.all(st[:, 0] > 0)
    assert np.all(st[:, 1] > st[:, 0])
    assert np.all(sc.top[None] > st[:, -1])


def test_pixel_directions_cover_the_cone():
    d = inputs.pixel_directions(8, 16, max_zenith_deg=45.0)
    d = np.asarray(d).reshape(-1, 3)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    zen = np.degrees(np.arccos(d[:, 2]))
    assert zen.min() > 0 and zen.max() < 45.0
