"""Pins of the oracle's ray march (opacity as a line integral of the layered
density, Sec. 2.1.1; layer density eq. def_LM_density_grid in its continuum
form).  Each test checks the oracle against something other than itself:
closed forms, brute-force sampling with a rigorous error bound, or exact
invariances of the line integral."""
import math

import numpy as np
import pytest

from tests.helpers import (box_exit, brute_force_lengths, make_scenario, opacity_from_lengths,
                           unit)


def flat_problem(oracle_mod, levels, X=300.0, Y=200.0, R=7, C=5, density=(1.8, 0.0, 2.7)):
    S = len(levels)
    free = np.stack([np.full((R, C), c) for c in levels[:-1]])
    sc = make_scenario(S, R, C, X, Y, free, np.full((R, C), levels[-1]), density,
                       [[150.0, 100.0, 0.0]], [[[0, 0, 1.0]]])
    return oracle_mod.OracleProblem(sc), free


def test_flat_layers_closed_form(oracle_mod):
    """Flat horizontal layers: L_l = clamp((c_l - q_z)/d_z, 0, T); with no
    lateral exit the opacity is sum_units rho * thickness / cos(zenith)."""
    levels = [60.0, 75.0, 200.0]
    dens = (1.8, 0.0, 2.7)
    prob, free = flat_problem(oracle_mod, levels, density=dens)
    rng = np.random.default_rng(0)
    for _ in range(200):
        q = np.array([rng.uniform(0, 300), rng.uniform(0, 200), rng.uniform(0, 50)])
        th = rng.uniform(0, math.radians(60))
        ph = rng.uniform(0, 2 * math.pi)
        d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        O, L, _ = prob.march_one(free, q, d)
        T = box_exit(q, d, 300.0, 200.0, 200.0)
        for l, c in enumerate(levels):
            assert L[l] == pytest.approx(min(max((c - q[2]) / d[2], 0.0), T), abs=1e-9)
    # no lateral exit: vertical-ish rays from the centre
    q = np.array([150.0, 100.0, 0.0])
    for th in np.radians([0.0, 5.0, 10.0, 20.0]):
        d = np.array([math.sin(th), 0.0, math.cos(th)])
        O, L, _ = prob.march_one(free, q, d)
        expect = (1.8 * 60.0 + 0.0 * 15.0 + 2.7 * 125.0) / math.cos(th)
        assert O == pytest.approx(expect, rel=1e-12)


def test_tilted_plane_crossing(oracle_mod):
    """A plane is reproduced exactly by bilinear interpolation; its crossing is
    t* = (h0 + g.q_xy - q_z) / (d_z - g.d_xy)."""
    R, C, X, Y = 5, 4, 40.0, 30.0
    xs, ys = np.linspace(0, X, R), np.linspace(0, Y, C)
    h0, gx, gy = 20.0, 0.3, -0.2
    plane = h0 + gx * xs[:, None] + gy * ys[None, :]
    sc = make_scenario(2, R, C, X, Y, plane[None], np.full((R, C), 100.0), (2.0, 1.0),
                       [[1, 1, 0.0]], [[[0, 0, 1.0]]])
    prob = oracle_mod.OracleProblem(sc)
    rng = np.random.default_rng(1)
    checked = 0
    for _ in range(300):
        q = np.array([rng.uniform(0, X), rng.uniform(0, Y), rng.uniform(0, 10)])
        d = unit([rng.normal(), rng.normal(), rng.uniform(0.5, 2.0)])
        T = box_exit(q, d, X, Y, 100.0)
        den = d[2] - gx * d[0] - gy * d[1]
        ts = (h0 + gx * q[0] + gy * q[1] - q[2]) / den
        if den <= 0 or not (0 < ts < T):
            continue
        O, L, st = prob.march_one(plane[None], q, d)
        assert L[0] == pytest.approx(ts, abs=1e-9)
        assert st["crossings"] == 1
        checked += 1
    assert checked > 50


@pytest.mark.parametrize("c,k,v,roots", [
    (0.5, 0.25, 1.5, "one"),
    (0.2, 0.5, 0.6, "two"),
])
def test_saddle_cell_hand_solved(oracle_mod, c, k, v, roots):
    """One 2x2-node cell holding the saddle h = c + k(1-2x)(1-2y) on [0,1]^2.
    A ray from the origin along the diagonal sees h = c + k(1-2p)^2 and
    z = v p (p = x = y); crossings solve 4k p^2 - (4k+v) p + (c+k) = 0."""
    H1 = np.array([[c + k, c - k], [c - k, c + k]])
    sc = make_scenario(2, 2, 2, 1.0, 1.0, H1[None], np.full((2, 2), 10.0), (1.0, 0.5),
                       [[0, 0, 0.0]], [[[0, 0, 1.0]]])
    prob = oracle_mod.OracleProblem(sc)
    n = math.sqrt(2 + v * v)
    d = np.array([1.0, 1.0, v]) / n
    A, B, Cq = 4 * k, -(4 * k + v), c + k
    disc = math.sqrt(B * B - 4 * A * Cq)
    p1, p2 = (-B - disc) / (2 * A), (-B + disc) / (2 * A)
    if roots == "one":
        assert 0 < p1 < 1 < p2
        expect_L1 = n * p1
    else:
        assert 0 < p1 < p2 < 1
        expect_L1 = n * (p1 + (1 - p2))
    O, L, st = prob.march_one(H1[None], np.zeros(3), d)
    assert L[0] == pytest.approx(expect_L1, rel=1e-12)
    assert L[1] == pytest.approx(n, rel=1e-12)   # lateral exit at x = 1, below the top
    assert O == pytest.approx((1.0 - 0.5) * L[0] + 0.5 * L[1], rel=1e-12)
    assert st["crossings"] == (1 if roots == "one" else 2)


def random_grid_problem(oracle_mod, rng, R, C, X, Y, S=3, amp=6.0):
    """Random wavy surfaces (not necessarily ordered) on a small grid."""
    base = np.linspace(20.0, 40.0, S)
    surfs = np.stack([base[l] + amp * rng.standard_normal((R, C)) for l in range(S)])
    dens = rng.uniform(0.5, 3.0, S)
    sc = make_scenario(S, R, C, X, Y, surfs[:-1], surfs[-1], dens, [[0, 0, 0.0]], [[[0, 0, 1.0]]])
    return oracle_mod.OracleProblem(sc), surfs, dens


@pytest.mark.parametrize("R,C", [(3, 3), (4, 5), (5, 4), (5, 5)])
def test_bruteforce_fine_sampling(oracle_mod, R, C):
    """Midpoint sampling at step delta bounds |L_bf - L| <= (crossings/2 + 1) delta;
    the test also checks convergence as delta shrinks."""
    rng = np.random.default_rng(100 + 10 * R + C)
    X, Y = 30.0 + 5 * R, 25.0 + 4 * C
    prob, surfs, dens = random_grid_problem(oracle_mod, rng, R, C, X, Y)
    for _ in range(12):
        q = np.array([rng.uniform(0, X), rng.uniform(0, Y), rng.uniform(0, 15.0)])
        d = unit([rng.normal(), rng.normal(), rng.uniform(0.4, 1.5)])
        O, L, st = prob.march_one(surfs[:-1], q, d)
        prev = None
        for delta in (1e-2, 1e-3, 1e-4):
            Lbf, changes = brute_force_lengths(surfs, X, Y, q, d, delta)
            bound = (0.5 * changes + 1.0) * delta + 1e-9
            assert np.all(np.abs(Lbf - L) <= bound), (delta, Lbf, L, changes)
            err = np.max(np.abs(Lbf - L))
            if prev is not None and prev > 10 * delta:
                assert err < prev
            prev = err
        assert O == pytest.approx(opacity_from_lengths(L, dens), rel=1e-12)


def test_bruteforce_opacity_with_explicit_units(oracle_mod):
    """Opacity written as sum over units of density x (length inside the unit),
    from brute-force sampling of which unit each sample lies in."""
    rng = np.random.default_rng(7)
    R, C, X, Y = 4, 6, 50.0, 70.0
    base = rng.uniform(5, 8, (R, C))
    H1 = base
    H2 = H1 + rng.uniform(0.5, 6.0, (R, C))
    top = 40.0 + rng.uniform(-3, 3, (R, C))
    dens = np.array([1.8, 0.0, 2.7])
    sc = make_scenario(3, R, C, X, Y, np.stack([H1, H2]), top, dens, [[0, 0, 0.0]], [[[0, 0, 1.0]]])
    prob = oracle_mod.OracleProblem(sc)
    surfs = np.stack([H1, H2, top])
    from tests.helpers import bilinear_at
    for _ in range(10):
        q = np.array([rng.uniform(0, X), rng.uniform(0, Y), 0.0])
        d = unit([rng.normal(), rng.normal(), rng.uniform(0.8, 2.0)])
        O, L, st = prob.march_one(surfs[:-1], q, d)
        delta = 1e-4
        T = box_exit(q, d, X, Y, float(top.max()))
        n = int(math.ceil(T / delta))
        e = np.minimum(np.arange(n + 1) * delta, T)
        tm = 0.5 * (e[1:] + e[:-1])
        x, y, z = q[0] + tm * d[0], q[1] + tm * d[1], q[2] + tm * d[2]
        h = [bilinear_at(s, X, Y, x, y) for s in surfs]
        unit_density = np.where(z < h[0], dens[0], np.where(z < h[1], dens[1], np.where(z < h[2], dens[2], 0.0)))
        Obf = float(np.sum(unit_density * np.diff(e)))
        assert O == pytest.approx(Obf, abs=3.0 * 2.7 * 6 * delta)


def test_invariants_monotone_zero_and_lengths(oracle_mod):
    rng = np.random.default_rng(3)
    R, C, X, Y = 6, 5, 60.0, 50.0
    H1 = 20 + 3 * rng.standard_normal((R, C))
    H2 = H1 + 2 + np.abs(3 * rng.standard_normal((R, C)))
    top = np.full((R, C), 80.0)
    free = np.stack([H1, H2])
    base_d = np.array([1.8, 0.0, 2.7])
    qs = [np.array([rng.uniform(0, X), rng.uniform(0, Y), 0.0]) for _ in range(20)]
    ds = [unit([rng.normal(), rng.normal(), rng.uniform(0.7, 2)]) for _ in range(20)]

    def ops(dens):
        sc = make_scenario(3, R, C, X, Y, free, top, dens, [[0, 0, 0.0]], [[[0, 0, 1.0]]])
        prob = oracle_mod.OracleProblem(sc)
        return [prob.march_one(free, q, d) for q, d in zip(qs, ds)]

    base = ops(base_d)
    # zero density everywhere -> zero opacity
    for O, L, _ in ops(np.zeros(3)):
        assert O == 0.0
    # monotone in each unit density: dO/drho_u = length inside unit u >= 0
    for u in range(3):
        bumped = base_d.copy()
        bumped[u] += 0.5
        for (O0, L0, _), (O1, L1, _) in zip(base, ops(bumped)):
            assert O1 >= O0 - 1e-12
            inside = L0[u] - (L0[u - 1] if u > 0 else 0.0)
            assert O1 - O0 == pytest.approx(0.5 * inside, abs=1e-9)
    # the unit lengths add up to the in-box length (flat top: L_top = T)
    for (O, L, _), q, d in zip(base, qs, ds):
        assert L[2] == pytest.approx(box_exit(q, d, X, Y, 80.0), rel=1e-12)
        assert 0 <= L[0] <= L[1] + 1e-12 <= L[2] + 2e-12


def test_zero_opacity_in_air(oracle_mod):
    """A ray that starts in the air gap and only meets air before leaving the
    box through the side has zero opacity."""
    R, C, X, Y = 3, 3, 20.0, 20.0
    free = np.stack([np.full((R, C), 5.0), np.full((R, C), 50.0)])
    sc = make_scenario(3, R, C, X, Y, free, np.full((R, C), 60.0), (1.8, 0.0, 2.7),
                       [[10, 10, 6.0]], [[[0, 0, 1.0]]])
    prob = oracle_mod.OracleProblem(sc)
    O, L, _ = prob.march_one(free, np.array([10, 10, 6.0]), unit([1.0, 0.3, 0.5]))
    assert O == 0.0


def test_mirror_and_rotation_symmetry(oracle_mod):
    """x -> X - x with d_x -> -d_x, and a 90-degree rotation of a square
    grid, leave every opacity unchanged."""
    rng = np.random.default_rng(11)
    R = C = 6
    X = Y = 50.0
    H1 = 20 + 3 * rng.standard_normal((R, C))
    H2 = H1 + 1 + np.abs(4 * rng.standard_normal((R, C)))
    top = 70 + rng.standard_normal((R, C))
    dens = (1.8, 0.0, 2.7)

    def O_of(free, top_, q, d):
        sc = make_scenario(3, R, C, X, Y, free, top_, dens, [[0, 0, 0.0]], [[[0, 0, 1.0]]])
        return oracle_mod.OracleProblem(sc).march_one(free, q, d)[0]

    free = np.stack([H1, H2])
    for _ in range(10):
        q = np.array([rng.uniform(5, 45), rng.uniform(5, 45), 0.0])
        d = unit([rng.normal(), rng.normal(), rng.uniform(0.7, 2)])
        O = O_of(free, top, q, d)
        Om = O_of(free[:, ::-1, :].copy(), top[::-1, :].copy(), np.array([X - q[0], q[1], q[2]]),
                  np.array([-d[0], d[1], d[2]]))
        assert Om == pytest.approx(O, rel=1e-11)
        # rotation by 90 degrees: (x, y) -> (y, X - x); node (i, j) -> (j, R-1-i)
        Hr = np.stack([np.rot90(f, k=-1) for f in free])
        # np.rot90(k=-1): new[j, R-1-i] = old[i, j]
        Or = O_of(Hr.copy(), np.rot90(top, k=-1).copy(), np.array([q[1], X - q[0], q[2]]),
                  np.array([d[1], -d[0], d[2]]))
        assert Or == pytest.approx(O, rel=1e-11)


def test_cell_shift_invariance(oracle_mod):
    """Shifting the sensor and the surfaces together by whole cells leaves the
    opacity unchanged while the ray stays inside the footprint."""
    rng = np.random.default_rng(5)
    R, C, h = 12, 10, 10.0
    X, Y = h * (R - 1), h * (C - 1)
    H1 = 20 + 3 * rng.standard_normal((R, C))
    H2 = H1 + 1 + np.abs(3 * rng.standard_normal((R, C)))
    top = np.full((R, C), 40.0)
    dens = (1.8, 0.0, 2.7)
    free = np.stack([H1, H2])
    sc = make_scenario(3, R, C, X, Y, free, top, dens, [[0, 0, 0.0]], [[[0, 0, 1.0]]])
    prob = oracle_mod.OracleProblem(sc)
    for sa, sb in [(2, 1), (1, 3), (3, 0)]:
        shifted = np.zeros_like(free)
        shifted[:, sa:, sb:] = free[:, : R - sa, : C - sb]
        shifted[:, :sa, :] = 30.0
        shifted[:, :, :sb] = 30.0
        for _ in range(5):
            q = np.array([rng.uniform(35, 45), rng.uniform(35, 45), 0.0])
            d = unit([rng.normal(), rng.normal(), 2.5])
            if box_exit(q, d, X - sa * h, Y - sb * h, 40.0) < (40.0 / d[2]) or \
               min(q[0] + 40 / d[2] * d[0], q[1] + 40 / d[2] * d[1]) < 0:
                continue
            O = prob.march_one(free, q, d)[0]
            Os = prob.march_one(shifted, q + np.array([sa * h, sb * h, 0.0]), d)[0]
            assert Os == pytest.approx(O, rel=1e-11)
