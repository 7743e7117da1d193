"""Small geometry builders and an independent brute-force ray sampler for tests.

The brute-force sampler below is deliberately a different algorithm from the
oracle's exact march: it samples the ray at the midpoints of short steps and
looks up the bilinear surface at each sample.
"""
from __future__ import annotations

import math
import types

import numpy as np


def make_scenario(n_surfaces, n_rows, n_cols, X, Y, free, top, density, sensor_pos, dirs,
                  exposure=None, atten=400.0, car_r=None, counts=None):
    """A minimal scenario-like object accepted by oracle.OracleProblem and the binding."""
    sensor_pos = np.asarray(sensor_pos, dtype=np.float64).reshape(-1, 3)
    n_s = sensor_pos.shape[0]
    if n_s == 0:
        dirs = np.zeros((0, 0, 3))
    else:
        dirs = np.asarray(dirs, dtype=np.float64).reshape(n_s, -1, 3)
    n_pix = dirs.shape[1]
    if exposure is None:
        exposure = np.full((n_s, n_pix), 1e4)
    if car_r is None:
        car_r = np.full(n_surfaces - 1, 0.5)
    return types.SimpleNamespace(
        name="test", n_surfaces=n_surfaces, n_rows=n_rows, n_cols=n_cols, extent_x=X, extent_y=Y,
        density=np.asarray(density, np.float64), top=np.asarray(top, np.float64).reshape(n_rows, n_cols),
        car_r=np.asarray(car_r, np.float64), truth=np.asarray(free, np.float64),
        sensor_pos=sensor_pos, dirs=dirs, exposure=np.asarray(exposure, np.float64).reshape(n_s, n_pix),
        atten_len=atten, counts=counts, n_sensors=n_s, n_pix=n_pix, n_rays=n_s * n_pix)


def unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def box_exit(q, d, X, Y, ztop):
    T = (ztop - q[2]) / d[2]
    if d[0] > 0:
        T = min(T, (X - q[0]) / d[0])
    if d[0] < 0:
        T = min(T, -q[0] / d[0])
    if d[1] > 0:
        T = min(T, (Y - q[1]) / d[1])
    if d[1] < 0:
        T = min(T, -q[1] / d[1])
    return max(T, 0.0)


def bilinear_at(H, X, Y, x, y):
    """Bilinear interpolation of node values H[R,C] (nodes at i*X/(R-1), j*Y/(C-1))."""
    R, C = H.shape
    hx, hy = X / (R - 1), Y / (C - 1)
    a = np.clip(np.floor(x / hx).astype(int), 0, R - 2)
    b = np.clip(np.floor(y / hy).astype(int), 0, C - 2)
    s = x / hx - a
    w = y / hy - b
    return (H[a, b] * (1 - s) * (1 - w) + H[a + 1, b] * s * (1 - w) +
            H[a, b + 1] * (1 - s) * w + H[a + 1, b + 1] * s * w)


def brute_force_lengths(surfs, X, Y, q, d, delta):
    """Below-lengths per surface by midpoint sampling with step delta.

    surfs: [S, R, C] all surfaces (top last).  Returns (L[S], sign_changes[S]).
    The error of each L is at most delta/2 per crossing of that surface.
    """
    ztop = float(np.max(surfs[-1]))
    T = box_exit(q, d, X, Y, ztop)
    n = int(math.ceil(T / delta))
    edges = np.minimum(np.arange(n + 1) * delta, T)
    lens = np.diff(edges)
    tm = 0.5 * (edges[:-1] + edges[1:])
    x, y, z = q[0] + tm * d[0], q[1] + tm * d[1], q[2] + tm * d[2]
    L = np.zeros(surfs.shape[0])
    changes = np.zeros(surfs.shape[0])
    for l in range(surfs.shape[0]):
        below = z < bilinear_at(surfs[l], X, Y, x, y)
        L[l] = float(np.sum(lens[below]))
        changes[l] = float(np.count_nonzero(below[1:] != below[:-1]))
    return L, changes


def opacity_from_lengths(L, density):
    S = len(density)
    rho_above = np.append(np.asarray(density[1:], np.float64), 0.0)
    return float(np.sum((np.asarray(density) - rho_above) * L[:S]))


def central_differences(oracle_mod, sc, x0, n_coords, h, seed):
    """Central differences of the oracle's float64 log posterior at the free
    state x0 [S-1, R, C] on n_coords seeded coordinates of all S surfaces
    (a coordinate of the fixed top perturbs the problem's top).  Returns a
    list of (surface, i, j, forward, backward, central) differences."""
    import copy

    S, R, C = sc.n_surfaces, sc.n_rows, sc.n_cols
    rng = np.random.default_rng(seed)
    picks = [np.unravel_index(k, (S, R, C)) for k in rng.choice(S * R * C, n_coords, replace=False)]
    orc = oracle_mod.OracleProblem(sc)
    f0 = orc.logpost(x0)
    free_states, free_idx, out = [], [], []
    for (l, i, j) in picks:
        if l < S - 1:
            xp, xm = x0.copy(), x0.copy()
            xp[l, i, j] += h
            xm[l, i, j] -= h
            free_idx.append((l, i, j))
            free_states += [xp, xm]
    vals = orc.logpost_batch(np.stack(free_states)) if free_states else []
    for k, (l, i, j) in enumerate(free_idx):
        fp, fm = vals[2 * k], vals[2 * k + 1]
        out.append((int(l), int(i), int(j), (fp - f0) / h, (f0 - fm) / h, (fp - fm) / (2 * h)))
    for (l, i, j) in picks:
        if l < S - 1:
            continue
        fv = []
        for sgn in (1.0, -1.0):
            sc2 = copy.copy(sc)
            sc2.top = sc.top.copy()
            sc2.top[i, j] += sgn * h
            fv.append(oracle_mod.OracleProblem(sc2).logpost(x0))
        out.append((int(l), int(i), int(j), (fv[0] - f0) / h, (f0 - fv[1]) / h, (fv[0] - fv[1]) / (2 * h)))
    return out


def is_kink(fwd, bwd, tol):
    """The two one-sided differences disagree by more than 10x the tolerance:
    the coordinate sits on a kink of the piecewise-smooth log posterior."""
    return abs(fwd - bwd) > 10 * tol + 1e-2 * abs(fwd + bwd)
