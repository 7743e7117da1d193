"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This module only *generates inputs*: grids, true surfaces, sensor positions,
pixel directions, exposures, initial chain states, Poisson draws from a given
mean and job-arrival streams.  It contains none of the method's arithmetic
(no ray march, no likelihood, no prior density): whoever needs expected counts
computes them with their own forward model and passes them to `draw_counts`.

Workload shapes follow the paper's setting: a box domain with sensors under
the cave (Sec. "Muon attenuation"), a layer model with three interfaces
muck/air, air/rock and rock/terrain on an n_rows x n_cols grid (Sec.
"Low-dimensional representation of the cave geometry"), radiographs binned by
solid angle into pixels, and Poisson counts.  The paper's own cave model and
25-sensor layout are not public; the synthetic recipes below stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Unit densities (g/cm^3) for the block-cave layer model: unit 1 (floor..muck
# top) is muck, unit 2 (muck top..cave back) is air, unit 3 (cave back..terrain)
# is in-situ rock.
DEFAULT_DENSITY = (1.8, 0.0, 2.7)


@dataclasses.dataclass
class Scenario:
    """One inference problem: geometry, sensors, exposure and (optionally) counts.

    Heights are metres above the floor of the box domain.  Arrays are float64
    host arrays in C order; `truth` and chain states hold the free surfaces
    only (surfaces 1..S-1); the fixed top surface S is `top`.
    """

    name: str
    n_surfaces: int
    n_rows: int
    n_cols: int
    extent_x: float
    extent_y: float
    density: np.ndarray          # [S]
    top: np.ndarray              # [R, C]
    car_r: np.ndarray            # [S-1]
    truth: np.ndarray            # [S-1, R, C]
    sensor_pos: np.ndarray       # [n_s, 3]
    dirs: np.ndarray             # [n_s, n_pix, 3]
    exposure: np.ndarray         # [n_s, n_pix]
    atten_len: float
    counts: Optional[np.ndarray] = None   # [n_s, n_pix] int32
    seed: int = 0

    @property
    def n_sensors(self) -> int:
        return int(self.sensor_pos.shape[0])

    @property
    def n_pix(self) -> int:
        return int(self.dirs.shape[1]) if self.dirs.ndim == 3 else 0

    @property
    def n_rays(self) -> int:
        return self.n_sensors * self.n_pix

    def all_surfaces(self, free: np.ndarray) -> np.ndarray:
        """Stack free surfaces [.., S-1, R, C] with the fixed top -> [.., S, R, C]."""
        free = np.asarray(free, dtype=np.float64)
        top = np.broadcast_to(self.top, free.shape[:-3] + (1,) + self.top.shape)
        return np.concatenate([free, top], axis=-3)


# ----------------------------------------------------------------------------
# Elementary generators
# ----------------------------------------------------------------------------

def pixel_directions(n_zen: int, n_az: int, max_zenith_deg: float = 45.0) -> np.ndarray:
    """Unit vectors at pixel centres of an (n_zen x n_az) zenith/azimuth radiograph.

    Zenith (k+1/2)*max/n_zen, azimuth (m+1/2)*360/n_az, pixel p = k*n_az + m
    (zenith-major).  Returned as [n_zen*n_az, 3] with d_z > 0.
    """
    k = (np.arange(n_zen) + 0.5) * (math.radians(max_zenith_deg) / n_zen)
    m = (np.arange(n_az) + 0.5) * (2.0 * math.pi / n_az)
    th, ph = np.meshgrid(k, m, indexing="ij")
    d = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1)
    return d.reshape(-1, 3).astype(np.float64)


def pixel_subrays(n_zen: int, n_az: int, q: int, max_zenith_deg: float = 45.0, exposure: float = 1e4,
                  efficiency=None):
    """Sub-rays of the same radiograph for the solid-angle pixel integral:
    each pixel (as in pixel_directions) is split into q x q zenith/azimuth
    sub-cells, one ray at each sub-cell centre, pixel-major ([n_pix*q*q, 3]).
    The weights are exposure * efficiency(zenith) * solid angle of the
    sub-cell / solid angle of the pixel's centre cell, so that they sum to
    about exposure * efficiency per pixel.  efficiency defaults to a smooth
    synthetic detector response 0.9 - 0.3 sin^2(zenith)."""
    if efficiency is None:
        efficiency = lambda th: 0.9 - 0.3 * np.sin(th) ** 2   # noqa: E731
    dth = math.radians(max_zenith_deg) / n_zen
    dph = 2.0 * math.pi / n_az
    dirs, w = [], []
    for k in range(n_zen):
        pix_sa = dph * (math.cos(k * dth) - math.cos((k + 1) * dth))
        for m in range(n_az):
            for a in range(q):
                lo, hi = (k + a / q) * dth, (k + (a + 1) / q) * dth
                th = 0.5 * (lo + hi)
                sa = (dph / q) * (math.cos(lo) - math.cos(hi))
                for b in range(q):
                    ph = (m + (b + 0.5) / q) * dph
                    dirs.append((math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)))
                    w.append(exposure * efficiency(th) * sa / pix_sa)
    return np.asarray(dirs, np.float64), np.asarray(w, np.float64)


def intensity_table(n_tab: int = 256, o_max: float = 2000.0, atten: float = 400.0) -> np.ndarray:
    """A synthetic stand-in for the tabulated muon intensity: log I(O) at
    n_tab uniform opacity nodes over [0, o_max], I(O) = exp(-O/atten) /
    sqrt(1 + O/100) (smooth, positive, decreasing)."""
    O = np.linspace(0.0, o_max, n_tab)
    return -O / atten - 0.5 * np.log1p(O / 100.0)


def gaussian_bumps(rng: np.random.Generator, xs: np.ndarray, ys: np.ndarray, n_bumps: int,
                   amp=(5.0, 20.0), width=(10.0, 30.0), centre_lo=20.0, centre_hi=80.0) -> np.ndarray:
    """Sum of isotropic Gaussian bumps on the node grid (xs along rows, ys along columns)."""
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    out = np.zeros_like(X)
    for _ in range(n_bumps):
        a = rng.uniform(*amp)
        w = rng.uniform(*width)
        cx, cy = rng.uniform(centre_lo, centre_hi, size=2)
        out += a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))
    return out


def periodic_grf(rng: np.random.Generator, n_rows: int, n_cols: int, extent_x: float,
                 extent_y: float, length_scale: float = 50.0, nu: float = 1.5) -> np.ndarray:
    """Unit-variance periodic Gaussian random field by FFT synthesis.

    Spectrum of Matern type, S(k) ~ (kappa^2 + |k|^2)^-(nu+1) with
    kappa = sqrt(2 nu)/length_scale; the sample is standardised to zero mean
    and unit sample variance.
    """
    kx = 2 * math.pi * np.fft.fftfreq(n_rows, d=extent_x / n_rows)
    ky = 2 * math.pi * np.fft.fftfreq(n_cols, d=extent_y / n_cols)
    KX, KY = np.meshgrid(kx, ky, indexing="ij")
    kappa = math.sqrt(2 * nu) / length_scale
    spec = (kappa * kappa + KX * KX + KY * KY) ** (-(nu + 1.0))
    noise = rng.standard_normal((n_rows, n_cols)) + 1j * rng.standard_normal((n_rows, n_cols))
    f = np.real(np.fft.ifft2(noise * np.sqrt(spec)))
    f -= f.mean()
    sd = f.std()
    return f / sd if sd > 0 else f


def central_sensors(rng: np.random.Generator, n: int, extent_x: float, extent_y: float,
                    frac: float = 0.5, z: float = 0.0) -> np.ndarray:
    """n sensor positions uniform in the central `frac` of the footprint, at height z."""
    lo_x, hi_x = extent_x * (0.5 - frac / 2), extent_x * (0.5 + frac / 2)
    lo_y, hi_y = extent_y * (0.5 - frac / 2), extent_y * (0.5 + frac / 2)
    pos = np.empty((n, 3))
    pos[:, 0] = rng.uniform(lo_x, hi_x, n)
    pos[:, 1] = rng.uniform(lo_y, hi_y, n)
    pos[:, 2] = z
    return pos


def draw_counts(lam: np.ndarray, seed: int, mode: str = "poisson") -> np.ndarray:
    """Observed counts from expected counts `lam` (computed by the caller).

    mode="poisson": numpy PCG64 Poisson draws; mode="round": nearest integer,
    as in the paper's simulation experiment.
    """
    lam = np.asarray(lam, dtype=np.float64)
    if mode == "round":
        return np.rint(lam).astype(np.int32)
    rng = np.random.default_rng(seed)
    return rng.poisson(lam).astype(np.int32)


# ----------------------------------------------------------------------------
# Workload recipes
# ----------------------------------------------------------------------------

def _node_coords(n_rows, n_cols, extent_x, extent_y):
    return np.linspace(0.0, extent_x, n_rows), np.linspace(0.0, extent_y, n_cols)


def tiny_bumps(seed: int = 0, n_grid: int = 16, extent: float = 100.0, n_sensors: int = 2,
               pix_side: int = 32, car_r: float = 0.99) -> Scenario:
    """Small three-surface cave: 16x16 grid over 100 m, muck top/cave back with
    three Gaussian bumps, flat terrain at 200 m, 2 sensors x 32x32 pixels."""
    rng = np.random.default_rng(seed)
    xs, ys = _node_coords(n_grid, n_grid, extent, extent)
    bumps = gaussian_bumps(rng, xs, ys, 3, centre_lo=0.2 * extent, centre_hi=0.8 * extent)
    h1 = 60.0 + 0.5 * bumps
    h2 = 61.0 + bumps
    top = np.full((n_grid, n_grid), 200.0)
    sensors = central_sensors(rng, n_sensors, extent, extent)
    dirs1 = pixel_directions(pix_side, pix_side)
    dirs = np.broadcast_to(dirs1, (n_sensors,) + dirs1.shape).copy()
    return Scenario(
        name=f"tiny_bumps_{n_grid}x{n_grid}_s{n_sensors}_p{pix_side}", n_surfaces=3,
        n_rows=n_grid, n_cols=n_grid, extent_x=extent, extent_y=extent,
        density=np.array(DEFAULT_DENSITY), top=top, car_r=np.full(2, car_r),
        truth=np.stack([h1, h2]), sensor_pos=sensors, dirs=dirs,
        exposure=np.full((n_sensors, dirs1.shape[0]), 1e4), atten_len=400.0, seed=seed)


def grf_cave(seed: int = 10, n_grid: int = 64, extent: float = 400.0, n_sensors: int = 8,
             pix_side: int = 64, car_r: float = 0.99, length_scale: float = 50.0) -> Scenario:
    """Paper-scale three-surface cave from seeded periodic random fields:
    H1 = 80 + 8 G1, H2 = H1 + 1 + 10 max(G2, 0), H3 = 200 + 3 G3 (metres)."""
    rng = np.random.default_rng(seed)
    g = [periodic_grf(rng, n_grid, n_grid, extent, extent, length_scale) for _ in range(3)]
    h1 = 80.0 + 8.0 * g[0]
    h2 = h1 + 1.0 + 10.0 * np.maximum(g[1], 0.0)
    top = 200.0 + 3.0 * g[2]
    sensors = central_sensors(rng, n_sensors, extent, extent)
    dirs1 = pixel_directions(pix_side, pix_side)
    dirs = np.broadcast_to(dirs1, (n_sensors,) + dirs1.shape).copy()
    return Scenario(
        name=f"grf_cave_{n_grid}x{n_grid}_s{n_sensors}_p{pix_side}", n_surfaces=3,
        n_rows=n_grid, n_cols=n_grid, extent_x=extent, extent_y=extent,
        density=np.array(DEFAULT_DENSITY), top=top, car_r=np.full(2, car_r),
        truth=np.stack([h1, h2]), sensor_pos=sensors, dirs=dirs,
        exposure=np.full((n_sensors, dirs1.shape[0]), 1e4), atten_len=400.0, seed=seed)


def heterogeneous_problem_spec(i: int, base_seed: int = 20) -> dict:
    """Sizes of problem i in a heterogeneous batch: grid side in {16,32,64,128}
    over 400 m, 2-16 sensors, pixel side 32-64, chains in {64,128,256,512}."""
    rng = np.random.default_rng(base_seed + i)
    return dict(seed=base_seed + i,
                n_grid=int(rng.choice([16, 32, 64, 128])),
                n_sensors=int(rng.integers(2, 17)),
                pix_side=int(rng.integers(32, 65)),
                n_chains=int(rng.choice([64, 128, 256, 512])))


def heterogeneous_problem(i: int, base_seed: int = 20, scale_pixels: float = 1.0) -> tuple:
    """(Scenario, n_chains) for problem i of a heterogeneous batch."""
    spec = heterogeneous_problem_spec(i, base_seed)
    pix = max(2, int(round(spec["pix_side"] * scale_pixels)))
    sc = grf_cave(seed=spec["seed"], n_grid=spec["n_grid"], n_sensors=spec["n_sensors"], pix_side=pix)
    return sc, spec["n_chains"]


def poisson_arrivals(rate_per_s: float, duration_s: float, seed: int = 40) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate over [0, duration)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t >= duration_s:
            return np.array(out)
        out.append(t)


def init_states(sc: Scenario, n_chains: int, seed: int, jitter: float = 0.3,
                min_gap: float = 0.05) -> np.ndarray:
    """Initial chain states [n_chains, S-1, R, C]: the truth plus independent
    Gaussian jitter, kept strictly ordered inside (0, top)."""
    rng = np.random.default_rng(seed)
    S1 = sc.n_surfaces - 1
    st = sc.truth[None] + jitter * rng.standard_normal((n_chains, S1, sc.n_rows, sc.n_cols))
    lo = np.full((n_chains, sc.n_rows, sc.n_cols), min_gap)
    for l in range(S1):
        st[:, l] = np.maximum(st[:, l], lo)
        lo = st[:, l] + min_gap
    hi = sc.top[None] - min_gap
    for l in reversed(range(S1)):
        st[:, l] = np.minimum(st[:, l], hi)
        hi = st[:, l] - min_gap
    return st


def named_workload(name: str) -> tuple:
    """(Scenario, n_chains) for the named single-problem workloads."""
    if name == "tiny_bumps":
        return tiny_bumps(), 4
    if name == "grf_cave_64":
        return grf_cave(), 1024
    if name == "grf_cave_128":
        return grf_cave(n_grid=128), 512
    raise KeyError(name)
