"""FP64 CPU oracle for the block-cave muon-tomography posterior (arXiv 2603.28907).

TEST INFRASTRUCTURE ONLY.  Imported by `tests/`, by the smoke check in
`__graft_entry__.py` and by the CPU-baseline leg of `bench.py`; the product
path (`paper_2603_28907_amd`) never imports it.  The numerics live in
`muon_oracle.c` (plain C, FP64), compiled with gcc by `build()`; this module
only marshals numpy arrays into it.  It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "muon_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmuon_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over chains)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(ct.Structure):
    _fields_ = [("S", ct.c_int), ("R", ct.c_int), ("C", ct.c_int),
                ("X", ct.c_double), ("Y", ct.c_double),
                ("density", ct.c_void_p), ("top", ct.c_void_p), ("car_r", ct.c_void_p),
                ("n_s", ct.c_int), ("n_pix", ct.c_int),
                ("pos", ct.c_void_p), ("dirs", ct.c_void_p), ("exposure", ct.c_void_p),
                ("atten", ct.c_double), ("counts", ct.c_void_p),
                ("n_z", ct.c_int), ("gamma", ct.c_double), ("vox_ref", ct.c_void_p),
                ("n_sub", ct.c_int), ("sub_w", ct.c_void_p), ("n_tab", ct.c_int), ("tab_omax", ct.c_double),
                ("tab_logI", ct.c_void_p)]


class _Stats(ct.Structure):
    _fields_ = [("cells", ct.c_double), ("tests", ct.c_double), ("roots", ct.c_double),
                ("crossings", ct.c_double), ("min_fprime", ct.c_double), ("gcond", ct.c_void_p),
                ("cond_g", ct.c_double), ("cond_gerr", ct.c_double), ("eps_z", ct.c_double),
                ("eps_rel", ct.c_double), ("eps_w", ct.c_double), ("lid_band", ct.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ct.CDLL(_LIB_PATH)
    P, D, V, I, I64 = ct.POINTER(_Problem), ct.c_double, ct.c_void_p, ct.c_int, ct.c_int64
    U64, U32 = ct.c_uint64, ct.c_uint32
    sig = {
        "orc_opacity": (None, [P, V, V, V, ct.POINTER(_Stats)]),
        "orc_loglik": (D, [P, V]),
        "orc_log_prior": (D, [P, V]),
        "orc_log_prior_grad": (D, [P, V, V]),
        "orc_logpost": (D, [P, V]),
        "orc_logpost_batch": (None, [P, I, V, V]),
        "orc_grad": (D, [P, V, V]),
        "orc_grad_batch": (None, [P, I, V, V, V]),
        "orc_max_threads": (I, []),
        "orc_ndtri_lower": (D, [D]),
        "orc_car_consts": (None, [I, I, D, V, V]),
        "orc_philox4x32_10": (None, [V, V, V]),
        "orc_uniform_pair": (None, [U64, U32, U64, U32, U32, V]),
        "orc_normal_pair": (None, [U64, U32, U64, U32, U32, V]),
        "orc_raw_philox": (None, [U64, U32, U64, U32, U32, V]),
        "orc_mcmc_rw": (None, [P, I, V, V, V, I64, U64, D, U64, I, V]),
        "orc_mcmc_rw_r": (None, [P, I, V, V, V, V, V, I64, U64, D, D, U64, I, V]),
        "orc_log_prior_r": (D, [P, V, V]),
        "orc_mcmc_mala": (None, [P, I, V, V, V, I64, U64, D, V, U64, I, V]),
        "orc_march_one": (D, [P, V, V, V, V, ct.POINTER(_Stats)]),
        "orc_ray_stats": (None, [P, V, V, V, V]),
        "orc_grad_conditioning": (None, [P, V, D, D, D, D, V, D, V, V, V]),
        "orc_sigmoid": (D, [D, D]),
        "orc_voxel_weights": (None, [P, V, I, D, V]),
        "orc_voxel_density": (None, [P, V, I, D, V]),
        "orc_voxel_pieces": (I, [P, I, I, V, V]),
        "orc_voxel_loglik": (D, [P, V, V]),
        "orc_voxel_logpost_lik": (D, [P, V, V]),
        "orc_nuts": (None, [P, ct.c_size_t, V, I, I, V, V, V, V, I, D, I64, I64, D, U64, U64, I, V, V, V, V, V]),
        "orc_latent_to_heights": (None, [P, V, V]),
        "orc_log_intensity": (D, [P, D]),
        "orc_quad_loglik": (D, [P, V, V]),
        "orc_heights_to_latent": (None, [P, V, V]),
        "orc_latent_logpost_grad": (D, [P, V, V]),
        "orc_latent_r_logpost_grad": (D, [P, V, V]),
        "orc_nested_rhat": (None, [I, I, ct.c_size_t, V, V]),
        "orc_nuts_dense": (None, [ct.c_size_t, V, I, V, D, V, I, D, I64, U64, U64, V, V, V, V, V, V]),
        "orc_nuts_set_fault": (None, [I]),
        "orc_warmup_window_end": (I, [I64, I64]),
        "orc_warmup_in_slow": (I, [I64, I64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """One problem (geometry + sensors + counts) bound to the C oracle.

    Accepts any object with the attributes of `paper_2603_28907_amd.inputs.Scenario`.
    """

    def __init__(self, sc, counts: Optional[np.ndarray] = None, density=None, car_r=None,
                 atten_len: Optional[float] = None):
        self.lib = _load()
        self.S, self.R, self.C = int(sc.n_surfaces), int(sc.n_rows), int(sc.n_cols)
        self._density = _f64(sc.density if density is None else density)
        self._top = _f64(sc.top)
        self._car_r = _f64(sc.car_r if car_r is None else car_r)
        self._pos = _f64(sc.sensor_pos).reshape(-1, 3)
        n_s = self._pos.shape[0]
        self._dirs = _f64(sc.dirs).reshape(n_s, -1, 3) if n_s else np.zeros((0, 0, 3))
        n_pix = self._dirs.shape[1] if n_s else 0
        self._exp = _f64(sc.exposure).reshape(n_s, n_pix) if n_s else np.zeros((0, 0))
        c = counts if counts is not None else sc.counts
        self._counts = (np.ascontiguousarray(c, dtype=np.int32).reshape(n_s, n_pix)
                        if c is not None else np.zeros((n_s, n_pix), np.int32))
        self.n_rays = n_s * n_pix
        self.prob = _Problem(self.S, self.R, self.C, float(sc.extent_x), float(sc.extent_y),
                             _p(self._density), _p(self._top), _p(self._car_r), n_s, n_pix,
                             _p(self._pos), _p(self._dirs), _p(self._exp),
                             float(sc.atten_len if atten_len is None else atten_len),
                             _p(self._counts))
        self.M = (self.S - 1) * self.R * self.C

    def _free(self, free) -> np.ndarray:
        f = _f64(free)
        assert f.size == self.M, (f.shape, self.M)
        return f

    def opacity(self, free, with_lengths: bool = False, with_stats: bool = False):
        f = self._free(free)
        O = np.empty(self.n_rays)
        L = np.empty((self.n_rays, self.S)) if with_lengths else None
        st = _Stats()
        self.lib.orc_opacity(ct.byref(self.prob), _p(f), _p(O), _p(L), ct.byref(st))
        out = [O]
        if with_lengths:
            out.append(L)
        if with_stats:
            out.append(dict(cells=st.cells, tests=st.tests, roots=st.roots,
                            crossings=st.crossings, min_fprime=st.min_fprime))
        return out[0] if len(out) == 1 else tuple(out)

    # -- the paper's smoothed voxel forward model, linearised ----------------
    def _surf(self, free) -> np.ndarray:
        return np.concatenate([self._free(free).reshape(self.S - 1, self.R, self.C), self._top[None]])

    def voxel_weights(self, free, n_z: int, gamma: float = 1.0) -> np.ndarray:
        """Normalised weights [R, C, n_z, S+1] (units 1..S, then the air)."""
        W = np.empty((self.R, self.C, n_z, self.S + 1))
        self.lib.orc_voxel_weights(ct.byref(self.prob), _p(self._surf(free)), int(n_z), float(gamma), _p(W))
        return W

    def voxel_density(self, free, n_z: int, gamma: float = 1.0) -> np.ndarray:
        R = np.empty((self.R, self.C, n_z))
        self.lib.orc_voxel_density(ct.byref(self.prob), _p(self._surf(free)), int(n_z), float(gamma), _p(R))
        return R

    def voxel_pieces(self, ray: int, n_z: int):
        cap = self.R + self.C + n_z + 1
        vox = np.empty(cap, np.int32)
        ln = np.empty(cap)
        m = self.lib.orc_voxel_pieces(ct.byref(self.prob), int(ray), int(n_z), _p(vox), _p(ln))
        return vox[:m].copy(), ln[:m].copy()

    def set_voxel_model(self, n_z: int, gamma: float = 1.0, ref_free=None):
        """Switch the likelihood to the linearised voxel model around
        R0 = Rhat(ref_free); n_z = 0 switches back to the exact march."""
        if n_z <= 0:
            self.prob.n_z, self.prob.gamma, self.prob.vox_ref = 0, 0.0, None
            self._vox_ref = None
            return
        self._vox_ref = np.ascontiguousarray(self.voxel_density(ref_free, n_z, gamma))
        self.prob.n_z, self.prob.gamma = int(n_z), float(gamma)
        self.prob.vox_ref = _p(self._vox_ref)

    def set_pixel_quadrature(self, n_sub, weights, log_intensity, o_max, pixel_counts):
        """Solid-angle pixels: this problem's rays become sub-rays, n_sub per pixel
        with quadrature weights [n_rays]; log I tabulated over [0, o_max];
        counts per pixel [n_rays / n_sub]."""
        self._sub_w = _f64(weights).reshape(-1)
        self._tab = _f64(log_intensity).reshape(-1)
        self._counts = np.ascontiguousarray(pixel_counts, dtype=np.int32).reshape(-1)
        assert self._sub_w.size == self.n_rays and self._counts.size * n_sub == self.n_rays
        self.prob.n_sub, self.prob.sub_w = int(n_sub), _p(self._sub_w)
        self.prob.n_tab, self.prob.tab_omax, self.prob.tab_logI = self._tab.size, float(o_max), _p(self._tab)
        self.prob.counts = _p(self._counts)

    def log_intensity(self, O):
        return np.array([self.lib.orc_log_intensity(ct.byref(self.prob), float(o)) for o in np.ravel(O)])

    def pixel_lambda(self, free):
        """Expected counts per pixel under the solid-angle quadrature."""
        O = self.opacity(free)
        lam = np.empty(self.n_rays // self.prob.n_sub)
        self.lib.orc_quad_loglik(ct.byref(self.prob), _p(O), _p(lam))
        return lam

    def voxel_loglik(self, free, with_opacity: bool = False):
        O = np.empty(self.n_rays)
        ll = self.lib.orc_voxel_logpost_lik(ct.byref(self.prob), _p(self._free(free)), _p(O))
        return (float(ll), O) if with_opacity else float(ll)

    def expected_counts(self, free) -> np.ndarray:
        O = self.opacity(free)
        return self._exp.reshape(-1) * np.exp(-O / self.prob.atten)

    def loglik(self, O) -> float:
        O = _f64(O)
        return float(self.lib.orc_loglik(ct.byref(self.prob), _p(O)))

    def log_prior(self, free) -> float:
        return float(self.lib.orc_log_prior(ct.byref(self.prob), _p(self._free(free))))

    def log_prior_r(self, free, r) -> float:
        """log p(H | r) with the per-surface dependence parameters r[S-1] given."""
        return float(self.lib.orc_log_prior_r(ct.byref(self.prob), _p(self._free(free)), _p(_f64(r))))

    def log_prior_grad(self, free):
        g = np.zeros((self.S, self.R, self.C))
        v = self.lib.orc_log_prior_grad(ct.byref(self.prob), _p(self._free(free)), _p(g))
        return float(v), g

    def logpost(self, free) -> float:
        return float(self.lib.orc_logpost(ct.byref(self.prob), _p(self._free(free))))

    def logpost_batch(self, states) -> np.ndarray:
        s = _f64(states)
        n = s.size // self.M
        lp = np.empty(n)
        self.lib.orc_logpost_batch(ct.byref(self.prob), n, _p(s), _p(lp))
        return lp

    def grad(self, free):
        g = np.empty((self.S, self.R, self.C))
        lp = self.lib.orc_grad(ct.byref(self.prob), _p(self._free(free)), _p(g))
        return float(lp), g

    def grad_batch(self, states):
        s = _f64(states)
        n = s.size // self.M
        lp = np.empty(n)
        g = np.empty((n, self.S, self.R, self.C))
        self.lib.orc_grad_batch(ct.byref(self.prob), n, _p(s), _p(lp), _p(g))
        return lp, g

    def march_one(self, free, q, d):
        L = np.empty(self.S)
        st = _Stats()
        O = self.lib.orc_march_one(ct.byref(self.prob), _p(self._free(free)), _p(_f64(q)),
                                   _p(_f64(d)), _p(L), ct.byref(st))
        return float(O), L, dict(cells=st.cells, tests=st.tests, roots=st.roots,
                                 crossings=st.crossings, min_fprime=st.min_fprime)

    def ray_stats(self, free):
        cr, mf, ce = np.empty(self.n_rays), np.empty(self.n_rays), np.empty(self.n_rays)
        self.lib.orc_ray_stats(ct.byref(self.prob), _p(self._free(free)), _p(cr), _p(mf), _p(ce))
        return dict(crossings=cr, min_fprime=mf, cells=ce)

    def grad_conditioning(self, free, eps_z, eps_rel, eps_w=0.0, lid_band=0.0, dO=None, o_rel=1e-5, g=None,
                          g_err=None):
        """Per-node bound [S, R, C] on how far an evaluation of the likelihood
        gradient that rounds z - h by eps_z, each contribution by eps_rel and
        each bilinear weight by eps_w, drops crossings within lid_band of the
        box lid, with opacity errors dO per ray (or the bound o_rel |O| + ...),
        can move (see orc_grad_conditioning).  g, g_err [n_rays]: dL/dO of each
        ray and its error, given in place of the one-ray model's."""
        out = np.empty((self.S, self.R, self.C))
        d = None if dO is None else _f64(dO)
        if (g is None) != (g_err is None):
            raise ValueError("g and g_err go together")
        gr = None if g is None else _f64(g)
        ge = None if g_err is None else _f64(g_err)
        for a in (gr, ge):
            if a is not None and a.size != self.n_rays:
                raise ValueError("g and g_err take one value per ray")
        self.lib.orc_grad_conditioning(ct.byref(self.prob), _p(self._free(free)), float(eps_z), float(eps_rel),
                                       float(eps_w), float(lid_band), _p(d), float(o_rel), _p(gr), _p(ge),
                                       _p(out))
        return out

    def mcmc_rw(self, states, lp, n_accept, n_steps, step_offset, sigma, seed,
                state_f32=False, want_margins=False):
        """Runs in place on float64 copies; returns (states, lp, n_accept, margins)."""
        s = _f64(states).copy()
        n = s.size // self.M
        lpa = _f64(lp).copy()
        acc = np.ascontiguousarray(n_accept, dtype=np.int64).copy()
        marg = np.empty((n, n_steps)) if want_margins else None
        self.lib.orc_mcmc_rw(ct.byref(self.prob), n, _p(s), _p(lpa), _p(acc), int(n_steps),
                             int(step_offset), float(sigma), int(seed), int(bool(state_f32)), _p(marg))
        return s.reshape(np.shape(states)), lpa, acc, marg

    def mcmc_rw_r(self, states, r, lp, n_accept, n_steps, step_offset, sigma, tau, seed, n_accept_r=None,
                  state_f32=False, want_margins=False):
        """RW on H with Metropolis-within-Gibbs updates of r (logit scale, step tau).
        Returns (states, r, lp, n_accept, n_accept_r, margins [n, n_steps, S])."""
        s = _f64(states).copy()
        n = s.size // self.M
        rr = _f64(r).reshape(n, self.S - 1).copy()
        lpa = _f64(lp).copy()
        acc = np.ascontiguousarray(n_accept, dtype=np.int64).copy()
        accr = (np.zeros((n, self.S - 1), np.int64) if n_accept_r is None
                else np.ascontiguousarray(n_accept_r, dtype=np.int64).reshape(n, self.S - 1).copy())
        marg = np.empty((n, n_steps, self.S)) if want_margins else None
        self.lib.orc_mcmc_rw_r(ct.byref(self.prob), n, _p(s), _p(rr), _p(lpa), _p(acc), _p(accr), int(n_steps),
                               int(step_offset), float(sigma), float(tau), int(seed), int(bool(state_f32)), _p(marg))
        return s.reshape(np.shape(states)), rr, lpa, acc, accr, marg

    def nuts(self, states, lp, eps, inv_mass=None, max_depth=8, max_dh=1000.0, n_warmup=0, n_steps=1,
             target_accept=0.8, seed=0, step_offset=0, state_f32=False, latent=False, r=None):
        """NUTS on this posterior; states [n, S-1, R, C] (heights, or the latent CAR fields with
        latent=True); eps [n]; inv_mass [n, S-1, R, C] or None.  With r [n, S-1] (latent only) the
        chains also sample r: the state is (x, logit r), inv_mass is [n, (S-1) R C + S-1], and
        out["r"] holds the final r."""
        n = np.shape(states)[0]
        if r is None:
            s = _f64(states).reshape(-1, self.M)
            im = None if inv_mass is None else _f64(inv_mass).reshape(-1, self.M)
            out = _nuts_call(ct.byref(self.prob), self.M, None, s, lp, eps, im, max_depth, max_dh, n_warmup,
                             n_steps, target_accept, seed, step_offset, state_f32, latent)
            out["x"] = out["x"].reshape(np.shape(states))
            if im is not None:
                out["inv_mass"] = out["inv_mass"].reshape(np.shape(states))
            return out
        assert latent, "r is sampled on the latent parametrisation"
        S1 = self.S - 1
        ra = _f64(r).reshape(n, S1)
        z = np.concatenate([_f64(states).reshape(n, self.M), np.log(ra / (1.0 - ra))], axis=1)
        im = None if inv_mass is None else _f64(inv_mass).reshape(n, self.M + S1)
        out = _nuts_call(ct.byref(self.prob), self.M + S1, None, z, lp, eps, im, max_depth, max_dh, n_warmup,
                         n_steps, target_accept, seed, step_offset, state_f32, 2)
        zf = out["x"]
        out["x"] = zf[:, :self.M].reshape(np.shape(states))
        out["r"] = 1.0 / (1.0 + np.exp(-zf[:, self.M:]))
        return out

    def latent_r_logpost(self, x, r, with_grad=False):
        """Log density of the latent vector (x, logit r) and optionally its
        gradient (x part [S-1, R, C], logit-r part [S-1])."""
        S1 = self.S - 1
        z = np.concatenate([_f64(x).reshape(-1), np.log(_f64(r) / (1.0 - _f64(r)))])
        g = np.empty(z.size) if with_grad else None
        v = float(self.lib.orc_latent_r_logpost_grad(ct.byref(self.prob), _p(z), _p(g)))
        if not with_grad:
            return v
        return v, g[:self.M].reshape(S1, self.R, self.C), g[self.M:].copy()

    def latent_to_heights(self, x):
        x = _f64(x).reshape(-1, self.M)
        H = np.empty_like(x)
        for c in range(x.shape[0]):
            self.lib.orc_latent_to_heights(ct.byref(self.prob), _p(x[c]), _p(H[c]))
        return H.reshape(-1, self.S - 1, self.R, self.C)

    def heights_to_latent(self, H):
        H = _f64(H).reshape(-1, self.M)
        x = np.empty_like(H)
        for c in range(H.shape[0]):
            self.lib.orc_heights_to_latent(ct.byref(self.prob), _p(H[c]), _p(x[c]))
        return x.reshape(-1, self.S - 1, self.R, self.C)

    def latent_logpost(self, x, with_grad=False):
        x = self._free(x)
        g = np.empty(self.M) if with_grad else None
        lp = float(self.lib.orc_latent_logpost_grad(ct.byref(self.prob), _p(x), _p(g)))
        return (lp, g.reshape(self.S - 1, self.R, self.C)) if with_grad else lp

    def mcmc_mala(self, states, lp, n_accept, n_steps, step_offset, eps, seed, inv_mass=None,
                  state_f32=False, want_margins=False):
        s = _f64(states).copy()
        n = s.size // self.M
        lpa = _f64(lp).copy()
        acc = np.ascontiguousarray(n_accept, dtype=np.int64).copy()
        marg = np.empty((n, n_steps)) if want_margins else None
        im = None if inv_mass is None else _f64(inv_mass)
        self.lib.orc_mcmc_mala(ct.byref(self.prob), n, _p(s), _p(lpa), _p(acc), int(n_steps),
                               int(step_offset), float(eps), _p(im), int(seed),
                               int(bool(state_f32)), _p(marg))
        return s.reshape(np.shape(states)), lpa, acc, marg


def _nuts_call(prob, n_dim, sd, x, lp, eps, inv_mass, max_depth, max_dh, n_warmup, n_steps, target_accept, seed,
               step_offset, state_f32, latent=False):
    lib = _load()
    n = x.shape[0]
    x = _f64(x).copy()
    lpa = _f64(lp).copy()
    ea = _f64(eps).copy()
    im = None if inv_mass is None else _f64(inv_mass).copy()
    total = n_warmup + n_steps
    depth = np.zeros((n, total), np.int32)
    nl = np.zeros((n, total), np.int32)
    dv = np.zeros((n, total), np.int32)
    acc = np.zeros((n, total))
    marg = np.zeros(n)
    lib.orc_nuts(prob, int(n_dim), _p(sd), int(latent), n, _p(x), _p(lpa), _p(ea), _p(im), int(max_depth),
                 float(max_dh),
                 int(n_warmup), int(n_steps), float(target_accept), int(seed), int(step_offset), int(bool(state_f32)),
                 _p(depth), _p(nl), _p(dv), _p(acc), _p(marg))
    return dict(x=x, lp=lpa, eps=ea, inv_mass=im, depth=depth, n_leap=nl, diverged=dv, accept_stat=acc,
                margin=marg)


def nuts_gauss(sd, x0, eps, inv_mass=None, max_depth=8, max_dh=1000.0, n_warmup=0, n_steps=1,
               target_accept=0.8, seed=0, step_offset=0):
    """NUTS on the test target N(0, diag(sd^2)); x0: [n_chains, dim]."""
    sd = _f64(sd)
    x0 = _f64(x0)
    return _nuts_call(None, sd.size, sd, x0, np.full(x0.shape[0], np.nan), eps, inv_mass, max_depth, max_dh,
                      n_warmup, n_steps, target_accept, seed, step_offset, False)


def nuts_dense(prec, x0, eps, inv_mass=None, max_depth=8, max_dh=1000.0, n_steps=1, seed=0, step_offset=0):
    """n_steps NUTS transitions at step size eps on the test target
    N(0, prec^-1) (dense precision matrix); x0: [n_chains, dim], chain c uses
    Philox chain index c; inv_mass: [dim] shared by the chains, or None."""
    lib = _load()
    prec = _f64(prec)
    x = _f64(x0).copy()
    n, M = x.shape
    assert prec.shape == (M, M)
    im = None if inv_mass is None else _f64(inv_mass)
    out = {k: np.zeros((n, n_steps), np.int32) for k in ("depth", "n_leap", "diverged", "turned")}
    acc = np.zeros((n, n_steps))
    marg = np.zeros(n)
    lib.orc_nuts_dense(M, _p(prec), n, _p(x), float(eps), _p(im), int(max_depth), float(max_dh), int(n_steps),
                       int(seed), int(step_offset), _p(out["depth"]), _p(out["n_leap"]), _p(out["diverged"]),
                       _p(out["turned"]), _p(acc), _p(marg))
    return dict(x=x, accept_stat=acc, margin=marg, **out)


def set_nuts_fault(flags: int) -> None:
    """Plant a mistake in the oracle's NUTS (tests of the pins' power only):
    bit 0 skips the U-turn checks inside subtrees, bit 1 merges subtrees that
    turned inside.  0 restores the correct sampler."""
    _load().orc_nuts_set_fault(int(flags))


def nested_rhat(x, n_super, n_within):
    """Nested R-hat per coordinate from one draw per chain; x: [n_super*n_within, dim]."""
    x = _f64(x)
    x2 = x.reshape(x.shape[0], -1)
    out = np.empty(x2.shape[1])
    _load().orc_nested_rhat(int(n_super), int(n_within), x2.shape[1], _p(x2), _p(out))
    return out.reshape(x.shape[1:])


def warmup_window_ends(n_warmup):
    lib = _load()
    return [k for k in range(n_warmup) if lib.orc_warmup_window_end(int(n_warmup), k)]


def ndtri_lower(u: float) -> float:
    return float(_load().orc_ndtri_lower(float(u)))


def car_consts(R: int, C: int, r: float):
    a, b = ct.c_double(), ct.c_double()
    _load().orc_car_consts(int(R), int(C), float(r), ct.byref(a), ct.byref(b))
    return a.value, b.value


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    _load().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def raw_philox(seed, chain, step, tag, j) -> np.ndarray:
    out = np.empty(4, np.uint32)
    _load().orc_raw_philox(int(seed), int(chain), int(step), int(tag), int(j), _p(out))
    return out


def uniform_pair(seed, chain, step, tag, j) -> np.ndarray:
    out = np.empty(2)
    _load().orc_uniform_pair(int(seed), int(chain), int(step), int(tag), int(j), _p(out))
    return out


def normal_pair(seed, chain, step, tag, j) -> np.ndarray:
    out = np.empty(2)
    _load().orc_normal_pair(int(seed), int(chain), int(step), int(tag), int(j), _p(out))
    return out


def max_threads() -> int:
    """OpenMP threads the oracle's batch calls use."""
    return int(_load().orc_max_threads())


def make_counts(sc, seed: int, mode: str = "poisson") -> np.ndarray:
    """Observed counts for a scenario: expected counts of the true surfaces from
    the oracle's forward model, then a seeded draw (inputs.draw_counts)."""
    from paper_2603_28907_amd.inputs import draw_counts
    lam = OracleProblem(sc).expected_counts(sc.truth)
    return draw_counts(lam, seed, mode).reshape(sc.n_sensors, sc.n_pix)
