"""Thin ctypes binding over the muoncave C ABI (include/muoncave.h).

Argument marshalling only: every numerical step runs in the HIP library.
Device buffers are torch tensors (PyTorch supplies device memory and streams);
the library must be built (``python -m paper_2603_28907_amd.build``) and the
binding raises if it is missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmuoncave.so")

MC_F32, MC_F64 = 0, 1
KERNEL_RW, KERNEL_MALA = 0, 1
_STATUS = {0: "MC_OK", -1: "MC_ERR_ARG", -2: "MC_ERR_STATE", -3: "MC_ERR_NOMEM",
           -4: "MC_ERR_DEVICE", -5: "MC_ERR_UNSUPPORTED"}

_lib = None


class MuonCaveError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Tuning(ct.Structure):
    _fields_ = [("march_variant", ct.c_int), ("block", ct.c_int),
                ("rays_per_thread", ct.c_int), ("top_in_lds", ct.c_int), ("multi_blocks_per_cu", ct.c_int),
                ("grad_slots", ct.c_int), ("adjoint_rows", ct.c_int)]


class RunConfig(ct.Structure):
    _fields_ = [("kernel", ct.c_int), ("n_steps", ct.c_int64), ("graph_steps", ct.c_int),
                ("step_size", ct.c_double), ("inv_mass", ct.c_void_p), ("seed", ct.c_uint64),
                ("step_offset", ct.c_uint64), ("r_state", ct.c_void_p), ("r_step", ct.c_double),
                ("n_accept_r", ct.c_void_p)]


class NutsConfig(ct.Structure):
    _fields_ = [("n_warmup", ct.c_int64), ("n_steps", ct.c_int64), ("max_depth", ct.c_int), ("adapt_mass", ct.c_int),
                ("max_delta_h", ct.c_double), ("target_accept", ct.c_double), ("seed", ct.c_uint64),
                ("step_offset", ct.c_uint64), ("latent", ct.c_int), ("r_state", ct.c_void_p)]


class ServerConfig(ct.Structure):
    _fields_ = [("device", ct.c_int), ("precision", ct.c_int), ("memory_budget", ct.c_size_t),
                ("reserve", ct.c_size_t), ("max_jobs", ct.c_int), ("steps_per_round", ct.c_int)]


class JobDesc(ct.Structure):
    _fields_ = [("n_surfaces", ct.c_int), ("n_rows", ct.c_int), ("n_cols", ct.c_int),
                ("extent_x", ct.c_double), ("extent_y", ct.c_double),
                ("density", ct.c_void_p), ("top", ct.c_void_p), ("car_r", ct.c_void_p),
                ("n_sensors", ct.c_int), ("n_pix", ct.c_int),
                ("sensor_pos", ct.c_void_p), ("dirs", ct.c_void_p), ("exposure", ct.c_void_p),
                ("atten_len", ct.c_double), ("counts", ct.c_void_p),
                ("n_chains", ct.c_int), ("init", ct.c_void_p), ("n_steps", ct.c_int64),
                ("step_size", ct.c_double), ("seed", ct.c_uint64),
                ("block", ct.c_int), ("rays_per_thread", ct.c_int), ("r_step", ct.c_double)]


class JobInfo(ct.Structure):
    _fields_ = [("status", ct.c_int), ("map_chain", ct.c_int), ("steps_done", ct.c_int64),
                ("t_submit", ct.c_double), ("t_admit", ct.c_double), ("t_done", ct.c_double),
                ("accept_rate", ct.c_double), ("map_logpost", ct.c_double), ("footprint", ct.c_size_t),
                ("r_mean", ct.c_double * 3), ("r_accept_rate", ct.c_double)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("admitted", ct.c_int64), ("done", ct.c_int64),
                ("failed", ct.c_int64), ("rounds", ct.c_int64), ("resident", ct.c_int),
                ("queued", ct.c_int), ("max_resident", ct.c_int), ("bytes_in_use", ct.c_size_t),
                ("peak_bytes", ct.c_size_t), ("budget", ct.c_size_t), ("busy_seconds", ct.c_double),
                ("now", ct.c_double)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


def load_library(path: Optional[str] = None):
    """Load libmuoncave.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    # PyTorch brings its own HIP runtime; load it first so that this library
    # binds to the same one (a second runtime loaded first leaves torch
    # without devices)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2603_28907_amd.build`")
    lib = ct.CDLL(path)
    V, I, D, P = ct.c_void_p, ct.c_int, ct.c_double, ct.POINTER
    sigs = {
        "mc_create": (I, [I, I, P(V)]),
        "mc_destroy": (None, [V]),
        "mc_last_error": (ct.c_char_p, [V]),
        "load_geometry_grid": (I, [V, I, I, I, D, D, V, V, V]),
        "set_sensors": (I, [V, I, V, I, V, V, D]),
        "set_counts": (I, [V, V]),
        "logpost_batch": (I, [V, I, V, V, V, V]),
        "logpost_batch_noalloc": (I, [V, I, V, V, V, V]),
        "logpost_grad_batch": (I, [V, I, V, V, V, V]),
        "mcmc_run": (I, [V, P(RunConfig), I, V, V, V, V]),
        "mc_debug_philox": (I, [I, ct.c_uint64, ct.c_uint32, ct.c_uint64, ct.c_uint32, ct.c_uint32, I, V, V]),
        "mc_version": (ct.c_char_p, []),
        "mc_time_march": (I, [V, I, V, I, V, P(ct.c_float)]),
        "mc_set_tuning": (I, [V, P(Tuning)]),
        "mc_get_tuning": (I, [V, P(Tuning)]),
        "mcmc_run_multi": (I, [I, P(V), P(RunConfig), P(I), P(V), P(V), P(V), V]),
        "mc_measure_valu_rate": (I, [I, I, P(D)]),
        "mc_time_adjoint": (I, [V, I, V, I, V, P(ct.c_float)]),
        "set_voxel_model": (I, [V, I, D, V]),
        "mc_time_voxel": (I, [V, I, V, I, V, P(ct.c_float), P(ct.c_float)]),
        "mc_voxel_info": (I, [V, P(I), P(ct.c_int64)]),
        "set_pixel_quadrature": (I, [V, I, V, I, D, V]),
        "nuts_run": (I, [V, P(NutsConfig), I, V, V, V, V, V, V, V, V, V]),
        "nested_rhat": (I, [V, I, I, V, V, V]),
        "latent_to_heights": (I, [V, I, V, V, V]),
        "heights_to_latent": (I, [V, I, V, V, V]),
        "mc_server_create": (I, [P(ServerConfig), P(V)]),
        "mc_server_destroy": (None, [V, I]),
        "mc_server_last_error": (ct.c_char_p, [V]),
        "mc_server_submit": (I, [V, P(JobDesc), P(ct.c_int64)]),
        "mc_server_poll": (I, [V, ct.c_int64, P(JobInfo), V, V, V]),
        "mc_server_release": (I, [V, ct.c_int64]),
        "mc_server_wait_idle": (I, [V, D]),
        "mc_server_get_stats": (I, [V, P(ServerStats)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED_SYMBOLS = ("mc_create", "mc_destroy", "mc_last_error", "load_geometry_grid", "set_sensors",
                    "set_counts", "logpost_batch", "logpost_grad_batch", "mcmc_run", "mc_debug_philox",
                    "mc_version", "mc_time_march", "mc_set_tuning", "mc_get_tuning", "mcmc_run_multi",
                    "mc_server_create", "mc_server_destroy", "mc_server_last_error", "mc_server_submit",
                    "mc_server_poll", "mc_server_release", "mc_server_wait_idle", "mc_server_get_stats",
                    "mc_measure_valu_rate", "mc_time_adjoint", "set_voxel_model", "mc_time_voxel", "mc_voxel_info",
                    "nuts_run", "nested_rhat", "latent_to_heights", "heights_to_latent",
                    "set_pixel_quadrature", "logpost_batch_noalloc")


def _host(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ct.c_void_p(stream.cuda_stream)


class Problem:
    """One inference problem on one GPU (an mc_problem handle)."""

    def __init__(self, device: int = 0, precision: str = "f32"):
        self.lib = load_library()
        self.device = int(device)
        self.precision = precision
        self.prec = MC_F64 if precision == "f64" else MC_F32
        h = ct.c_void_p()
        st = self.lib.mc_create(self.device, self.prec, ct.byref(h))
        if st != 0:
            raise MuonCaveError(st, self.lib.mc_last_error(None).decode())
        self.h = h
        self.S = self.R = self.C = 0
        self.n_rays = 0

    # -- errors -------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise MuonCaveError(st, self.lib.mc_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.prec == MC_F64 else torch.float32

    # -- launch shape -------------------------------------------------------
    def set_tuning(self, march_variant=4, block=256, rays_per_thread=16, top_in_lds=0,
                   multi_blocks_per_cu=0, grad_slots=0, adjoint_rows=0):
        t = Tuning(int(march_variant), int(block), int(rays_per_thread), int(top_in_lds),
                   int(multi_blocks_per_cu), int(grad_slots), int(adjoint_rows))
        self._check(self.lib.mc_set_tuning(self.h, ct.byref(t)))

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(self.lib.mc_get_tuning(self.h, ct.byref(t)))
        return {f: getattr(t, f) for f, _ in Tuning._fields_}

    # -- set-up ---------------------------------------------------------------
    def load_geometry_grid(self, n_surfaces, n_rows, n_cols, extent_x, extent_y, density, top, car_r):
        d, t, r = _host(density), _host(top), _host(car_r)
        self._check(self.lib.load_geometry_grid(self.h, int(n_surfaces), int(n_rows), int(n_cols),
                                                float(extent_x), float(extent_y), _hp(d), _hp(t), _hp(r)))
        self.S, self.R, self.C = int(n_surfaces), int(n_rows), int(n_cols)

    def set_sensors(self, pos, dirs, exposure, atten_len):
        pos = _host(pos).reshape(-1, 3)
        n_s = pos.shape[0]
        dirs = _host(dirs).reshape(n_s, -1, 3) if n_s else np.zeros((0, 0, 3))
        n_pix = dirs.shape[1] if n_s else 0
        e = _host(exposure).reshape(n_s, n_pix) if n_s else np.zeros((0, 0))
        self._check(self.lib.set_sensors(self.h, n_s, _hp(pos), n_pix, _hp(dirs), _hp(e), float(atten_len)))
        self.n_rays = n_s * n_pix

    def set_counts(self, counts):
        c = _host(counts, np.int32).reshape(-1)
        self._check(self.lib.set_counts(self.h, _hp(c)))

    def set_voxel_model(self, n_z: int, gamma: float = 1.0, ref_heights=None):
        """Switch the likelihood to the paper's smoothed voxel model linearised
        around R-hat(ref_heights) [S-1, R, C]; n_z = 0 switches back."""
        if n_z == 0:
            self._check(self.lib.set_voxel_model(self.h, 0, 0.0, None))
            return
        ref = _host(ref_heights).reshape(-1)
        if ref.size != (self.S - 1) * self.R * self.C:
            raise ValueError("ref_heights must hold (S-1)*R*C values")
        self._check(self.lib.set_voxel_model(self.h, int(n_z), float(gamma), _hp(ref)))

    def set_pixel_quadrature(self, n_sub: int, weights=None, log_intensity=None, o_max: float = 0.0):
        """Solid-angle pixels: n_sub consecutive rays per pixel with quadrature weights [n_rays] and log I
        tabulated over [0, o_max]; set_counts then takes one count per pixel.  n_sub = 0 switches back."""
        if n_sub == 0:
            self._check(self.lib.set_pixel_quadrature(self.h, 0, None, 0, 0.0, None))
            return
        w = _host(weights).reshape(-1)
        t = _host(log_intensity).reshape(-1)
        if w.size != self.n_rays:
            raise ValueError("one weight per ray")
        self._check(self.lib.set_pixel_quadrature(self.h, int(n_sub), _hp(w), int(t.size), float(o_max), _hp(t)))

    def voxel_info(self):
        """(levels, ray-voxel pieces) of the voxel model; (0, 0) when it is off."""
        nz, npc = ct.c_int(), ct.c_int64()
        self._check(self.lib.mc_voxel_info(self.h, ct.byref(nz), ct.byref(npc)))
        return int(nz.value), int(npc.value)

    @classmethod
    def from_scenario(cls, sc, counts=None, device: int = 0, precision: str = "f32"):
        p = cls(device, precision)
        p.load_geometry_grid(sc.n_surfaces, sc.n_rows, sc.n_cols, sc.extent_x, sc.extent_y, sc.density,
                             sc.top, sc.car_r)
        p.set_sensors(sc.sensor_pos, sc.dirs, sc.exposure, sc.atten_len)
        c = counts if counts is not None else sc.counts
        if p.n_rays:
            if c is None:
                raise ValueError("scenario has no counts")
            p.set_counts(c)
        return p

    # -- device calls ---------------------------------------------------------
    def _check_tensor(self, t, shape, dtype, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.device.index != self.device:
            raise ValueError(f"{name} is on cuda:{t.device.index}, the problem on cuda:{self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def heights_shape(self, n_chains):
        return (n_chains, self.S - 1, self.R, self.C)

    def logpost_batch(self, heights, logpost=None, opacity=None, stream=None):
        import torch
        n = int(heights.shape[0])
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        if logpost is None:
            logpost = torch.empty(n, dtype=torch.float64, device=heights.device)
        self._check_tensor(logpost, (n,), torch.float64, "logpost")
        if opacity is not None:
            self._check_tensor(opacity, (n, self.n_rays), self.torch_dtype, "opacity")
        self._check(self.lib.logpost_batch(self.h, n, ct.c_void_p(heights.data_ptr()),
                                           ct.c_void_p(logpost.data_ptr()),
                                           ct.c_void_p(opacity.data_ptr()) if opacity is not None else None,
                                           _stream_handle(stream, self.device)))
        return logpost

    def logpost_batch_noalloc(self, heights, logpost, opacity=None, stream=None):
        """logpost_batch through the allocation-free entry point: the caller
        passes every output (the library's workspace is a fixed per-device
        array)."""
        n = int(heights.shape[0])
        import torch
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        self._check_tensor(logpost, (n,), torch.float64, "logpost")
        if opacity is not None:
            self._check_tensor(opacity, (n, self.n_rays), self.torch_dtype, "opacity")
        self._check(self.lib.logpost_batch_noalloc(self.h, n, ct.c_void_p(heights.data_ptr()),
                                                   ct.c_void_p(logpost.data_ptr()),
                                                   ct.c_void_p(opacity.data_ptr()) if opacity is not None else None,
                                                   _stream_handle(stream, self.device)))
        return logpost

    def logpost_grad_batch(self, heights, logpost=None, grad=None, stream=None):
        import torch
        n = int(heights.shape[0])
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        if logpost is None:
            logpost = torch.empty(n, dtype=torch.float64, device=heights.device)
        if grad is None:
            grad = torch.empty((n, self.S, self.R, self.C), dtype=self.torch_dtype, device=heights.device)
        self._check_tensor(logpost, (n,), torch.float64, "logpost")
        self._check_tensor(grad, (n, self.S, self.R, self.C), self.torch_dtype, "grad")
        self._check(self.lib.logpost_grad_batch(self.h, n, ct.c_void_p(heights.data_ptr()),
                                                ct.c_void_p(logpost.data_ptr()), ct.c_void_p(grad.data_ptr()),
                                                _stream_handle(stream, self.device)))
        return logpost, grad

    def nuts_run(self, heights, logpost, step_size, n_steps, seed, n_warmup=0, max_depth=8, inv_mass=None,
                 adapt_mass=False, max_delta_h=1000.0, target_accept=0.8, step_offset=0, stats=True, latent=False,
                 r_state=None, stream=None):
        """NUTS (with optional warm-up adaptation) on the chains in place.  step_size [n] float64 and
        inv_mass [n, S-1, R, C] float64 (or None) are device tensors, updated by the warm-up.  With
        r_state [n, S-1] float64 (latent only) every chain also samples its r (inv_mass is then
        [n, (S-1) R C + S-1]).  With stats, returns dict of per-transition tree_depth, n_leapfrog,
        diverged, accept_stat tensors."""
        import torch
        n = int(heights.shape[0])
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        self._check_tensor(logpost, (n,), torch.float64, "logpost")
        self._check_tensor(step_size, (n,), torch.float64, "step_size")
        rp = None
        if r_state is not None:
            self._check_tensor(r_state, (n, self.S - 1), torch.float64, "r_state")
            rp = r_state.data_ptr()
        im = None
        if inv_mass is not None:
            shape = self.heights_shape(n) if r_state is None else (n, (self.S - 1) * (self.R * self.C + 1))
            self._check_tensor(inv_mass, shape, torch.float64, "inv_mass")
            im = inv_mass.data_ptr()
        total = int(n_warmup) + int(n_steps)
        out = None
        ptrs = [None] * 4
        if stats and total > 0:
            dev = heights.device
            out = dict(tree_depth=torch.zeros((n, total), dtype=torch.int32, device=dev),
                       n_leapfrog=torch.zeros((n, total), dtype=torch.int32, device=dev),
                       diverged=torch.zeros((n, total), dtype=torch.int32, device=dev),
                       accept_stat=torch.zeros((n, total), dtype=torch.float64, device=dev))
            ptrs = [out[k].data_ptr() for k in ("tree_depth", "n_leapfrog", "diverged", "accept_stat")]
        cfg = NutsConfig(int(n_warmup), int(n_steps), int(max_depth), int(bool(adapt_mass)), float(max_delta_h),
                         float(target_accept), int(seed), int(step_offset), int(bool(latent)), rp)
        self._check(self.lib.nuts_run(self.h, ct.byref(cfg), n, ct.c_void_p(heights.data_ptr()),
                                      ct.c_void_p(logpost.data_ptr()), ct.c_void_p(step_size.data_ptr()),
                                      im, *ptrs, _stream_handle(stream, self.device)))
        return out

    def latent_to_heights(self, x, out=None, stream=None):
        """Heights of latent CAR states x [n, S-1, R, C] (device tensors)."""
        import torch
        n = int(x.shape[0])
        self._check_tensor(x, self.heights_shape(n), self.torch_dtype, "x")
        out = torch.empty_like(x) if out is None else out
        self._check_tensor(out, self.heights_shape(n), self.torch_dtype, "heights")
        self._check(self.lib.latent_to_heights(self.h, n, ct.c_void_p(x.data_ptr()), ct.c_void_p(out.data_ptr()),
                                               _stream_handle(stream, self.device)))
        return out

    def heights_to_latent(self, heights, out=None, stream=None):
        """Latent CAR states of ordered heights [n, S-1, R, C] (device tensors)."""
        import torch
        n = int(heights.shape[0])
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        out = torch.empty_like(heights) if out is None else out
        self._check_tensor(out, self.heights_shape(n), self.torch_dtype, "x")
        self._check(self.lib.heights_to_latent(self.h, n, ct.c_void_p(heights.data_ptr()),
                                               ct.c_void_p(out.data_ptr()), _stream_handle(stream, self.device)))
        return out

    def nested_rhat(self, heights, n_super, n_within, stream=None):
        """Nested R-hat of every free node from the chains' current states (one draw per chain)."""
        import torch
        n = int(heights.shape[0])
        if n != int(n_super) * int(n_within):
            raise ValueError(f"{n} chains are not {n_super} super-chains of {n_within}")
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        out = torch.empty(self.heights_shape(1)[1:], dtype=torch.float64, device=heights.device)
        self._check(self.lib.nested_rhat(self.h, int(n_super), int(n_within), ct.c_void_p(heights.data_ptr()),
                                         ct.c_void_p(out.data_ptr()), _stream_handle(stream, self.device)))
        return out

    def mcmc_run(self, heights, logpost, n_accept, n_steps, step_size, seed, step_offset=0, kernel=KERNEL_RW,
                 graph_steps=1, inv_mass=None, stream=None, r_state=None, r_step=0.0, n_accept_r=None):
        import torch
        n = int(heights.shape[0])
        self._check_tensor(heights, self.heights_shape(n), self.torch_dtype, "heights")
        self._check_tensor(logpost, (n,), torch.float64, "logpost")
        self._check_tensor(n_accept, (n,), torch.int64, "n_accept")
        im = None
        if inv_mass is not None:
            self._check_tensor(inv_mass, (self.S - 1, self.R, self.C), torch.float64, "inv_mass")
            im = inv_mass.data_ptr()
        rs = ar = None
        if r_state is not None:
            self._check_tensor(r_state, (n, self.S - 1), torch.float64, "r_state")
            rs = r_state.data_ptr()
        if n_accept_r is not None:
            self._check_tensor(n_accept_r, (n, self.S - 1), torch.int64, "n_accept_r")
            ar = n_accept_r.data_ptr()
        cfg = RunConfig(int(kernel), int(n_steps), int(graph_steps), float(step_size), im, int(seed),
                        int(step_offset), rs, float(r_step), ar)
        self._check(self.lib.mcmc_run(self.h, ct.byref(cfg), n, ct.c_void_p(heights.data_ptr()),
                                      ct.c_void_p(logpost.data_ptr()), ct.c_void_p(n_accept.data_ptr()),
                                      _stream_handle(stream, self.device)))


def mcmc_run_multi(problems, heights, logposts, n_accepts, n_steps, step_sizes, seeds, step_offsets=None,
                   graph_steps=1, r_states=None, r_step=0.0, n_accept_r=None, stream=None):
    """Random-walk Metropolis on several problems in shared launches.

    problems, heights, logposts, n_accepts, step_sizes and seeds are per-problem
    sequences (the tensors as for Problem.mcmc_run); n_steps and graph_steps are
    common to all.  r_states (per problem [n, S-1] float64 tensors, with
    r_step and optional n_accept_r [n, S-1] int64) samples r as in mcmc_run."""
    import torch
    n = len(problems)
    if not (len(heights) == len(logposts) == len(n_accepts) == len(step_sizes) == len(seeds) == n) or n == 0:
        raise ValueError("one entry per problem in every sequence")
    offs = step_offsets if step_offsets is not None else [0] * n
    lib = problems[0].lib
    hs = (ct.c_void_p * n)()
    cfgs = (RunConfig * n)()
    nch = (ct.c_int * n)()
    hp, lpp, ap = (ct.c_void_p * n)(), (ct.c_void_p * n)(), (ct.c_void_p * n)()
    for i, pr in enumerate(problems):
        c = int(heights[i].shape[0])
        pr._check_tensor(heights[i], pr.heights_shape(c), pr.torch_dtype, f"heights[{i}]")
        pr._check_tensor(logposts[i], (c,), torch.float64, f"logposts[{i}]")
        pr._check_tensor(n_accepts[i], (c,), torch.int64, f"n_accepts[{i}]")
        hs[i] = pr.h
        rp = ar = None
        if r_states is not None and r_states[i] is not None:
            pr._check_tensor(r_states[i], (c, pr.S - 1), torch.float64, f"r_states[{i}]")
            rp = r_states[i].data_ptr()
            if n_accept_r is not None and n_accept_r[i] is not None:
                pr._check_tensor(n_accept_r[i], (c, pr.S - 1), torch.int64, f"n_accept_r[{i}]")
                ar = n_accept_r[i].data_ptr()
        cfgs[i] = RunConfig(KERNEL_RW, int(n_steps), int(graph_steps), float(step_sizes[i]), None, int(seeds[i]),
                            int(offs[i]), rp, float(r_step), ar)
        nch[i] = c
        hp[i], lpp[i], ap[i] = heights[i].data_ptr(), logposts[i].data_ptr(), n_accepts[i].data_ptr()
    st = lib.mcmc_run_multi(n, hs, cfgs, nch, hp, lpp, ap, _stream_handle(stream, problems[0].device))
    if st != 0:
        raise MuonCaveError(st, lib.mc_last_error(problems[0].h).decode())


def time_march(problem: "Problem", heights, iters: int = 20, stream=None) -> float:
    """Mean milliseconds per launch of the ray-march kernel (HIP events on `stream`)."""
    ms = ct.c_float()
    n = int(heights.shape[0])
    problem._check_tensor(heights, problem.heights_shape(n), problem.torch_dtype, "heights")
    problem._check(problem.lib.mc_time_march(problem.h, n, ct.c_void_p(heights.data_ptr()), int(iters),
                                             _stream_handle(stream, problem.device), ct.byref(ms)))
    return float(ms.value)


def time_adjoint(problem: "Problem", heights, iters: int = 10, stream=None) -> float:
    """Mean milliseconds per launch of the adjoint march kernel (HIP events on `stream`)."""
    ms = ct.c_float()
    n = int(heights.shape[0])
    problem._check_tensor(heights, problem.heights_shape(n), problem.torch_dtype, "heights")
    problem._check(problem.lib.mc_time_adjoint(problem.h, n, ct.c_void_p(heights.data_ptr()), int(iters),
                                               _stream_handle(stream, problem.device), ct.byref(ms)))
    return float(ms.value)


def time_voxel(problem: "Problem", heights, iters: int = 10, stream=None):
    """Mean milliseconds per launch of the voxel model's density and
    likelihood kernels (HIP events on `stream`)."""
    a, b = ct.c_float(), ct.c_float()
    n = int(heights.shape[0])
    problem._check_tensor(heights, problem.heights_shape(n), problem.torch_dtype, "heights")
    problem._check(problem.lib.mc_time_voxel(problem.h, n, ct.c_void_p(heights.data_ptr()), int(iters),
                                             _stream_handle(stream, problem.device), ct.byref(a), ct.byref(b)))
    return float(a.value), float(b.value)


def measure_valu_rate(device: int = 0, kind: str = "f32") -> float:
    """Sustained non-packed FMA issue rate (lane-ops/s) measured on the device."""
    lib = load_library()
    v = ct.c_double()
    st = lib.mc_measure_valu_rate(int(device), 0 if kind == "f32" else 1, ct.byref(v))
    if st != 0:
        raise MuonCaveError(st, "mc_measure_valu_rate failed")
    return float(v.value)


def debug_philox(device, seed, chain, step, tag, j0, n):
    """Raw Philox words [n,4] (uint32 as int64) and Box-Muller normals [n,2] from the GPU."""
    import torch
    lib = load_library()
    words = torch.empty((n, 4), dtype=torch.int32, device=f"cuda:{device}")
    normals = torch.empty((n, 2), dtype=torch.float64, device=f"cuda:{device}")
    st = lib.mc_debug_philox(int(device), int(seed), int(chain), int(step), int(tag), int(j0), int(n),
                             ct.c_void_p(words.data_ptr()), ct.c_void_p(normals.data_ptr()))
    if st != 0:
        raise MuonCaveError(st, "mc_debug_philox failed")
    w = words.cpu().numpy().view(np.uint32)
    return w, normals.cpu().numpy()


class Server:
    """Serving loop on one GPU (mc_server_*): submit jobs at any time, poll
    for their posterior summaries.  The scheduler runs in a native thread."""

    def __init__(self, device: int = 0, precision: str = "f32", memory_budget: int = 0,
                 reserve: int = 8 << 30, max_jobs: int = 64, steps_per_round: int = 50):
        self.lib = load_library()
        self.precision = precision
        cfg = ServerConfig(int(device), MC_F64 if precision == "f64" else MC_F32, int(memory_budget),
                           int(reserve), int(max_jobs), int(steps_per_round))
        h = ct.c_void_p()
        st = self.lib.mc_server_create(ct.byref(cfg), ct.byref(h))
        if st != 0:
            raise MuonCaveError(st, self.lib.mc_server_last_error(None).decode())
        self.h = h
        self.shapes = {}

    def _check(self, st):
        if st != 0:
            raise MuonCaveError(st, self.lib.mc_server_last_error(self.h).decode())

    def submit(self, sc, n_chains, n_steps, step_size, seed, init=None, counts=None, block=0,
               rays_per_thread=0, r_step=0.0) -> int:
        """Queue one job for scenario `sc`; every chain starts at `init`
        ([S-1, R, C], default the scenario's truth); r_step > 0 samples every
        chain's r too (start: sc.car_r).  Returns the job id."""
        init = sc.truth if init is None else init
        c = sc.counts if counts is None else counts
        keep = dict(density=_host(sc.density), top=_host(sc.top), car_r=_host(sc.car_r),
                    pos=_host(sc.sensor_pos).reshape(-1), dirs=_host(sc.dirs).reshape(-1),
                    expo=_host(sc.exposure).reshape(-1), init=_host(init).reshape(-1))
        n_s = int(np.asarray(sc.sensor_pos).reshape(-1, 3).shape[0])
        n_pix = int(sc.n_pix) if n_s else 0
        cnt = _host(c, np.int32).reshape(-1) if n_s else np.zeros(0, np.int32)
        d = JobDesc(int(sc.n_surfaces), int(sc.n_rows), int(sc.n_cols), float(sc.extent_x), float(sc.extent_y),
                    _hp(keep["density"]), _hp(keep["top"]), _hp(keep["car_r"]), n_s, n_pix,
                    _hp(keep["pos"]), _hp(keep["dirs"]), _hp(keep["expo"]), float(sc.atten_len), _hp(cnt),
                    int(n_chains), _hp(keep["init"]), int(n_steps), float(step_size), int(seed), int(block),
                    int(rays_per_thread), float(r_step))
        jid = ct.c_int64()
        self._check(self.lib.mc_server_submit(self.h, ct.byref(d), ct.byref(jid)))
        self.shapes[jid.value] = (int(sc.n_surfaces) - 1, int(sc.n_rows), int(sc.n_cols))
        return jid.value

    def poll(self, job_id: int, arrays: bool = True) -> dict:
        info = JobInfo()
        shape = self.shapes[job_id]
        n = int(np.prod(shape))
        mean, sd, mp = (np.empty(n), np.empty(n), np.empty(n)) if arrays else (None, None, None)
        self._check(self.lib.mc_server_poll(self.h, int(job_id), ct.byref(info),
                                            _hp(mean) if arrays else None, _hp(sd) if arrays else None,
                                            _hp(mp) if arrays else None))
        out = {f: getattr(info, f) for f, _ in JobInfo._fields_}
        out["r_mean"] = list(info.r_mean)
        if info.status == JOB_FAILED:
            out["error"] = self.lib.mc_server_last_error(self.h).decode()
        if arrays and info.status == JOB_DONE:
            out.update(mean=mean.reshape(shape), std=sd.reshape(shape), map_state=mp.reshape(shape))
        return out

    def release(self, job_id: int):
        self._check(self.lib.mc_server_release(self.h, int(job_id)))
        self.shapes.pop(job_id, None)

    def wait_idle(self, timeout_s: float = 600.0):
        self._check(self.lib.mc_server_wait_idle(self.h, float(timeout_s)))

    def stats(self) -> dict:
        st = ServerStats()
        self._check(self.lib.mc_server_get_stats(self.h, ct.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self, drain: bool = True):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.mc_server_destroy(self.h, 1 if drain else 0)
            self.h = None

    def __del__(self):
        try:
            self.close(drain=False)
        except Exception:
            pass
