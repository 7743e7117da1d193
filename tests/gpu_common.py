"""Shared helpers for the GPU parity tests (imported only by tests marked gpu)."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28907_amd import binding
    binding.load_library()   # raises if the HIP library is missing: no silent fallback
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x, dtype, device=0):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=f"cuda:{device}")


def rounded_states(states, precision):
    """The states as the GPU stores them (float32 rounding in f32 mode)."""
    s = np.asarray(states, np.float64)
    return s.astype(np.float32).astype(np.float64) if precision == "f32" else s


def f32_eps_z(ztop=210.0):
    """Rounding of f = z - h in the float32 march: 3 ulps at the box height
    (z = q_z + t d_z rounds once, the bilinear height twice in its lerps)."""
    return 3.0 * float(np.spacing(np.float32(ztop)))


def opacity_tolerance(O_ref, crossings, min_fprime, precision, rho_max=2.7, ztop=210.0):
    """Per-ray opacity tolerance: relative 1e-5 (f32) or 1e-10 (f64), widened for
    ill-conditioned rays by the root sensitivity |dt| <= eps_z / |f'| of each
    crossing (eps_z = rounding of z and h in the march precision)."""
    if precision == "f32":
        rel, eps_z = 1e-5, f32_eps_z(ztop)
    else:
        rel, eps_z = 1e-10, 1e-12
    mf = np.where(np.isfinite(min_fprime), np.maximum(min_fprime, 1e-12), 1.0)
    return rel * np.abs(O_ref) + rho_max * crossings * eps_z / mf + (1e-6 if precision == "f32" else 1e-12)


def f32_gradient_tolerance(orc, state, dO, g_prior, g=None, g_err=None):
    """Per-node tolerance of a float32 gradient: the oracle's conditioning
    report over every crossing (root shift eps_z/|f'| moving the bilinear
    weights and 1/|f'|; the weights' own rounding, 2^-22 (max(R, C) - 1) in
    local coordinates that reach the cell index; pairs within eps_z of
    tangency; cell edges where |f'| jumps; crossings within 16 float32 ulps
    of the box lid, which the GPU takes for the lid's kink; 4e-6 relative
    rounding per contribution; the error of dLL/dO from the measured opacity
    error dO of each ray), plus the float32 prior workspace (1e-5 of the
    prior gradient) and 1e-6 absolute.  g, g_err: each ray's dLL/dO and its
    error where the one-ray model's do not apply (solid-angle pixels)."""
    ztop = float(np.max(orc._top))
    eps_w = 2.0 ** -22 * (max(orc.R, orc.C) - 1)
    lid = 16.0 * float(np.spacing(np.float32(ztop)))
    cond = orc.grad_conditioning(state, f32_eps_z(ztop), 4e-6, eps_w=eps_w, lid_band=lid, dO=dO, g=g,
                                 g_err=g_err)
    return cond + 1e-5 * np.abs(g_prior) + 1e-6


def f64_gradient_tolerance(orc, state, dO, g_prior, g=None, g_err=None):
    """Per-node tolerance of a float64 gradient: the same conditioning report
    at float64 rounding (3 ulps of z - h at the box height, 2^-50 (max(R, C)
    - 1) on the bilinear weights, 1e-13 relative per contribution, the
    float64 lid band of 256 eps (|z_top| + |min top| + 1)), with the measured
    float64 opacity error of each ray, plus 1e-10 of the prior gradient and
    64 roundings of the 2^-32 fixed point in which the likelihood gradient
    is summed (2^-33 each)."""
    ztop = float(np.max(orc._top))
    eps_z = 3.0 * float(np.spacing(ztop))
    eps_w = 2.0 ** -50 * (max(orc.R, orc.C) - 1)
    lid = 256.0 * 2.0 ** -52 * (abs(ztop) + abs(float(np.min(orc._top))) + 1.0)
    cond = orc.grad_conditioning(state, eps_z, 1e-13, eps_w=eps_w, lid_band=lid, dO=dO, g=g, g_err=g_err)
    return cond + 1e-10 * np.abs(g_prior) + 64 * 2.0 ** -33
