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


def opacity_tolerance(O_ref, crossings, min_fprime, precision, rho_max=2.7):
    """Per-ray opacity tolerance: relative 1e-5 (f32) or 1e-10 (f64), widened for
    ill-conditioned rays by the root sensitivity |dt| <= eps_z / |f'| of each
    crossing (eps_z = rounding of z and h in the march precision)."""
    if precision == "f32":
        rel, eps_z = 1e-5, 4e-5
    else:
        rel, eps_z = 1e-10, 1e-12
    mf = np.where(np.isfinite(min_fprime), np.maximum(min_fprime, 1e-12), 1.0)
    return rel * np.abs(O_ref) + rho_max * crossings * eps_z / mf + (1e-6 if precision == "f32" else 1e-12)
