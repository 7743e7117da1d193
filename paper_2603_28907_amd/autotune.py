"""Launch-shape autotuner for the ray-march kernel and the gradient.

For one problem the tuner times the march kernel (HIP events on the given
stream, through mc_time_march) over a small grid of launch shapes and keeps
the fastest; tune_gradient does the same for the log posterior + gradient
evaluation.  For a heterogeneous batch it tunes one representative problem
per grid class -- (surfaces, rows, cols, precision) -- and applies the winner
to every problem of that class, so mcmc_run_multi then groups the class into
one launch of that shape.  Results are cached in memory and, when a path is
given, in a JSON file keyed by the device name and class.

Launch shape changes only performance: each chain's log posterior is the
same quantity whatever the shape, and for a fixed shape the results are
deterministic.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Sequence

F32_SHAPES = [dict(march_variant=4, block=b, rays_per_thread=r, top_in_lds=0)
              for b in (256, 512, 1024) for r in (2, 4, 8, 16)]
F64_SHAPES = [dict(march_variant=3, block=256, rays_per_thread=r, top_in_lds=1) for r in (1, 2, 4, 8)]
# the gradient (march with crossing records, record adjoint): 512- and
# 1024-thread blocks (256-thread blocks lose to both on every grid measured)
GRAD_SHAPES = [dict(march_variant=4, block=b, rays_per_thread=r, top_in_lds=0)
               for b in (512, 1024) for r in (4, 8, 16)]

_memo: Dict[str, dict] = {}


def class_key(problem, device_name: str = "") -> str:
    return f"{device_name}|S{problem.S}|{problem.R}x{problem.C}|{problem.precision}"


def _device_name(problem) -> str:
    import torch
    return torch.cuda.get_device_name(problem.device)


def tune_problem(problem, heights, shapes: Optional[Sequence[dict]] = None, iters: int = 5,
                 stream=None) -> dict:
    """Time every shape on `heights` ([n_chains, S-1, R, C] on the device) and
    leave the fastest set on the problem.  Returns {"tuning":..., "ms":...,
    "trials": [(shape, ms), ...]}."""
    from .binding import MuonCaveError, time_march
    if problem.n_rays == 0:
        return {"tuning": problem.get_tuning(), "ms": 0.0, "trials": []}
    if shapes is None:
        shapes = F64_SHAPES if problem.precision == "f64" else F32_SHAPES
    base = problem.get_tuning()
    trials = []
    for sh in shapes:
        t = dict(base)
        t.update(sh)
        try:
            problem.set_tuning(**t)
            time_march(problem, heights, iters=1, stream=stream)   # first launch: code load
            ms = time_march(problem, heights, iters=iters, stream=stream)
        except MuonCaveError:
            continue
        trials.append((t, ms))
    if not trials:
        problem.set_tuning(**base)
        return {"tuning": base, "ms": float("nan"), "trials": []}
    best, ms = min(trials, key=lambda x: x[1])
    problem.set_tuning(**best)
    return {"tuning": best, "ms": ms, "trials": trials}


def tune_gradient(problem, heights, shapes: Optional[Sequence[dict]] = None, iters: int = 5,
                  stream=None) -> dict:
    """Time the log posterior + gradient evaluation (logpost_grad_batch: the
    gradient march, the adjoint and the prior gradient) on `heights` for every
    shape, with HIP events on the stream, and leave the fastest set on the
    problem.  The best shape depends on the chain count as well as the grid
    (few chains leave too few blocks for the GPU at many rays per thread), so
    the caller tunes with the chains it will run.  Float32 problems only; a
    float64 problem keeps its shape.  Returns {"tuning":..., "ms":...,
    "trials": [(shape, ms), ...]}."""
    import torch
    from .binding import MuonCaveError
    base = problem.get_tuning()
    if problem.n_rays == 0 or problem.precision != "f32":
        return {"tuning": base, "ms": float("nan"), "trials": []}
    if shapes is None:
        shapes = GRAD_SHAPES
    n = int(heights.shape[0])
    lp = torch.empty(n, dtype=torch.float64, device=heights.device)
    g = torch.empty((n, problem.S, problem.R, problem.C), dtype=torch.float32, device=heights.device)
    s = stream if stream is not None else torch.cuda.current_stream(heights.device)
    trials = []
    for sh in shapes:
        t = dict(base)
        t.update(sh)
        try:
            problem.set_tuning(**t)
            problem.logpost_grad_batch(heights, lp, g, stream=s)   # code load, workspaces
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(iters):
                problem.logpost_grad_batch(heights, lp, g, stream=s)
            e1.record(s)
            e1.synchronize()
        except MuonCaveError:
            continue
        trials.append((t, e0.elapsed_time(e1) / iters))
    if not trials:
        problem.set_tuning(**base)
        return {"tuning": base, "ms": float("nan"), "trials": []}
    best, ms = min(trials, key=lambda x: x[1])
    problem.set_tuning(**best)
    return {"tuning": best, "ms": ms, "trials": trials}


def tune_batch(problems: Sequence, heights: Sequence, cache_path: Optional[str] = None, iters: int = 5,
               max_tune_chains: int = 512, stream=None) -> Dict[str, dict]:
    """Tune one representative per grid class (the problem with the most
    chain-rays) and apply its shape to the whole class.  Returns the
    class -> tuning map."""
    disk = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            disk = json.load(f)
    dev = _device_name(problems[0]) if problems else ""
    classes: Dict[str, list] = {}
    for i, p in enumerate(problems):
        classes.setdefault(class_key(p, dev), []).append(i)
    out = {}
    for key, members in classes.items():
        if key in _memo:
            tun = _memo[key]
        elif key in disk:
            tun = disk[key]
        else:
            rep = max(members, key=lambda i: heights[i].shape[0] * problems[i].n_rays)
            h = heights[rep][:max_tune_chains].contiguous()
            tun = tune_problem(problems[rep], h, iters=iters, stream=stream)["tuning"]
        _memo[key] = tun
        disk[key] = tun
        out[key] = tun
        for i in members:
            problems[i].set_tuning(**tun)
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(disk, f, indent=1, sort_keys=True)
    return out


def apply_cached(problems: Iterable, device_name: Optional[str] = None) -> int:
    """Apply tunings already found in this process; returns how many problems got one."""
    n = 0
    for p in problems:
        key = class_key(p, device_name if device_name is not None else _device_name(p))
        if key in _memo:
            p.set_tuning(**_memo[key])
            n += 1
    return n
