"""Throughput benchmark of the batched MCMC hot path on one MI355X.

A "step" is one random-walk Metropolis step of every chain: propose, march
every ray of every chain through the proposed surfaces, Poisson likelihood,
copula-CAR prior, accept/reject.  The default workload is the paper-scale
single problem: three surfaces on a 64x64 grid over 400 m x 400 m, 8 sensors
with 64x64 pixels each (32768 rays), 1024 chains, float32 march with float64
sums, HIP graphs of 50 steps.  Inputs are seeded synthetic stand-ins for the
paper's (unpublished) cave model and sensor layout; counts are Poisson draws
from the library's own forward model at the synthetic truth.

Prints one JSON line (see README/DESIGN): value = ray-opacity evaluations
per second over the timed steps; the line also carries log-posterior
evaluations per second, the roofline of the ray-march kernel (timed alone
with HIP events on the benchmark's stream) and the FP64 CPU oracle timed on a
bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ray-opacity evals/s + log-posterior evals/s (chains) at 1 GPU; p50/p99 job latency")

# Algorithmic work of the exact march, in VALU lane-operations per ray:
#   per cell visited: 8 (2-D cell-walk step) + S x 9 (bound test of one
#   surface patch: min/max of 4 corners, 2 compares, 1 accumulate);
#   per crossing: 45 (end values, curvature, stable quadratic root);
#   per ray: 40 set-up (exit parameter, band window, cell of entry) + 40 for
#   the float64 Poisson term (exp, 2 FMA, accumulate).
# Cells and crossings per ray are the oracle's exact counts on this workload
# (18.93 and 2.94 per ray over 8 initial states).
OPS_CELL_BASE, OPS_TEST, OPS_CROSS, OPS_RAY = 8.0, 9.0, 45.0, 80.0
WORKLOAD_COUNTS = {"grf_cave_64": dict(cells=18.93, crossings=2.94, S=3)}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed VALU lane-op
# per lane per clock; wave64 instructions issue over 4 clocks)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def ops_per_ray(name):
    c = WORKLOAD_COUNTS[name]
    return OPS_RAY + c["cells"] * (OPS_CELL_BASE + c["S"] * OPS_TEST) + c["crossings"] * OPS_CROSS


def make_workload(name):
    from paper_2603_28907_amd import inputs
    if name == "grf_cave_64":
        sc = inputs.grf_cave(seed=10)
        return sc, 1024, dict(counts_seed=11, init_seed=12, sigma=0.05)
    raise SystemExit(f"unknown workload {name}")


def gpu_counts(sc, torch):
    """Poisson counts from the library's forward model at the synthetic truth."""
    from paper_2603_28907_amd import inputs
    from paper_2603_28907_amd.binding import Problem
    p = Problem.from_scenario(sc, counts=np.zeros((sc.n_sensors, sc.n_pix), np.int32), precision="f32")
    H = torch.as_tensor(sc.truth[None], dtype=torch.float32, device="cuda:0")
    O = torch.empty((1, sc.n_rays), dtype=torch.float32, device="cuda:0")
    p.logpost_batch(H, opacity=O)
    lam = sc.exposure.reshape(-1) * np.exp(-O[0].double().cpu().numpy() / sc.atten_len)
    p.close()
    return inputs.draw_counts(lam, 11).reshape(sc.n_sensors, sc.n_pix)


def cpu_baseline(name, budget_s=10.0):
    """FP64 oracle (plain C, OpenMP over chains) on a bounded sample of the
    same workload: batches of chains, one log-posterior evaluation each."""
    import oracle
    from paper_2603_28907_amd import inputs
    sc, n_chains, w = make_workload(name)
    sc.counts = oracle.make_counts(sc, seed=w["counts_seed"])
    orc = oracle.OracleProblem(sc)
    states = inputs.init_states(sc, 256, seed=w["init_seed"])
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    done, t0 = 0, time.perf_counter()
    batch = max(cores, 8)
    while done < states.shape[0] and time.perf_counter() - t0 < budget_s:
        orc.logpost_batch(states[done:done + batch])
        done += batch
    dt = time.perf_counter() - t0
    return {"value": done * sc.n_rays / dt, "unit": "ray-evals/s", "cores": cores, "kind": "oracle",
            "logpost_evals_per_s": done / dt,
            "sample": f"{done} chains x 1 log-posterior evaluation ({sc.n_rays} rays each) of the "
                      f"{name} workload, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grf_cave_64")
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--march-iters", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); chains and problems are independent "
              f"and would be sharded across GPUs without communication", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_28907_amd import binding, inputs
    from paper_2603_28907_amd.binding import Problem

    sc, n_chains, w = make_workload(args.workload)
    print(f"[bench] workload {args.workload}: {n_chains} chains x {sc.n_rays} rays", file=sys.stderr, flush=True)
    sc.counts = gpu_counts(sc, torch)
    prob = Problem.from_scenario(sc, precision="f32")
    H = torch.as_tensor(inputs.init_states(sc, n_chains, seed=w["init_seed"]), dtype=torch.float32,
                        device="cuda:0").contiguous()
    lp = torch.full((n_chains,), float("nan"), dtype=torch.float64, device="cuda:0")
    acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda:0")
    G = max(1, min(args.graph_steps, args.steps))
    prob.mcmc_run(H, lp, acc, n_steps=args.warmup, step_size=w["sigma"], seed=1, step_offset=0,
                  graph_steps=min(G, max(args.warmup, 1)))
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.mcmc_run(H, lp, acc, n_steps=args.steps, step_size=w["sigma"], seed=1, step_offset=args.warmup,
                  graph_steps=G)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed region done", file=sys.stderr, flush=True)
    lp_h = lp.cpu().numpy()
    assert np.all(np.isfinite(lp_h)), "non-finite log posterior"
    ray_evals = n_chains * sc.n_rays * args.steps
    # roofline of the dominant kernel: the ray march, timed alone with HIP events
    ms_march = binding.time_march(prob, H, iters=args.march_iters)
    opr = ops_per_ray(args.workload)
    achieved = opr * n_chains * sc.n_rays / (ms_march * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": ray_evals / dt,
        "unit": "ray-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3 surfaces on 64x64 nodes over 400x400 m, 8 sensors x "
                               f"64x64 pixels ({sc.n_rays} rays), {n_chains} chains, random-walk Metropolis "
                               f"sigma {w['sigma']} m, float32 march with float64 sums, HIP graphs of {G} steps",
                   "chains": n_chains, "rays": sc.n_rays, "graph_steps": G},
        "logpost_evals_per_s": n_chains * args.steps / dt,
        "accept_rate": float(acc.double().mean().item()) / (args.warmup + args.steps),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TVALUop/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_march_lik", "ms_per_launch": ms_march,
                     "ops_per_ray": opr, "rays_per_launch": n_chains * sc.n_rays},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
