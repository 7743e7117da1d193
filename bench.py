"""Throughput benchmark of the batched MCMC hot path on one MI355X.

A "step" is one random-walk Metropolis step of every chain: propose, march
every ray of every chain through the proposed surfaces, Poisson likelihood,
copula-CAR prior, accept/reject.  The default workload is the paper-scale
single problem: three surfaces on a 64x64 grid over 400 m x 400 m, 8 sensors
with 64x64 pixels each (32768 rays), 1024 chains, float32 march with float64
sums, HIP graphs of 50 steps.  Inputs are seeded synthetic stand-ins for the
paper's (unpublished) cave model and sensor layout; counts are Poisson draws
from the library's own forward model at the synthetic truth.

Prints one JSON line: value = ray-opacity evaluations per second over the
timed steps; the line also carries log-posterior
evaluations per second, the roofline of the ray-march kernel (timed alone
with HIP events on the benchmark's stream) and the FP64 CPU oracle timed on a
bounded sample on the host cores.  Other workloads (--workload hetero,
grad128, hier, voxel, nuts, quad, serve) print their own line; by default a short run of each is
summarised under "workloads" on the headline line.
"""
from __future__ import annotations

import argparse
import json
import math
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
# (18.93 and 2.94 per ray, averaged over 8 initial chain states).
OPS_CELL_BASE, OPS_TEST, OPS_CROSS, OPS_RAY = 8.0, 9.0, 45.0, 80.0
WORKLOAD_COUNTS = {"grf_cave_64": dict(cells=18.93, crossings=2.94, S=3),
                   "grf_cave_128": dict(cells=37.24, crossings=2.92, S=3)}
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one non-packed VALU lane-op
# per lane per clock; wave64 instructions issue over 4 clocks)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


# HBM bytes per launch of the march kernel, from two rocprofv3 --pmc runs of
# this script (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) scaled by what
# the same counters read for a 256 MiB device-to-device copy in the same run
# (FETCH_SIZE reads 131089 KiB for 262144 KiB moved: scale 2.0; WRITE_SIZE
# reads exactly: scale 1.0).  Valid only for the kernel sources they were
# taken on: the entry is dropped when the hash of those sources changes.
# The march keeps nothing in scratch: its WRITE_SIZE is the partial sums.
KERNEL_SOURCES = {"grf_cave_64": ("device_common.h", "march_common.h", "march3.h", "march5.h"),
                  "voxel64": ("device_common.h", "voxel.h"),
                  "grad128_adjoint": ("device_common.h", "march_common.h", "march5.h", "adjoint.h")}
MEASURED_TRAFFIC = {
    "grf_cave_64": dict(source_sha="0b8b340510832dff", fetch_kib=23174.0, fetch_scale=262144 / 131093.3,
                        write_kib=32.0, write_scale=1.0),
    # k_adjoint_rec on the 128x128 gradient workload (512 chains)
    "grad128_adjoint": dict(source_sha="a98a85b4ce252dfa", shape=(1024, 16), fetch_kib=431173.5,
                            fetch_scale=262144 / 131088.5, write_kib=196608.0, write_scale=1.0),
    # k_vox_lik: FETCH_SIZE counts what leaves the L2 for the fabric, so hits
    # in the memory-side cache are included
    "voxel64": dict(source_sha="f13683eefc9dc6a8", fetch_kib=2417941.5, fetch_scale=262144 / 131092.9,
                    write_kib=67260.1, write_scale=1.0),
}


# Executed-instruction counters of one 1024-chain march launch (rocprofv3
# --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU
# SQ_BUSY_CU_CYCLES SQ_INSTS_SALU GRBM_GUI_ACTIVE GRBM_COUNT with the kernel
# trace, same run; same source hash rule as the traffic).  GRBM_GUI_ACTIVE is
# summed over the 8 XCDs.  The FMA probe of the same run reads exactly its
# known instruction count (32768 waves x 2^16 x 8 = 1.718e10) at 0.969
# instructions per CU-clock, the full-lane issue limit.
MEASURED_VALU = {
    "grf_cave_64": dict(source_sha="0b8b340510832dff", valu_insts=8.934e8, thread_cycles_valu=2.695e10,
                        active_inst_valu=9.140e8, grbm_gui_active_per_xcd=2.3925e6, cus=256),
}


def measured_valu(name, rays_per_launch):
    """Issue rate and executed active-lane operations of the march launch
    from the stored counters (None when the kernel sources changed)."""
    m = MEASURED_VALU.get(name)
    if m is None or m["source_sha"] != kernel_source_sha(name):
        return None
    clocks = m["grbm_gui_active_per_xcd"]
    lane_ops = m["thread_cycles_valu"]   # active lanes summed over the VALU instructions
    return {"valu_insts_per_cu_clock": m["valu_insts"] / (m["cus"] * clocks),
            "lane_utilisation": m["thread_cycles_valu"] / (64.0 * m["active_inst_valu"]),
            "executed_lane_ops_per_ray": lane_ops / rays_per_launch,
            "executed_lane_ops_frac": lane_ops / (m["cus"] * 64.0 * clocks),
            "source_sha": m["source_sha"]}


def kernel_source_sha(name):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[name]:
        with open(os.path.join(ROOT, "paper_2603_28907_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name, shape=None):
    """Stored HBM bytes per launch (None when the kernel sources, or the
    launch shape (block, rays per thread) where one is stored, differ)."""
    m = MEASURED_TRAFFIC.get(name)
    if m is None or m["source_sha"] != kernel_source_sha(name):
        return None
    if shape is not None and "shape" in m and tuple(m["shape"]) != tuple(shape):
        return None
    return (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024


def algorithmic_bytes(sc, n_chains, rays_per_block):
    """Bytes one march launch must move at least: every chain's free surfaces
    (float32), the top surface, the per-ray tables once (9 float32 + 2
    float64 per ray) and one float64 partial per (chain, tile)."""
    N = sc.n_rows * sc.n_cols
    tiles = -(-sc.n_rays // rays_per_block)
    return (n_chains * (sc.n_surfaces - 1) * N * 4 + N * 4 + sc.n_rays * (9 * 4 + 2 * 8)
            + n_chains * tiles * 8)


def ops_per_ray(name):
    c = WORKLOAD_COUNTS[name]
    return OPS_RAY + c["cells"] * (OPS_CELL_BASE + c["S"] * OPS_TEST) + c["crossings"] * OPS_CROSS


def survey_ops_per_ray(name):
    """The plainer count cells x (10 S + 6): a cell step and one bound test
    per surface, nothing for the crossings' root solves or the float64
    Poisson term."""
    c = WORKLOAD_COUNTS[name]
    return c["cells"] * (10.0 * c["S"] + 6.0)


def adjoint_bytes(name, sc, n_chains, block, rays_per_thread):
    """Bytes one launch of the record adjoint must move at least: every
    crossing record once (16 B; the oracle's crossings per ray), the record
    counts of every (chain, tile, surface, thread), dLL/dO of every ray
    (4 B), and the 64-bit fixed-point gradient of every node written once."""
    c = WORKLOAD_COUNTS[name]
    rays = n_chains * sc.n_rays
    tiles = -(-sc.n_rays // (block * rays_per_thread))
    N = sc.n_rows * sc.n_cols
    return (rays * c["crossings"] * 16 + n_chains * tiles * sc.n_surfaces * block * 4 + rays * 4
            + n_chains * sc.n_surfaces * N * 8)


def make_workload(name):
    from paper_2603_28907_amd import inputs
    if name == "grf_cave_64":
        sc = inputs.grf_cave(seed=10)
        return sc, 1024, dict(counts_seed=11, init_seed=12, sigma=0.005)
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


def cpu_model():
    """The host CPU's model name (as lscpu reports it) or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(name, budget_s=10.0):
    """FP64 oracle (plain C, OpenMP over chains) on bounded samples: the
    headline workload (batches of chains, one log-posterior evaluation each,
    about budget_s), the tiny cave in full (4 chains x 1000 random-walk
    steps) and the 128x128 gradient (batches of chains, one log posterior and
    gradient each, about budget_s / 2).  Counts come from the oracle's own
    forward model (the GPU legs draw theirs from the library's); the timing
    does not depend on their values."""
    import oracle
    from paper_2603_28907_amd import inputs
    threads = oracle.max_threads()
    sc, n_chains, w = make_workload(name)
    sc.counts = oracle.make_counts(sc, seed=w["counts_seed"])
    orc = oracle.OracleProblem(sc)
    states = inputs.init_states(sc, 256, seed=w["init_seed"])
    done, t0 = 0, time.perf_counter()
    batch = max(threads, 8)
    while done < states.shape[0] and time.perf_counter() - t0 < budget_s:
        orc.logpost_batch(states[done:done + batch])
        done += batch
    dt = time.perf_counter() - t0
    out = {"value": done * sc.n_rays / dt, "unit": "ray-evals/s", "cores": threads, "kind": "oracle",
           "logpost_evals_per_s": done / dt,
           "sample": f"{done} chains x 1 log-posterior evaluation ({sc.n_rays} rays each) of the "
                     f"{name} workload, FP64, {threads} OpenMP threads",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    # the tiny cave in full
    tiny = inputs.tiny_bumps(seed=0)
    tiny.counts = oracle.make_counts(tiny, seed=1)
    ot = oracle.OracleProblem(tiny)
    st0 = inputs.init_states(tiny, 4, seed=2)
    t0 = time.perf_counter()
    _, _, acc, _ = ot.mcmc_rw(st0, np.full(4, np.nan), np.zeros(4, np.int64), 1000, 0, 0.05, 3)
    dt = time.perf_counter() - t0
    out["tiny_full"] = {"seconds": dt, "ray_evals_per_s": 4 * 1000 * tiny.n_rays / dt,
                        "logpost_evals_per_s": 4000 / dt, "accept_rate": float(acc.sum()) / 4000,
                        "threads": min(threads, 4),
                        "sample": f"tiny cave ({tiny.n_rays} rays, 16x16 nodes), 4 chains x 1000 random-walk "
                                  f"steps (sigma 0.05 m), FP64: the whole run"}
    # the 128x128 gradient
    sg = inputs.grf_cave(seed=10, n_grid=128)
    sg.counts = oracle.make_counts(sg, seed=11)
    og = oracle.OracleProblem(sg)
    sgs = inputs.init_states(sg, 64, seed=12)
    done, t0 = 0, time.perf_counter()
    while done < sgs.shape[0] and time.perf_counter() - t0 < budget_s / 2:
        og.grad_batch(sgs[done:done + threads])
        done += threads
    dt = time.perf_counter() - t0
    out["grad128"] = {"gradient_evals_per_s": done / dt, "ray_evals_per_s": done * sg.n_rays / dt,
                      "threads": threads,
                      "sample": f"{done} chains x 1 log posterior + gradient of the 128x128 geometry "
                                f"({sg.n_rays} rays), FP64"}
    return out


def build_hetero(n_problems, torch, precision="f32"):
    """The heterogeneous batch: problem i has seed 20+i, grid side in
    {16,32,64,128} over 400 m, 2-16 sensors, pixel side 32-64, 64-512 chains."""
    from paper_2603_28907_amd import inputs
    from paper_2603_28907_amd.binding import Problem
    probs, H, lp, acc = [], [], [], []
    dt = torch.float32 if precision == "f32" else torch.float64
    for i in range(n_problems):
        sc, n = inputs.heterogeneous_problem(i)
        sc.counts = gpu_counts(sc, torch)
        probs.append(Problem.from_scenario(sc, precision=precision))
        H.append(torch.as_tensor(inputs.init_states(sc, n, seed=500 + i), dtype=dt, device="cuda:0"))
        lp.append(torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0"))
        acc.append(torch.zeros(n, dtype=torch.int64, device="cuda:0"))
    return probs, H, lp, acc


def bench_hetero(args, torch):
    """Batched heterogeneous problems (mcmc_run_multi, autotuned shapes, HIP
    graphs) against the plain per-problem sampler (one problem at a time, one
    launch per kernel per step, no graph) on the same GPU and inputs."""
    from paper_2603_28907_amd import autotune
    from paper_2603_28907_amd.binding import mcmc_run_multi
    n_prob = args.problems

    def gap():
        """With --phase-gaps: 300 ms of idle GPU between phases, so that a
        kernel trace splits them."""
        if getattr(args, "phase_gaps", False):
            torch.cuda.synchronize()
            time.sleep(0.3)

    t0 = time.perf_counter()
    probs, H, lp, acc = build_hetero(n_prob, torch)
    sigma = [0.005] * n_prob
    seeds = [1000 + i for i in range(n_prob)]
    chain_rays = sum(h.shape[0] * p.n_rays for h, p in zip(H, probs))
    chains = sum(h.shape[0] for h in H)
    print(f"[bench] {n_prob} problems, {chains} chains, {chain_rays:.3e} chain-rays per step "
          f"(set-up {time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    # plain sampler with the library's default shapes
    for i, p in enumerate(probs):
        p.mcmc_run(H[i], lp[i], acc[i], 1, sigma[i], seeds[i], step_offset=0, graph_steps=1)
    torch.cuda.synchronize()
    gap()
    k_plain = max(1, args.plain_steps)
    t0 = time.perf_counter()
    for i, p in enumerate(probs):
        p.mcmc_run(H[i], lp[i], acc[i], k_plain, sigma[i], seeds[i], step_offset=1, graph_steps=1)
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t0
    print(f"[bench] plain sampler: {dt_plain / k_plain * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    gap()
    # autotuned shapes per grid class
    t0 = time.perf_counter()
    tuned = autotune.tune_batch(probs, H)
    dt_tune = time.perf_counter() - t0
    print(f"[bench] autotuned {len(tuned)} classes in {dt_tune:.1f} s", file=sys.stderr, flush=True)
    # plain sampler again, with the autotuned shapes (separates batching from tuning)
    off = 1 + k_plain
    for i, p in enumerate(probs):
        p.mcmc_run(H[i], lp[i], acc[i], 1, sigma[i], seeds[i], step_offset=off, graph_steps=1)
    torch.cuda.synchronize()
    off += 1
    t0 = time.perf_counter()
    for i, p in enumerate(probs):
        p.mcmc_run(H[i], lp[i], acc[i], k_plain, sigma[i], seeds[i], step_offset=off, graph_steps=1)
    torch.cuda.synchronize()
    dt_plain_tuned = time.perf_counter() - t0
    off += k_plain
    G = max(1, min(args.graph_steps, args.steps))

    def batched(blocks_per_cu):
        """Warm-up and timed steps of the batched form: one launch per grid
        class per step (blocks_per_cu = 0), or the persistent grid of
        blocks_per_cu blocks per CU over each class's work table."""
        nonlocal off
        t = probs[0].get_tuning()
        t["multi_blocks_per_cu"] = blocks_per_cu
        probs[0].set_tuning(**t)
        mcmc_run_multi(probs, H, lp, acc, args.warmup, sigma, seeds, step_offsets=[off] * n_prob,
                       graph_steps=min(G, max(args.warmup, 1)))
        torch.cuda.synchronize()
        off += args.warmup
        gap()
        t0 = time.perf_counter()
        mcmc_run_multi(probs, H, lp, acc, args.steps, sigma, seeds, step_offsets=[off] * n_prob, graph_steps=G)
        torch.cuda.synchronize()
        off += args.steps
        dt = time.perf_counter() - t0
        gap()
        return dt

    forms = {}
    for k in (0, 1, 2):
        forms[k] = batched(k)
        print(f"[bench] batched, blocks per CU {k}: {forms[k] / args.steps * 1e3:.2f} ms/step", file=sys.stderr,
              flush=True)
    best = min(forms, key=forms.get)
    dt = forms[best]
    print("[bench] timed region done", file=sys.stderr, flush=True)
    for x in lp:
        assert torch.isfinite(x).all(), "non-finite log posterior"
    value = chain_rays * args.steps / dt
    plain_value = chain_rays * k_plain / dt_plain
    return {
        "metric": METRIC, "value": value, "unit": "ray-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"hetero_{n_prob}: {n_prob} problems (seeds 20..{19 + n_prob}), grids "
                               f"{{16,32,64,128}}^2 over 400 m, 2-16 sensors, 32-64 px side, 64-512 chains; "
                               f"random-walk Metropolis sigma 0.005 m; float32 march, float64 sums; HIP graphs "
                               f"of {G} steps; autotuned launch shapes",
                   "problems": n_prob, "chains": chains, "chain_rays_per_step": chain_rays},
        "logpost_evals_per_s": chains * args.steps / dt,
        "plain": {"value": plain_value, "unit": "ray-evals/s", "ms_per_step": dt_plain / k_plain * 1e3,
                  "steps": k_plain, "logpost_evals_per_s": chains * k_plain / dt_plain,
                  "kind": "per-problem mcmc_run, graph_steps=1, default launch shapes"},
        "plain_tuned": {"value": chain_rays * k_plain / dt_plain_tuned, "unit": "ray-evals/s",
                        "ms_per_step": dt_plain_tuned / k_plain * 1e3, "steps": k_plain,
                        "kind": "per-problem mcmc_run, graph_steps=1, autotuned launch shapes"},
        "speedup_vs_plain": value / plain_value,
        "batched_form": "one launch per grid class" if best == 0 else f"persistent grid, {best} blocks per CU",
        "batched_forms_ms_per_step": {("per_class" if k == 0 else f"persistent_{k}_per_cu"): v / args.steps * 1e3
                                      for k, v in forms.items()},
        "autotune": {"seconds": dt_tune, "classes": {k: {f: v[f] for f in ("block", "rays_per_thread")}
                                                     for k, v in tuned.items()}},
    }


def bench_grad(args, torch):
    """Gradient-driven sampling on the 128x128 geometry: full log-posterior +
    gradient evaluations (forward march, adjoint march, prior gradient) and
    MALA steps on 512 chains; HBM roofline of the record adjoint."""
    from paper_2603_28907_amd import autotune, binding, inputs
    from paper_2603_28907_amd.binding import KERNEL_MALA, Problem
    sc = inputs.grf_cave(seed=10, n_grid=128)
    n_chains, eps = 512, args.mala_eps
    sc.counts = gpu_counts(sc, torch)
    prob = Problem.from_scenario(sc, precision="f32")
    H = torch.as_tensor(inputs.init_states(sc, n_chains, seed=12), dtype=torch.float32, device="cuda:0")
    lp = torch.empty(n_chains, dtype=torch.float64, device="cuda:0")
    g = torch.empty((n_chains, 3, 128, 128), dtype=torch.float32, device="cuda:0")
    tuned = autotune.tune_gradient(prob, H)   # launch shape of the gradient for these chains
    print(f"[bench] gradient launch shape {tuned['tuning']['block']}x{tuned['tuning']['rays_per_thread']}",
          file=sys.stderr, flush=True)
    prob.logpost_grad_batch(H, lp, g)
    torch.cuda.synchronize()
    k = max(1, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(k):
        prob.logpost_grad_batch(H, lp, g)
    torch.cuda.synchronize()
    dt_grad = (time.perf_counter() - t0) / k
    print(f"[bench] gradient evaluation: {dt_grad * 1e3:.2f} ms", file=sys.stderr, flush=True)
    lpm = torch.full((n_chains,), float("nan"), dtype=torch.float64, device="cuda:0")
    acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda:0")
    G = max(1, min(args.graph_steps, args.steps))
    prob.mcmc_run(H, lpm, acc, args.warmup, eps, 3, kernel=KERNEL_MALA, graph_steps=min(G, max(args.warmup, 1)))
    torch.cuda.synchronize()
    a0 = acc.clone()
    t0 = time.perf_counter()
    prob.mcmc_run(H, lpm, acc, args.steps, eps, 3, step_offset=args.warmup, kernel=KERNEL_MALA, graph_steps=G)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed region done", file=sys.stderr, flush=True)
    assert torch.isfinite(lpm).all(), "non-finite log posterior"
    ms_adj = binding.time_adjoint(prob, H, iters=args.march_iters)
    ms_fwd = binding.time_march(prob, H, iters=args.march_iters)
    t = prob.get_tuning()
    abytes = adjoint_bytes("grf_cave_128", sc, n_chains, t["block"], t["rays_per_thread"])
    achieved = abytes / (ms_adj * 1e-3) / 1e9
    return {
        "metric": METRIC, "value": n_chains * sc.n_rays * args.steps / dt, "unit": "ray-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"grad128: the paper-scale geometry regenerated on 128x128 nodes (8 sensors x "
                               f"64x64 pixels, {sc.n_rays} rays), {n_chains} chains, MALA eps {eps} m (one forward "
                               f"march, one adjoint march and the prior gradient per step), float32 march, float64 "
                               f"sums, HIP graphs of {G} steps", "chains": n_chains, "rays": sc.n_rays},
        "logpost_evals_per_s": n_chains * args.steps / dt,
        "accept_rate": float((acc - a0).double().mean().item()) / args.steps,
        "gradient_evals_per_s": n_chains / dt_grad, "ms_per_gradient_eval": dt_grad * 1e3,
        "forward_ms_per_launch": ms_fwd,
        "launch_shape": {"block": t["block"], "rays_per_thread": t["rays_per_thread"], "autotuned": True},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("grad128_adjoint", (t["block"], t["rays_per_thread"])),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes": abytes, "kernel": "k_adjoint_rec",
                     "ms_per_launch": ms_adj, "rays_per_launch": n_chains * sc.n_rays},
    }


def bench_hier(args, torch):
    """The paper-scale workload with every chain's CAR dependence r_l sampled
    (Metropolis-within-Gibbs on logit r after each H decision) beside the same
    chains at fixed r: the cost of the hierarchical prior."""
    from paper_2603_28907_amd import inputs
    from paper_2603_28907_amd.binding import Problem
    sc, n_chains, w = make_workload("grf_cave_64")
    sc.counts = gpu_counts(sc, torch)
    prob = Problem.from_scenario(sc, precision="f32")
    S1 = sc.n_surfaces - 1
    H0 = torch.as_tensor(inputs.init_states(sc, n_chains, seed=w["init_seed"]), dtype=torch.float32,
                         device="cuda:0").contiguous()
    G = max(1, min(args.graph_steps, args.steps))
    out = {}
    for mode in ("fixed", "sampled"):
        H = H0.clone()
        lp = torch.full((n_chains,), float("nan"), dtype=torch.float64, device="cuda:0")
        acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda:0")
        kw = {}
        if mode == "sampled":
            r = torch.full((n_chains, S1), 0.9, dtype=torch.float64, device="cuda:0")
            acc_r = torch.zeros((n_chains, S1), dtype=torch.int64, device="cuda:0")
            kw = dict(r_state=r, r_step=args.r_step, n_accept_r=acc_r)
        prob.mcmc_run(H, lp, acc, args.warmup, w["sigma"], 5, graph_steps=min(G, max(args.warmup, 1)), **kw)
        torch.cuda.synchronize()
        a0 = acc.clone()
        ar0 = kw["n_accept_r"].clone() if kw else None
        t0 = time.perf_counter()
        prob.mcmc_run(H, lp, acc, args.steps, w["sigma"], 5, step_offset=args.warmup, graph_steps=G, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert torch.isfinite(lp).all(), "non-finite log posterior"
        d = {"ms_per_step": dt / args.steps * 1e3, "value": n_chains * sc.n_rays * args.steps / dt,
             "logpost_evals_per_s": n_chains * args.steps / dt,
             "accept_rate": float((acc - a0).double().mean().item()) / args.steps}
        if kw:
            d["r_accept_rate"] = float((kw["n_accept_r"] - ar0).double().mean().item()) / args.steps
            d["r_mean"] = kw["r_state"].mean(dim=0).cpu().tolist()
        out[mode] = d
    s = out["sampled"]
    return {
        "metric": METRIC, "value": s["value"], "unit": "ray-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": s["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"hier_r_64: the grf_cave_64 workload ({n_chains} chains, {sc.n_rays} rays) with "
                               f"r_l sampled per chain (U(0,1) prior, logit step {args.r_step}, start 0.9), "
                               f"HIP graphs of {G} steps", "chains": n_chains, "rays": sc.n_rays},
        "logpost_evals_per_s": s["logpost_evals_per_s"], "accept_rate": s["accept_rate"],
        "r_accept_rate": s["r_accept_rate"], "r_mean": s["r_mean"],
        "fixed_r_ms_per_step": out["fixed"]["ms_per_step"],
        "overhead_vs_fixed_r": s["ms_per_step"] / out["fixed"]["ms_per_step"] - 1.0,
    }


def bench_voxel(args, torch):
    """The paper's own forward model on the paper-scale workload: the
    sigmoid-smoothed voxel density (n_z levels, gamma 1 m) and the likelihood
    linearised around the synthetic truth, random-walk Metropolis on 1024
    chains.  Roofline of each of its two kernels against HBM: the density
    kernel writes R-hat once; the likelihood kernel's minimum traffic is one
    read of R-hat plus the ray-voxel lists."""
    from paper_2603_28907_amd import binding, inputs
    from paper_2603_28907_amd.binding import Problem
    sc, n_chains, w = make_workload("grf_cave_64")
    sc.counts = gpu_counts(sc, torch)
    prob = Problem.from_scenario(sc, precision="f32")
    prob.set_voxel_model(args.n_z, 1.0, sc.truth)
    n_z, n_pieces = prob.voxel_info()
    H = torch.as_tensor(inputs.init_states(sc, n_chains, seed=w["init_seed"]), dtype=torch.float32,
                        device="cuda:0").contiguous()
    lp = torch.full((n_chains,), float("nan"), dtype=torch.float64, device="cuda:0")
    acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda:0")
    G = max(1, min(args.graph_steps, args.steps))
    prob.mcmc_run(H, lp, acc, args.warmup, w["sigma"], 1, graph_steps=min(G, max(args.warmup, 1)))
    torch.cuda.synchronize()
    a0 = acc.clone()
    t0 = time.perf_counter()
    prob.mcmc_run(H, lp, acc, args.steps, w["sigma"], 1, step_offset=args.warmup, graph_steps=G)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed region done", file=sys.stderr, flush=True)
    assert torch.isfinite(lp).all(), "non-finite log posterior"
    ms_dens, ms_lik = binding.time_voxel(prob, H, iters=args.march_iters)
    # log posterior + gradient under the voxel model (density, likelihood with
    # dLL/dO, back-projection, prior gradient), the evaluation MALA and NUTS make
    g = torch.empty((n_chains, sc.n_surfaces, sc.n_rows, sc.n_cols), dtype=torch.float32, device="cuda:0")
    lpg = torch.empty(n_chains, dtype=torch.float64, device="cuda:0")
    prob.logpost_grad_batch(H, lpg, g)
    torch.cuda.synchronize()
    kg = max(2, args.march_iters)
    t0 = time.perf_counter()
    for _ in range(kg):
        prob.logpost_grad_batch(H, lpg, g)
    torch.cuda.synchronize()
    ms_grad = (time.perf_counter() - t0) / kg * 1e3
    n_pad = (n_chains + 63) // 64 * 64
    n_vox = sc.n_rows * sc.n_cols * n_z
    rhat_bytes = n_vox * n_pad * 4
    lik_bytes = rhat_bytes + n_pieces * 8 + sc.n_rays * (4 + 3 * 8)
    dens_gbs = rhat_bytes / (ms_dens * 1e-3) / 1e9
    lik_gbs = lik_bytes / (ms_lik * 1e-3) / 1e9
    dom = "k_vox_lik" if ms_lik >= ms_dens else "k_vox_density"
    achieved = lik_gbs if dom == "k_vox_lik" else dens_gbs
    out = {
        "metric": METRIC, "value": n_chains * sc.n_rays * args.steps / dt, "unit": "ray-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"voxel64: the grf_cave_64 workload ({n_chains} chains, {sc.n_rays} rays) under "
                               f"the paper's smoothed voxel model ({sc.n_rows}x{sc.n_cols}x{n_z} voxels, gamma 1 m) "
                               f"linearised around the synthetic truth; random-walk Metropolis sigma {w['sigma']} m, "
                               f"float32 densities, float64 sums, HIP graphs of {G} steps",
                   "chains": n_chains, "rays": sc.n_rays, "voxels": n_vox, "ray_voxel_pieces": n_pieces},
        "logpost_evals_per_s": n_chains * args.steps / dt,
        "accept_rate": float((acc - a0).double().mean().item()) / args.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("voxel64") if dom == "k_vox_lik" else None,
                     "traffic_unit": "bytes per launch (L2 to fabric: memory-side cache hits included)",
                     "algorithmic_bytes": lik_bytes if dom == "k_vox_lik" else rhat_bytes, "kernel": dom,
                     "ms_per_launch": max(ms_dens, ms_lik)},
        "kernels": {"k_vox_density": {"ms_per_launch": ms_dens, "algorithmic_bytes": rhat_bytes,
                                      "GB_per_s": dens_gbs, "frac_hbm": dens_gbs / HBM_PEAK_GBS},
                    "k_vox_lik": {"ms_per_launch": ms_lik, "algorithmic_bytes": lik_bytes, "GB_per_s": lik_gbs,
                                  "frac_hbm": lik_gbs / HBM_PEAK_GBS,
                                  "gathered_bytes": n_pieces * n_pad * 4}},
        "gradient_ms_per_eval": ms_grad, "gradient_evals_per_s": n_chains / (ms_grad * 1e-3),
    }
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.OracleProblem(sc)
        orc.set_voxel_model(n_z, 1.0, sc.truth)
        cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
        k = max(cores, 8)
        states = H[:k].double().cpu().numpy()
        t0 = time.perf_counter()
        orc.logpost_batch(states)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": k * sc.n_rays / t, "unit": "ray-evals/s", "cores": cores, "kind": "oracle",
                               "logpost_evals_per_s": k / t,
                               "sample": f"{k} chains x 1 log-posterior evaluation of the voxel64 workload, FP64"}
    return out


def bench_nuts(args, torch):
    """The paper's sampler on the paper-scale geometry: NUTS with a 256-step
    trajectory cap (tree depth 8) on 32 super-chains of 8 chains that share
    their initial states, a short warm-up (dual averaging and windowed
    diagonal mass), then timed transitions; nested R-hat of the final states.
    Roofline of the adjoint march, the dominant kernel of each leapfrog step."""
    from paper_2603_28907_amd import autotune, binding, inputs
    from paper_2603_28907_amd.binding import Problem
    sc, _, w = make_workload("grf_cave_64")
    sc.counts = gpu_counts(sc, torch)
    prob = Problem.from_scenario(sc, precision="f32")
    voxel = bool(getattr(args, "nuts_voxel", False))
    n_super, n_within = 32, 8
    n = n_super * n_within
    starts = inputs.init_states(sc, n_super, seed=w["init_seed"], jitter=args.nuts_jitter)
    H = torch.as_tensor(np.repeat(starts, n_within, axis=0), dtype=torch.float32, device="cuda:0").contiguous()
    if voxel:   # the paper's pipeline: NUTS on the linearised, smoothed voxel model
        prob.set_voxel_model(args.n_z, 1.0, sc.truth)
    else:
        tuned = autotune.tune_gradient(prob, H)   # launch shape of the gradient for these chains
        print(f"[bench] gradient launch shape {tuned['tuning']['block']}x{tuned['tuning']['rays_per_thread']}: "
              f"{tuned['ms']:.3f} ms per evaluation", file=sys.stderr, flush=True)
    latent = not args.nuts_heights
    if latent:   # the paper's parametrisation: the CAR fields behind the heights
        H = prob.heights_to_latent(H)
    lp = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    eps = torch.full((n,), args.nuts_eps, dtype=torch.float64, device="cuda:0")
    im = torch.ones((n,) + tuple(H.shape[1:]), dtype=torch.float64, device="cuda:0")
    t0 = time.perf_counter()
    prob.nuts_run(H, lp, eps, 0, 1, n_warmup=args.nuts_warmup, max_depth=8, inv_mass=im, adapt_mass=True,
                  stats=False, latent=latent)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    print(f"[bench] NUTS warm-up {args.nuts_warmup} transitions: {t_warm:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st = prob.nuts_run(H, lp, eps, args.steps, 2, max_depth=8, inv_mass=im, step_offset=args.nuts_warmup,
                       latent=latent)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed region done", file=sys.stderr, flush=True)
    leaps = float(st["n_leapfrog"].double().sum().item())
    lockstep = float(st["n_leapfrog"].max(dim=0).values.double().sum().item()) * n   # gradients evaluated
    if latent:
        H = prob.latent_to_heights(H)
    rhat = prob.nested_rhat(H, n_super, n_within)
    if voxel:   # roofline of the likelihood gather, as in the voxel workload
        n_z, n_pieces = prob.voxel_info()
        ms_dens, ms_lik = binding.time_voxel(prob, H, iters=args.march_iters)
        n_pad = (n + 63) // 64 * 64
        lik_bytes = sc.n_rows * sc.n_cols * n_z * n_pad * 4 + n_pieces * 8 + sc.n_rays * (4 + 3 * 8)
        achieved = lik_bytes / (ms_lik * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": lik_bytes,
                "kernel": "k_vox_lik", "ms_per_launch": ms_lik}
        model = f"the paper's smoothed voxel model ({sc.n_rows}x{sc.n_cols}x{n_z} voxels, gamma 1 m, linearised " \
                f"around the synthetic truth)"
    else:
        ms_adj = binding.time_adjoint(prob, H, iters=args.march_iters)
        t = prob.get_tuning()
        abytes = adjoint_bytes("grf_cave_64", sc, n, t["block"], t["rays_per_thread"])
        achieved = abytes / (ms_adj * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": abytes,
                "kernel": "k_adjoint_rec", "ms_per_launch": ms_adj, "rays_per_launch": n * sc.n_rays}
        model = "the exact march"
    out = {
        "metric": METRIC, "value": leaps * sc.n_rays / dt, "unit": "ray-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.nuts_warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{'nuts64_voxel' if voxel else 'nuts64'}: the grf_cave_64 geometry and rays "
                               f"({sc.n_rays}) under {model}, "
                               f"{'latent CAR fields' if latent else 'heights'} sampled, {n_super} super-chains x "
                               f"{n_within} chains sharing their starts, NUTS with tree depth cap 8 (256 leapfrog "
                               f"steps), starts at the truth + {args.nuts_jitter} m jitter, {args.nuts_warmup} warm-up transitions "
                               f"(dual averaging, diagonal mass), "
                               f"float32 states, float64 sums", "chains": n, "rays": sc.n_rays},
        "leapfrog_steps_per_s": leaps / dt, "gradient_evals_per_s": lockstep / dt,
        "useful_fraction": leaps / max(lockstep, 1.0),
        "mean_tree_depth": float(st["tree_depth"].double().mean().item()),
        "divergent_fraction": float(st["diverged"].double().mean().item()),
        "mean_accept_stat": float(st["accept_stat"].mean().item()),
        "step_size_median": float(eps.median().item()),
        "nested_rhat_max": float(rhat.max().item()), "warmup_s": t_warm,
        "roofline": roof,
    }
    if not voxel:
        out["launch_shape"] = {"block": t["block"], "rays_per_thread": t["rays_per_thread"], "autotuned": True}
    return out


def bench_quad(args, torch):
    """The solid-angle pixel integral on the paper-scale workload: every pixel
    of grf_cave_64 split into q x q sub-cells (a sub-ray each, midpoint rule,
    synthetic efficiency), the tabulated synthetic intensity, random-walk
    Metropolis on 1024 chains; beside it the one-ray model on the same chains.
    Roofline of the march over all sub-rays."""
    from paper_2603_28907_amd import binding, inputs
    from paper_2603_28907_amd.binding import Problem
    sc, n_chains, w = make_workload("grf_cave_64")
    q = args.quad_q
    side = int(round(math.sqrt(sc.n_pix)))
    dirs, wq = inputs.pixel_subrays(side, side, q, exposure=1e4)
    scq = inputs.Scenario(name=sc.name + f"_q{q}", n_surfaces=sc.n_surfaces, n_rows=sc.n_rows, n_cols=sc.n_cols,
                          extent_x=sc.extent_x, extent_y=sc.extent_y, density=sc.density, top=sc.top,
                          car_r=sc.car_r, truth=sc.truth, sensor_pos=sc.sensor_pos,
                          dirs=np.broadcast_to(dirs, (sc.n_sensors,) + dirs.shape).copy(),
                          exposure=np.ones((sc.n_sensors, dirs.shape[0])), atten_len=sc.atten_len)
    o_max = 3000.0
    tab = inputs.intensity_table(513, o_max, sc.atten_len)
    weights = np.tile(wq, sc.n_sensors)
    nsub = q * q
    prob = Problem.from_scenario(scq, counts=np.zeros(scq.n_rays, np.int32), precision="f32")
    prob.set_pixel_quadrature(nsub, weights, tab, o_max)
    # counts: Poisson draws from the quadrature's own expected counts at the truth
    Ht = torch.as_tensor(sc.truth[None], dtype=torch.float32, device="cuda:0")
    Ot = torch.empty((1, scq.n_rays), dtype=torch.float32, device="cuda:0")
    prob.set_counts(np.zeros(scq.n_rays // nsub, np.int32))
    prob.logpost_batch(Ht, opacity=Ot)
    O = Ot[0].double().cpu().numpy()
    nodes = np.linspace(0.0, o_max, tab.size)
    lam = (weights * np.exp(np.interp(O, nodes, tab))).reshape(-1, nsub).sum(axis=1)
    prob.set_counts(inputs.draw_counts(lam, 11))
    H = torch.as_tensor(inputs.init_states(sc, n_chains, seed=w["init_seed"]), dtype=torch.float32,
                        device="cuda:0").contiguous()
    lp = torch.full((n_chains,), float("nan"), dtype=torch.float64, device="cuda:0")
    acc = torch.zeros(n_chains, dtype=torch.int64, device="cuda:0")
    G = max(1, min(args.graph_steps, args.steps))
    prob.mcmc_run(H, lp, acc, args.warmup, w["sigma"], 1, graph_steps=min(G, max(args.warmup, 1)))
    torch.cuda.synchronize()
    a0 = acc.clone()
    t0 = time.perf_counter()
    prob.mcmc_run(H, lp, acc, args.steps, w["sigma"], 1, step_offset=args.warmup, graph_steps=G)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed region done", file=sys.stderr, flush=True)
    assert torch.isfinite(lp).all(), "non-finite log posterior"
    ms_march = binding.time_march(prob, H, iters=args.march_iters)
    opr = ops_per_ray("grf_cave_64")
    achieved = opr * n_chains * scq.n_rays / (ms_march * 1e-3) / 1e12
    return {
        "metric": METRIC, "value": n_chains * scq.n_rays * args.steps / dt, "unit": "ray-evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"quad64: the grf_cave_64 workload with every pixel integrated over its solid angle "
                               f"by {q}x{q} sub-rays ({scq.n_rays} rays for {scq.n_rays // nsub} pixels), synthetic "
                               f"efficiency and tabulated intensity; random-walk Metropolis sigma {w['sigma']} m on "
                               f"{n_chains} chains, HIP graphs of {G} steps",
                   "chains": n_chains, "rays": scq.n_rays, "pixels": scq.n_rays // nsub},
        "logpost_evals_per_s": n_chains * args.steps / dt,
        "accept_rate": float((acc - a0).double().mean().item()) / args.steps,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TVALUop/s",
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel": "k_march_lik4",
                     "ms_per_launch": ms_march, "ops_per_ray": opr, "rays_per_launch": n_chains * scq.n_rays},
    }


def bench_serve(args, torch):
    """Serving: Poisson arrivals of heterogeneous jobs (sizes as the hetero
    workload), each run to a fixed number of steps per chain; the same
    arrival stream is served with continuous batching (many resident jobs)
    and by the plain one-job-at-a-time loop (max_jobs = 1)."""
    from paper_2603_28907_amd import inputs
    from paper_2603_28907_amd.binding import JOB_DONE, Server
    if getattr(args, "n_jobs", 0) > 0:   # the first n_jobs arrivals of the stream
        horizon = 2.0 * args.n_jobs / args.rate + 10.0
        arrivals = inputs.poisson_arrivals(args.rate, horizon, seed=40)
        while len(arrivals) < args.n_jobs:
            horizon *= 2.0
            arrivals = inputs.poisson_arrivals(args.rate, horizon, seed=40)
        arrivals = arrivals[:args.n_jobs]
    else:
        arrivals = inputs.poisson_arrivals(args.rate, args.duration, seed=40)
    n_jobs = len(arrivals)
    t0 = time.perf_counter()
    jobs = []
    for i in range(n_jobs):
        sc, n = inputs.heterogeneous_problem(i)
        sc.counts = gpu_counts(sc, torch)
        jobs.append((sc, n))
    print(f"[bench] {n_jobs} jobs generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    work_chain_steps = sum(n for _, n in jobs) * args.job_steps
    work_ray_steps = sum(n * sc.n_rays for sc, n in jobs) * args.job_steps

    def serve(max_jobs):
        srv = Server(precision="f32", max_jobs=max_jobs, steps_per_round=args.graph_steps)
        ids = []
        start = time.perf_counter()
        for k, (sc, n) in enumerate(jobs):
            delay = arrivals[k] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            ids.append(srv.submit(sc, n, args.job_steps, 0.005, 7000 + k))
            if (k + 1) % max(1, n_jobs // 20) == 0:
                st = srv.stats()
                print(f"[bench] max_jobs {max_jobs}: {k + 1}/{n_jobs} jobs submitted, {st['done']} done",
                      file=sys.stderr, flush=True)
        done = 0
        while True:
            st = srv.stats()
            if st["done"] + st["failed"] >= n_jobs:
                break
            if st["done"] > done + max(1, n_jobs // 10):
                done = st["done"]
                print(f"[bench] max_jobs {max_jobs}: {done}/{n_jobs} jobs done", file=sys.stderr, flush=True)
            time.sleep(0.05)
        infos = [srv.poll(j, arrays=False) for j in ids]
        st = srv.stats()
        srv.close()
        assert all(i["status"] == JOB_DONE for i in infos), "a job failed"
        lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
        wait = np.array([i["t_admit"] - i["t_submit"] for i in infos])
        serv = np.array([i["t_done"] - i["t_admit"] for i in infos])
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        q = lambda a, p: float(np.percentile(a, p))
        return {"max_jobs": max_jobs, "p50_s": q(lat, 50), "p99_s": q(lat, 99),
                "queue_p50_s": q(wait, 50), "queue_p99_s": q(wait, 99),
                "service_p50_s": q(serv, 50), "service_p99_s": q(serv, 99),
                "logpost_evals_per_s": work_chain_steps / span, "ray_evals_per_s": work_ray_steps / span,
                "makespan_s": span, "busy_s": st["busy_seconds"], "rounds": st["rounds"],
                "max_resident": st["max_resident"], "peak_gb": st["peak_bytes"] / 1e9}

    batched = serve(args.max_jobs)
    print(f"[bench] batched: {batched}", file=sys.stderr, flush=True)
    plain = serve(1) if not args.no_plain else None
    # offered load: arrival rate x GPU-busy seconds per job of the batched run
    offered = args.rate * batched["busy_s"] / n_jobs
    return {
        "metric": METRIC, "value": batched["ray_evals_per_s"], "unit": "ray-evals/s", "n_gpus": 1,
        "steps": args.job_steps, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve: Poisson arrivals at {args.rate} jobs/s, the first {n_jobs} jobs "
                               f"(seed 40, {arrivals[-1]:.1f} s of arrivals), job sizes as the hetero workload, "
                               f"{args.job_steps} steps per chain, rounds of {args.graph_steps} steps, "
                               f"up to {args.max_jobs} resident jobs",
                   "jobs": n_jobs, "rate_per_s": args.rate},
        "p50_s": batched["p50_s"], "p99_s": batched["p99_s"],
        "queue_p99_s": batched["queue_p99_s"], "service_p99_s": batched["service_p99_s"],
        "logpost_evals_per_s": batched["logpost_evals_per_s"],
        "offered_load": offered,
        "batched": batched, "plain": plain,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grf_cave_64")
    ap.add_argument("--graph-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--march-iters", type=int, default=20)
    ap.add_argument("--problems", type=int, default=256, help="problems in the hetero workload")
    ap.add_argument("--plain-steps", type=int, default=5, help="steps of the plain per-problem sampler")
    ap.add_argument("--phase-gaps", action="store_true",
                    help="hetero: 300 ms of idle GPU between phases (for splitting a kernel trace)")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: mean arrivals per second")
    ap.add_argument("--duration", type=float, default=3.0, help="serve: seconds of arrivals")
    ap.add_argument("--n-jobs", type=int, default=0,
                    help="serve: take the first n arrivals of the stream instead of --duration seconds")
    ap.add_argument("--job-steps", type=int, default=2000, help="serve: steps per chain per job")
    ap.add_argument("--max-jobs", type=int, default=64, help="serve: resident jobs at once")
    ap.add_argument("--mala-eps", type=float, default=0.004, help="grad128: MALA step size (m)")
    ap.add_argument("--r-step", type=float, default=0.3, help="hier: step of the logit-r random walk")
    ap.add_argument("--n-z", type=int, default=100, help="voxel: levels of the voxel grid")
    ap.add_argument("--quad-q", type=int, default=2, help="quad: sub-cells per pixel side")
    ap.add_argument("--nuts-warmup", type=int, default=20, help="nuts: warm-up transitions")
    ap.add_argument("--nuts-eps", type=float, default=0.0005, help="nuts: initial step size")
    ap.add_argument("--nuts-jitter", type=float, default=0.3, help="nuts: jitter of the super-chain starts (m)")
    ap.add_argument("--nuts-heights", action="store_true",
                    help="nuts: sample the heights instead of the latent CAR fields")
    ap.add_argument("--nuts-voxel", action="store_true",
                    help="nuts: under the paper's smoothed voxel model (--n-z levels, gamma 1 m, linearised "
                         "around the truth) instead of the exact march")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the short hetero / grad128 / serve runs summarised after the headline line")
    ap.add_argument("--no-plain", action="store_true", help="serve: skip the one-job-at-a-time baseline")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed region (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); chains and problems are independent "
              f"and would be sharded across GPUs without communication", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_28907_amd import binding, inputs
    from paper_2603_28907_amd.binding import Problem

    if args.copy_calibration_mb > 0:
        src = torch.ones(args.copy_calibration_mb << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "hetero":
        print(json.dumps(bench_hetero(args, torch)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, torch)), flush=True)
        return
    if args.workload == "grad128":
        print(json.dumps(bench_grad(args, torch)), flush=True)
        return
    if args.workload == "quad":
        print(json.dumps(bench_quad(args, torch)), flush=True)
        return
    if args.workload == "nuts":
        print(json.dumps(bench_nuts(args, torch)), flush=True)
        return
    if args.workload == "voxel":
        print(json.dumps(bench_voxel(args, torch)), flush=True)
        return
    if args.workload == "hier":
        print(json.dumps(bench_hier(args, torch)), flush=True)
        return
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
    tune = prob.get_tuning()
    opr = ops_per_ray(args.workload)
    achieved = opr * n_chains * sc.n_rays / (ms_march * 1e-3) / 1e12
    sopr = survey_ops_per_ray(args.workload)
    sach = sopr * n_chains * sc.n_rays / (ms_march * 1e-3) / 1e12
    measured_f32 = binding.measure_valu_rate(0, "f32") / 1e12
    measured_f64 = binding.measure_valu_rate(0, "f64") / 1e12
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
                     "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(args.workload),
                     "traffic_unit": "bytes per launch", "algorithmic_bytes": algorithmic_bytes(sc, n_chains, tune["block"] * tune["rays_per_thread"]),
                     "kernel": "k_march_lik4", "launch_shape": tune, "ms_per_launch": ms_march,
                     "ops_per_ray": opr, "rays_per_launch": n_chains * sc.n_rays,
                     "ops_per_ray_cell_count": sopr, "frac_cell_count": sach / VALU_PEAK_TOPS,
                     "measured_fma_rate": {"f32": measured_f32, "f64": measured_f64, "unit": "Tlane-op/s"},
                     "counters": measured_valu(args.workload, n_chains * sc.n_rays)},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    if not args.no_extras:
        out["workloads"] = run_extras(args, torch)
    print(json.dumps(out), flush=True)


def run_extras(args, torch):
    """Short runs of the other workloads (batched heterogeneous problems,
    gradient sampling at 128x128, sampled r, the voxel model, NUTS, serving), summarised beside the headline
    line; each is independent and a failure is reported, not raised."""
    import copy
    res = {}
    jobs = [
        ("hetero_256", bench_hetero, dict(steps=20, warmup=3, plain_steps=2, graph_steps=20, problems=256)),
        ("grad128", bench_grad, dict(steps=20, warmup=4, graph_steps=10, march_iters=5, mala_eps=0.004)),
        ("hier_r_64", bench_hier, dict(steps=50, warmup=10, graph_steps=50, r_step=0.3)),
        ("voxel64", bench_voxel, dict(steps=20, warmup=4, graph_steps=10, march_iters=5, n_z=100,
                                      no_cpu_baseline=True)),
        ("nuts64", bench_nuts, dict(steps=2, nuts_warmup=10, nuts_eps=0.0005, nuts_jitter=0.3, nuts_heights=False,
                                    march_iters=3)),
        ("serve_20_per_s", bench_serve, dict(rate=20.0, n_jobs=100, job_steps=2000, max_jobs=16, graph_steps=50,
                                             no_plain=True)),
    ]
    keep = {
        "hetero_256": ("value", "ms_per_step", "logpost_evals_per_s", "speedup_vs_plain", "batched_form",
                       "batched_forms_ms_per_step"),
        "grad128": ("value", "ms_per_step", "logpost_evals_per_s", "accept_rate", "gradient_evals_per_s"),
        "hier_r_64": ("value", "ms_per_step", "fixed_r_ms_per_step", "overhead_vs_fixed_r", "accept_rate",
                      "r_accept_rate", "r_mean"),
        "voxel64": ("value", "ms_per_step", "logpost_evals_per_s", "accept_rate", "kernels"),
        "nuts64": ("value", "ms_per_step", "leapfrog_steps_per_s", "useful_fraction", "mean_tree_depth",
                   "divergent_fraction", "mean_accept_stat", "nested_rhat_max"),
        "serve_20_per_s": ("value", "p50_s", "p99_s", "queue_p99_s", "service_p99_s", "logpost_evals_per_s",
                           "offered_load"),
    }
    for name, fn, over in jobs:
        a = copy.copy(args)
        for k, v in over.items():
            setattr(a, k, v)
        print(f"[bench] extra workload {name}", file=sys.stderr, flush=True)
        try:
            r = fn(a, torch)
            d = {k: r.get(k) for k in keep[name]}
            d["unit"] = r["unit"]
            d["workload"] = r["config"]["workload"]
            if "roofline" in r:
                d["roofline_frac"] = r["roofline"]["frac"]
                d["kernel"] = r["roofline"]["kernel"]
            if "plain" in r and r["plain"]:
                d["plain_logpost_evals_per_s"] = r["plain"]["logpost_evals_per_s"]
            res[name] = d
        except Exception as e:  # noqa: BLE001 -- a report, the headline line stands
            res[name] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.synchronize()
    return res


if __name__ == "__main__":
    main()
