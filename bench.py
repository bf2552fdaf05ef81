#!/usr/bin/env python3
"""Throughput of the MetaDE inner-DE path on one MI355X.

Metric: inner-DE individual evaluations per second, sum over runs of
N * generations / wall time, with the inputs resident in HBM.  One step is one
full pass of the workload: for the default workload (full MetaDE at D=20:
evolver population 64, 10 outer generations of executors with N=100 and 1000
generations, the last one powered up 5x) that is every row of the path --
theta decode, initialisation, ranking, index sampling, mutation, crossover,
fitness, selection, float64 best record and the evolver step.

Prints one JSON line.  The generation kernel's average duration is taken with
HIP events on the library's stream around every launch of it inside the
timed region; its algorithmic work is the VALU lane-slot count of the
operations each trial needs (see ``alg_slots_per_trial``).
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

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz, one full-rate VALU
# instruction per lane per clock (packed float32 not used).
VALU_PEAK_SLOTS = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a workload's dominant kernel, from two rocprofv3
# counter runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) scaled by what the
# same counters read for a 2 GiB device copy (FETCH_SIZE reads 0.5x the copied
# bytes on this device, WRITE_SIZE 1.0x).  Keyed by a hash of the kernel's
# sources: a changed kernel reports null until measured again.
KERNEL_SOURCES = {
    "k_generations": ("paper_2502_10470_amd/csrc/kernels.hip",
                      "paper_2502_10470_amd/csrc/gen_common.h",
                      "paper_2502_10470_amd/csrc/device.h"),
    "k_generations_mfma": ("paper_2502_10470_amd/csrc/kernels_mfma.hip",
                           "paper_2502_10470_amd/csrc/gen_common.h",
                           "paper_2502_10470_amd/csrc/device.h"),
}
MEASURED_TRAFFIC = {
    # keyed by the kernel's source hash and the launch configuration the counters were
    # taken in (parts per trial, or precision and row tiles per rotation item)
    "a2860e14e11811ba:lp0": (472.075 * 2.0 + 526.0 * 1.0) * 1024,      # k_generations_kind, C3
    "3760489cb2075ba0:fp32:r4": (30396.6 * 2.0 + 7063607.6 * 1.0) * 1024,
    "3760489cb2075ba0:bf16:r4": (46001.8 * 2.0 + 6020998.0 * 1.0) * 1024,
}

PHILOX_SLOTS = 100   # 10 rounds x (2 quarter-rate 32x32->64 multiplies + 2 three-input XORs)
ELEM_SLOTS = {       # per element of z: square/accumulate + the element function
    "rastrigin": 9, "ackley": 9, "elliptic": 3, "rosenbrock": 6, "schwefel": 14,
}
ELEM_SLOTS["hybrid"] = (6 * ELEM_SLOTS["schwefel"] + 7 * ELEM_SLOTS["rastrigin"]
                        + 7 * ELEM_SLOTS["elliptic"]) / 20.0


def kernel_source_hash(kernel="k_generations"):
    """Hash of a kernel's sources' code: comments, whitespace and the stage-clock
    hooks of the diagnostic build (which expand to nothing in an ordinary
    build) are left out, so that only a change of the code itself invalidates a
    measurement."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"//[^\n]*", "", text)
        text = re.sub(r"#ifdef MDE_STAGE_CLOCKS.*?#endif", "", text, flags=re.S)
        text = re.sub(r"\bMDE_STAGE\w*(\(\w*\))?;?", "", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def decode(theta, n_cs):
    lo = np.array([0, 0, 1, 1, 1, 1], np.float32)
    hi = np.array([1, 1, 5, 5, 5, 1 + n_cs], np.float32)
    t = np.minimum(np.maximum(np.nan_to_num(theta, nan=0.0), lo), hi)
    cat = np.minimum(np.floor(t[:, 2:]).astype(int), [4, 4, 4, n_cs])
    return t[:, 0], t[:, 1], cat[:, 0], cat[:, 1], cat[:, 2], cat[:, 3]


def alg_slots_per_trial(N, D, kind, bl, br, dn, cs, CR):
    """VALU lane-slots one trial evaluation needs (algorithmic count, weighted
    by issue cost: quarter-rate integer multiplies and transcendentals = 4)."""
    m = int(1 in (bl, br)) + 2 * dn
    calls = 2 + (1 if m > 4 else 0)
    words = m + 3
    if cs == 1:
        calls += math.ceil(D / 4)
        words += D
    elif cs == 2:
        tests = sum(float(CR) ** k for k in range(max(D - 1, 0)))
        calls += tests / 4.0
        words += tests
    rng = calls * PHILOX_SLOTS + 3 * words
    sampler = m * 4 + m * (m + 1)
    mutation = D * (2 * dn + 1 + (3 if bl != br else 0))
    cross = D * (3 if cs in (1, 3) else 2)
    clip_shift = 3 * D
    rotation = D * D
    elem = D * ELEM_SLOTS[kind] + D
    ranking = 2 * math.log2(max(N, 2))
    return rng + sampler + mutation + cross + clip_shift + rotation + elem + ranking + 2


def ctrl_slots_per_trial(prob, bl, br, dn, cs, CR):
    """Lane-slots of one control trial: the DE part as for the other kinds plus
    the rollout's multiply-adds (float64 FMAs issue at the full rate), with the
    tanh evaluations not counted."""
    D, O, A, H1, H2 = prob.D, prob.A.shape[0], prob.B.shape[1], prob.hidden[0], prob.hidden[1]
    m = int(1 in (bl, br)) + 2 * dn
    calls = 3 + (math.ceil(D / 4) if cs == 1 else 1)
    rng = calls * PHILOX_SLOTS + 3 * (m + 3 + (D if cs == 1 else 0))
    de = D * (2 * dn + 1 + (3 if bl != br else 0)) + D * 3 + 2 * D
    macs = prob.steps * prob.x0.shape[0] * (H1 * O + H2 * H1 + A * H2 + O * O + O * A)
    return rng + m * (m + 5) + de + macs


def ctrl_rollout_macs(prob):
    """Multiply-adds of one policy's rollouts: layers and plant, every step."""
    O, A, H1, H2 = prob.A.shape[0], prob.B.shape[1], prob.hidden[0], prob.hidden[1]
    return prob.steps * prob.x0.shape[0] * (H1 * O + H2 * H1 + A * H2 + O * O + O * A)


def launch_slots(wl, theta, G):
    F, CR, bl, br, dn, cs = decode(theta, wl.n_cs)
    tot = 0.0
    for r in range(wl.n_runs):
        p = wl.problems[int(wl.problem[r])]
        N = int(wl.N[r])
        tot += N * G * alg_slots_per_trial(N, p.D, p.kind, bl[r], br[r], dn[r], cs[r], CR[r])
    return tot


def cpu_baseline(wl, budget_s=12.0):
    """The oracle (untuned) on a bounded sample of the same workload."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    from oracle import metade as ometa
    from oracle import pde

    X, y = ometa.outer_init(wl.outer["P"] if wl.outer else wl.n_runs, wl.seed, int(wl.stream[0]),
                            wl.n_cs)
    U, _ = ometa.outer_trials(X, y, 0, wl.seed, int(wl.stream[0]), wl.n_cs)
    th = pde.decode(U, wl.n_cs)
    evals = 0
    runs = 0
    G = 400
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and runs < wl.n_runs:
        r = runs
        prob = wl.problems[int(wl.problem[r])]
        t = {k: v[r] for k, v in th.items()}
        pde.run_executor(int(wl.N[r]), prob.D, t, G, wl.seed, int(wl.stream[r]), wl.lb, wl.ub, prob)
        evals += int(wl.N[r]) * G
        runs += 1
    dt = time.perf_counter() - t0
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {"value": evals / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} executor runs of the workload's shape (N={int(wl.N[0])}, "
                      f"D={wl.problems[0].D}, {wl.problems[0].kind}), {G} generations each, "
                      f"theta from the first evolver trial, {dt:.1f} s on one host core"}


POOL_WORKERS = 16   # host cores of the measurement machine's share


def _pool_run(args):
    """One executor run of the oracle on one core (worker of the all-cores baselines)."""
    name, r, G = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        pass
    import workloads as W
    from oracle import metade as ometa
    from oracle import pde
    if name == "c3":
        wl = W.workload_c3()
        X, y = ometa.outer_init(wl.outer["P"], wl.seed, int(wl.stream[0]), wl.n_cs)
        theta, _ = ometa.outer_trials(X, y, 0, wl.seed, int(wl.stream[0]), wl.n_cs)
    else:
        wl = W.workload_c4()
        theta = wl.theta
    th = pde.decode(theta, wl.n_cs)
    prob = wl.problems[int(wl.problem[r])]
    t = {k: v[r] for k, v in th.items()}
    pde.run_executor(int(wl.N[r]), prob.D, t, G, wl.seed, int(wl.stream[r]), wl.lb, wl.ub, prob)
    return int(wl.N[r]) * G


def cpu_baseline_pool_child(G3=2000, G4=30):
    """All-cores oracle figures: every executor run of the default workload's first
    evolver generation (its theta, G3 generations each) and every run of the D = 100
    workload (G4 generations each), on a pool of one-thread worker processes.  Runs in
    a process of its own that never touches the GPU; prints one JSON object."""
    import multiprocessing as mp
    import workloads as W
    workers = min(POOL_WORKERS, os.cpu_count() or 1)
    res = {}
    with mp.get_context("fork").Pool(workers) as pool:
        for name, wl, G in (("c3", W.workload_c3(), G3), ("c4", W.workload_c4(), G4)):
            t0 = time.perf_counter()
            evals = sum(pool.map(_pool_run, [(name, r, G) for r in range(wl.n_runs)], chunksize=1))
            dt = time.perf_counter() - t0
            res[name] = {"value": evals / dt, "cores": workers,
                         "sample": f"{wl.n_runs} executor runs x {G} generations, {dt:.1f} s wall "
                                   f"on {workers} worker processes"}
    print(json.dumps(res), flush=True)


def cpu_baseline_all_cores():
    """Start the all-cores baselines in a fresh interpreter (before this process
    starts the GPU runtime) and return {"c3": ..., "c4": ...}, or None."""
    import subprocess
    code = "import bench; bench.cpu_baseline_pool_child()"
    try:
        out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                             text=True, timeout=300)
        return json.loads(out.stdout.strip().splitlines()[-1])
    except Exception:  # pragma: no cover - reported as missing, never fatal
        return None


def cpu_baseline_c4(wl, budget_s=10.0, G=40):
    """The oracle (untuned) on a bounded sample of the D = 100 workload, one core."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    from oracle import pde
    th = pde.decode(wl.theta, wl.n_cs)
    evals = runs = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and runs < wl.n_runs:
        r = runs
        prob = wl.problems[int(wl.problem[r])]
        t = {k: v[r] for k, v in th.items()}
        pde.run_executor(int(wl.N[r]), prob.D, t, G, wl.seed, int(wl.stream[r]), wl.lb, wl.ub,
                         prob)
        evals += int(wl.N[r]) * G
        runs += 1
    dt = time.perf_counter() - t0
    if limiter is not None and hasattr(limiter, "unregister"):
        limiter.unregister()
    return {"value": evals / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} executor runs of the workload (N=256, D=100, elliptic and "
                      f"Rastrigin), {G} generations each, {dt:.1f} s on one host core"}


# Launch-shape choices measured by the library's autotuner on this device, one
# line per workload shape; a shape not in the file is measured and appended.
TUNING_TABLE = os.path.join(ROOT, "paper_2502_10470_amd", "tuning_gfx950.txt")

MFMA_F64_PEAK = 78.6e12
MFMA_BF16_PEAK = 2.5e15


def measure_batch(wl, name, precision, steps, warmup):
    """Independent executor runs (no evolver): one step = initialisation and
    first evaluation of every run, then all generations in one launch, then
    the float64 best record.  Returns the bench line's fields."""
    import torch
    from paper_2502_10470_amd import Batch, metade as M

    prec = M.BF16_REFINE if precision == "bf16" else M.FP32
    b = Batch(wl, precision=prec)
    evals = wl.evals_per_pass()
    tuning, _ = b.autotune(wl.G, TUNING_TABLE)

    def step():
        b.reset()
        b.inner_step(wl.G)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t_before, r_before = b.counters()
    b.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = b.kernel_time()
    b.kernel_timing(False)
    t_after, r_after = b.counters()
    b.close()
    dt = t1 - t0
    avg_ms = k_ms / max(k_launches, 1)
    F, CR, bl, br, dn, cs = decode(wl.theta, wl.n_cs)
    ctrl = name in ("c5", "t7", "c5e16")
    if ctrl:
        slots = sum(int(wl.N[r]) * wl.G * ctrl_slots_per_trial(wl.problems[int(wl.problem[r])],
                    bl[r], br[r], dn[r], cs[r], CR[r]) for r in range(wl.n_runs))
    else:
        slots = sum(int(wl.N[r]) * wl.G * alg_slots_per_trial(int(wl.N[r]), wl.D_of(r),
                    wl.problems[int(wl.problem[r])].kind, bl[r], br[r], dn[r], cs[r], CR[r])
                    for r in range(wl.n_runs))
    rot_flops = 0.0 if ctrl else sum(2.0 * int(wl.N[r]) * wl.D_of(r) ** 2 * wl.G
                                     for r in range(wl.n_runs))
    refine_rate = (r_after - r_before) / max(t_after - t_before, 1)
    at = {"c4": "D=100", "c2": "D in {10,20}", "c5": "D=5702 (control)",
          "t7": "D in {1539,1410,1506} (control, Table VII policies)",
          "c5e16": "D=5702 (control, 16 rollouts per policy)"}[name]
    ck = "k_ctrl_eval (timed with k_ctrl_rank, k_ctrl_trials, k_ctrl_commit)"
    kern = {"c4": "k_generations_mfma", "c2": "k_generations", "c5": ck, "t7": ck,
            "c5e16": "k_ctrl_eval_mx (timed with k_ctrl_rank, k_ctrl_trials, k_ctrl_commit)"
            }[name]
    line = {
        "metric": f"inner-DE individual-evals/sec (runs x N x gens / s) at {at}",
        "value": evals * steps / dt, "unit": "evals/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": 1000.0 * dt / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if ctrl else ("bf16+f64" if prec == M.BF16_REFINE else "f32"),
        "data": "synthetic",
        "config": {"workload": wl.name, "runs": wl.n_runs, "gens": wl.G,
                   "evals_per_step": evals, "precision": precision, "tuning": tuning,
                   "refine_rate": refine_rate if prec == M.BF16_REFINE else None},
        "roofline": {"bound": "alu", "achieved": slots / (avg_ms * 1e-3) / 1e12,
                     "peak": VALU_PEAK_SLOTS / 1e12, "unit": "Tslot/s",
                     "frac": slots / (avg_ms * 1e-3) / VALU_PEAK_SLOTS, "traffic": None,
                     "kernel": kern,
                     "avg_launch_ms": avg_ms, "launches": k_launches,
                     "rotation_tflops": rot_flops / (avg_ms * 1e-3) / 1e12,
                     "occupied_cu_frac": (1.0 if ctrl else min(wl.n_runs, 256) / 256.0)},
    }
    if name == "c4":
        # the D=100 kernel is bound by the rotation on the matrix cores: algorithmic
        # flops 2 N D^2 per trial (the bf16 mode's three split products and its
        # re-evaluations are not counted), against the peak of the dtype it runs in
        peak = MFMA_BF16_PEAK if prec == M.BF16_REFINE else MFMA_F64_PEAK
        ach = rot_flops / (avg_ms * 1e-3)
        traffic = MEASURED_TRAFFIC.get(f"{kernel_source_hash(kern)}:{precision}"
                                       f":r{tuning['mfma_rows']}")
        line["roofline"] = {"bound": "mfma", "achieved": ach / 1e12, "peak": peak / 1e12,
                            "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic,
                            "kernel": kern, "avg_launch_ms": avg_ms, "launches": k_launches,
                            "alu_frac": slots / (avg_ms * 1e-3) / VALU_PEAK_SLOTS,
                            "occupied_cu_frac": min(wl.n_runs, 256) / 256.0,
                            "frac_of_occupied_cus": ach / peak / (min(wl.n_runs, 256) / 256.0)}
    if name == "c5e16":
        # 16 rollouts per policy: the layers and the plant are float64 matrix-core
        # products; algorithmic flops are two per multiply-add of the rollouts
        # (padding of the tiles not counted), against the float64 matrix peak
        macs = sum(int(wl.N[r]) * wl.G * ctrl_rollout_macs(wl.problems[int(wl.problem[r])])
                   for r in range(wl.n_runs))
        ach = 2.0 * macs / (avg_ms * 1e-3)
        line["roofline"] = {"bound": "mfma", "achieved": ach / 1e12, "peak": MFMA_F64_PEAK / 1e12,
                            "unit": "TFLOP/s", "frac": ach / MFMA_F64_PEAK, "traffic": None,
                            "kernel": kern, "avg_launch_ms": avg_ms, "launches": k_launches,
                            "alu_frac": slots / (avg_ms * 1e-3) / VALU_PEAK_SLOTS,
                            "occupied_cu_frac": 1.0}
    return line


def bench_batch(args):
    import workloads as W
    wl = {"c4": W.workload_c4, "c2": W.workload_c2, "c5": W.workload_c5,
          "t7": W.workload_t7, "c5e16": W.workload_c5e16}[args.workload]()
    line = measure_batch(wl, args.workload, args.precision, args.steps, args.warmup)
    print(json.dumps(line), flush=True)


def d100_object(steps, warmup, pool=None, cpu=True):
    """The D = 100 half of the metric (128 runs x N = 256, 500 generations, elliptic
    and Rastrigin): the plain path and the bf16 + exact-refinement path, each with
    its roofline, plus the oracle timed on the host cores."""
    import workloads as W
    wl = W.workload_c4()
    out = {"workload": ("D=100: 128 executor runs x N=256, 500 generations, shifted-rotated "
                        "elliptic (cond 1e6) and Rastrigin, dense 100x100 rotations"),
           "evals_per_step": wl.evals_per_pass()}
    for prec in ("fp32", "bf16"):
        ln = measure_batch(wl, "c4", prec, steps, warmup)
        out[prec] = {"value": ln["value"], "unit": "evals/s", "ms_per_step": ln["ms_per_step"],
                     "dtype": ln["dtype"], "refine_rate": ln["config"]["refine_rate"],
                     "tuning": ln["config"]["tuning"], "roofline": ln["roofline"]}
    out["bf16_speedup"] = out["bf16"]["value"] / out["fp32"]["value"]
    if cpu:
        cb = cpu_baseline_c4(wl)
        if pool and "c4" in pool:
            cb["all_cores"] = pool["c4"]
        out["cpu_baseline"] = cb
    return out


def bench_c3_repetitions(args, reps=4):
    """Independent MetaDE repetitions of the default workload run concurrently,
    one context and one HIP stream each (the paper repeats every experiment;
    here the repetitions share the GPU, so together they occupy 4 x 64 CUs).
    Same problem instance, Philox key 2 + 1000 r for repetition r."""
    import dataclasses
    import threading
    import torch
    import workloads as W
    from paper_2502_10470_amd import Batch

    base = W.workload_c3()
    P, gens, G, pu = base.outer["P"], base.outer["gens"], base.G, base.outer["power_up"]
    streams = [torch.cuda.Stream() for _ in range(reps)]
    wls = [dataclasses.replace(base, seed=base.seed + 1000 * r) for r in range(reps)]
    batches = [Batch(wl, stream=st) for wl, st in zip(wls, streams)]
    evals = base.evals_per_pass() * reps

    thetas = []
    for b, wl in zip(batches, wls):
        b.outer_reset()
        th = []
        for g in range(gens):
            b.outer_step(G, pu if g == gens - 1 else 1)
            th.append(b.get_outer()[2].copy())
        thetas.append(th)
    slots = sum(launch_slots(wl, th[g], G * (pu if g == gens - 1 else 1))
                for wl, th in zip(wls, thetas) for g in range(gens))

    best = [None] * reps

    def one_pass():
        def work(r):
            best[r] = batches[r].run(gens, G, pu)
        ts = [threading.Thread(target=work, args=(r,)) for r in range(reps)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    achieved = slots * args.steps / dt
    line = {
        "metric": "inner-DE individual-evals/sec (runs x N x gens / s) at D=20",
        "value": evals * args.steps / dt, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{reps} independent repetitions of full MetaDE at D=20, run "
                               "concurrently on one GPU (one context and stream each)",
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4")),
                   "runs": P * reps, "N": 100, "D": 20, "inner_gens": G, "outer_gens": gens,
                   "evals_per_step": evals, "best_y": [b[0] for b in best]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / VALU_PEAK_SLOTS, "traffic": None,
                     "kernel": "k_generations (concurrent launches; work over the timed region)",
                     "occupied_cu_frac": min(P * reps, 256) / 256.0},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3",
                    choices=["c3", "c3x4", "paper", "c4", "c2", "c5", "t7", "c5e16"],
                    help="c3: full MetaDE at D=20 (default); c3x4: four independent "
                         "repetitions of it, concurrently; paper: MetaDE at the paper's scale "
                         "(evolver 100, three crossover schemes); c4: 128 runs x N=256 at D=100, "
                         "500 generations; c2: uneven batch of 256 runs, 200 generations; "
                         "c5: control workload, 16 runs x N=256 tanh policies (D=5702), "
                         "200-step rollouts, 100 generations; t7: the policy MLPs of "
                         "Table VII (hidden 32 x 32), 96 runs x N=100, 50 generations; "
                         "c5e16: c5 with 16 rollouts per policy, 10 generations")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"],
                    help="fitness contraction: plain (float64-accumulated) or bf16 matrix cores "
                         "with plain re-evaluation of near ties")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-d100", action="store_true",
                    help="default workload only: leave out the D=100 object")
    ap.add_argument("--budget-seconds", type=float, default=0.0,
                    help="c3 / paper only: equal-wall-clock mode, report the function "
                         "evaluations done within this many seconds")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration_mib:
        import torch
        n = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_calibration_mib, "launches": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation measures one GPU: the executor batch is not "
                                   "sharded across GPUs (run with --gpus 1)"}))
        sys.exit(2)
    if args.workload == "c3x4":
        # The repetitions overlap only if each stream gets a hardware queue of its
        # own: with HIP's default of 4 queues per process, two of the four streams
        # share one (the default stream holds another) and their launches run one
        # after the other.  Set before the HIP runtime starts.
        if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
            os.environ["GPU_MAX_HW_QUEUES"] = "8"
    # the all-cores oracle figure is taken first, in a separate process, while
    # this one has not started the GPU runtime
    pool_baseline = None
    if (not args.no_cpu_baseline and args.workload == "c3" and not args.budget_seconds):
        pool_baseline = cpu_baseline_all_cores()

    import torch
    import workloads as W
    from paper_2502_10470_amd import Batch

    if args.workload == "c3x4":
        return bench_c3_repetitions(args)
    if args.workload not in ("c3", "paper"):
        return bench_batch(args)
    wl = W.workload_c3() if args.workload == "c3" else W.workload_paper()
    if args.budget_seconds:
        return bench_budget(args, wl)
    args.pool_baseline = pool_baseline
    P, gens, G, pu = wl.outer["P"], wl.outer["gens"], wl.G, wl.outer["power_up"]
    b = Batch(wl)
    evals = wl.evals_per_pass()
    # theta of every outer generation (deterministic: identical in every pass)
    b.outer_reset()
    thetas = []
    for g in range(gens):
        b.outer_step(G, pu if g == gens - 1 else 1)
        thetas.append(b.get_outer()[2].copy())
    slots = sum(launch_slots(wl, thetas[g], G * (pu if g == gens - 1 else 1)) for g in range(gens))
    # launch shapes: tuned on the executors of the first evolver generation
    b.set_theta(thetas[0])
    b.reset()
    tuning, _ = b.autotune(G, TUNING_TABLE)

    for _ in range(args.warmup):
        b.run(gens, G, pu)
    torch.cuda.synchronize()
    b.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best = None
    for _ in range(args.steps):
        best = b.run(gens, G, pu)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_launches = b.kernel_time()
    b.kernel_timing(False)
    dt = t1 - t0
    ms_per_step = 1000.0 * dt / args.steps
    value = evals * args.steps / dt
    avg_launch_ms = k_ms / max(k_launches, 1)
    slots_per_launch = slots / gens
    achieved = slots_per_launch / (avg_launch_ms * 1e-3)
    D = wl.problems[0].D
    if args.workload == "c3":
        desc = ("full MetaDE at D=20 (evolver 64 x 10 gens, executors N=100, 1000 gens, "
                "power-up 5x, seeded hybrid Schwefel/Rastrigin/elliptic)")
    else:
        desc = (f"MetaDE at the paper's scale, D={D} (evolver 100 x {gens} gens, executors "
                "N=100, 1000 gens, power-up 5x, bin/exp/arith crossover: 192 strategies)")
    line = {
        "metric": f"inner-DE individual-evals/sec (runs x N x gens / s) at D={D}",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "runs": P, "N": 100, "D": D, "inner_gens": G,
                   "outer_gens": gens, "evals_per_step": evals, "best_y": best[0],
                   "tuning": tuning},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "Tslot/s", "frac": achieved / VALU_PEAK_SLOTS,
                     "traffic": (MEASURED_TRAFFIC.get(f"{kernel_source_hash()}"
                                                      f":lp{tuning['lane_parts']}")
                                 if args.workload == "c3" else None),
                     "kernel": "k_generations_kind<hybrid>", "avg_launch_ms": avg_launch_ms,
                     "launches": k_launches, "slots_per_launch": slots_per_launch,
                     "occupied_cu_frac": min(P, 256) / 256.0,
                     "frac_of_occupied_cus": achieved / VALU_PEAK_SLOTS / (min(P, 256) / 256.0)},
    }
    if not args.no_cpu_baseline and args.workload == "c3":
        line["cpu_baseline"] = cpu_baseline(wl)
        pool = getattr(args, "pool_baseline", None)
        if pool and "c3" in pool:
            line["cpu_baseline"]["all_cores"] = pool["c3"]
    if args.workload == "c3" and not args.no_d100:
        line["d100"] = d100_object(max(2, min(args.steps, 5)), 1,
                                   pool=getattr(args, "pool_baseline", None),
                                   cpu=not args.no_cpu_baseline)
    print(json.dumps(line), flush=True)


def bench_budget(args, wl):
    """Equal-wall-clock mode (the paper compares optimisers at a fixed time
    budget): outer generations run until the budget is nearly spent, the last
    one powered up; reports the function evaluations done and the best y."""
    import torch
    from paper_2502_10470_amd import Batch

    P, G, pu = wl.outer["P"], wl.G, wl.outer["power_up"]
    b = Batch(wl)
    N = int(wl.N[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.outer_reset()
    fe = 0
    gens = 0
    per_gen = None
    while True:
        elapsed = time.perf_counter() - t0
        # room for one more ordinary generation and the powered-up last one?
        if per_gen is not None and elapsed + per_gen * (1 + pu) > args.budget_seconds:
            break
        tg = time.perf_counter()
        b.outer_step(G, 1)
        torch.cuda.synchronize()
        per_gen = time.perf_counter() - tg
        fe += P * N * (G + 1)   # initial population and G generations of every executor
        gens += 1
    b.outer_step(G, pu)
    torch.cuda.synchronize()
    fe += P * N * (G * pu + 1)
    gens += 1
    dt = time.perf_counter() - t0
    _, y, _, _ = b.get_outer()
    best = float(np.nanmin(y))
    print(json.dumps({
        "metric": f"function evaluations within a {args.budget_seconds:g} s budget",
        "value": fe, "unit": "FE", "n_gpus": 1, "higher_is_better": True,
        "wall_s": dt, "outer_gens": gens, "best_y": best, "data": "synthetic",
        "config": {"workload": wl.name, "runs": P, "N": N, "D": wl.problems[0].D,
                   "inner_gens": G, "power_up": pu, "n_cs": wl.n_cs}}), flush=True)


if __name__ == "__main__":
    main()
