#!/usr/bin/env python3
"""Benchmark of the analytic partial-OT solver on one MI355X.

Workload (the measured configuration): 100,000 sites on a jittered cubic
lattice filling the lower 40% of the unit box (dam-break layout), prescribed
volumes 3.5e-6 each (0.35 of the box), start weights with ball radius
1.2 (3 nu / 4 pi)^(1/3); float32 geometry, float64 reductions and CG.

A step is one full OT solve (grid build, every Newton evaluation of all cells,
Hessian assembly, Jacobi-PCG, KMT step control) from the start weights to
max |V_i - nu_i| / nu_i <= 1e-5. Inputs are resident in HBM before timing.

Printed (one JSON line):
  value          Laguerre∩ball cell evaluations per second over the whole solve
                 (N x evaluations / wall time of the timed solves)
  ms_per_step    ms per OT solve (plain start)
  roofline       float32 cell kernel: algorithmic FLOPs per launch (cost model x
                 oracle work units of this workload) / mean launch duration (HIP
                 events on the library stream, inside the timed solves)
  cpu_baseline   the FP64 oracle on the host cores, brute-force neighbours, on a
                 bounded sample of cells of the same workload, in cells/s
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

# FP32 VALU peak of MI355X (published): 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the fast cell kernel from FETCH_SIZE / WRITE_SIZE counters
# (profiles/), valid only for the kernel sources they were taken with
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cells_fast32_dam_break_100k_traffic.json")
TRAFFIC_SOURCES = ("paper_2601_05765_amd/csrc/cells.hip", "paper_2601_05765_amd/csrc/lagot_internal.h")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record():
    """The committed counter profile of the fast cell kernel (HBM bytes per launch, VALU
    issue fraction), or {} when the kernel sources changed since the counters were taken
    (or there is no profile)."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return {}
    if rec.get("sources_sha256") != kernel_sources_digest():
        return {}
    return rec

# Algorithmic FLOPs of one cell evaluation per work unit (FMA = 2, sqrt/div/rcp/atan2 = 1),
# counted from the float32 kernel's arithmetic; the units come from the oracle.
COST = {
    "cand": 16.0,      # bisector setup: offset, |d|^2, rsqrt, t, unit normal
    "test": 5.0,       # vertex versus plane: dot product and compare
    "newv": 21.0,      # new vertex by interpolation along the cut edge
    "face": 12.0,      # facet setup: q, rho^2, cone factor, t*A and signed Omega sums
    "edge": 46.0,      # fan piece with no circle crossing: quadratic + one sector
    "cross": 86.0,     # extra for a crossing piece: roots, two points, second sector, triangle
    "cell": 10.0,      # K and V of the cell
}


def flops_per_cell(work_mean: np.ndarray) -> float:
    cand, tests, newv, faces, edges, cross = work_mean
    return (COST["cand"] * cand + COST["test"] * tests + COST["newv"] * newv + COST["face"] * faces
            + COST["edge"] * edges + COST["cross"] * cross + COST["cell"])


def cpu_baseline(sc, psi, seconds_target: float = 15.0):
    """The oracle (brute-force FP64) on a bounded random sample of cells of the workload."""
    import oracle
    cores = oracle.num_threads()
    rng = np.random.default_rng(7)
    probe = np.sort(rng.choice(sc.n, 400, replace=False))
    t0 = time.perf_counter()
    oracle.cells(sc.x, sc.y, sc.z, psi, idx=probe)
    rate = 400 / max(time.perf_counter() - t0, 1e-6)
    want = max(1000, rate * seconds_target)
    m = int(min(sc.n, want))
    reps = max(1, int(round(want / sc.n))) if m == sc.n else 1  # whole passes when one is short
    idx = np.sort(rng.choice(sc.n, m, replace=False))
    t0 = time.perf_counter()
    for _ in range(reps):
        c = oracle.cells(sc.x, sc.y, sc.z, psi, idx=idx, work=True)
    dt = time.perf_counter() - t0
    what = f"{reps} passes over all {sc.n} cells" if reps > 1 else f"{m} random cells"
    # the same oracle on one core, on a smaller sample (about a quarter of the time budget)
    m1 = int(min(sc.n, max(200, rate / max(oracle.num_threads(), 1) * seconds_target / 4)))
    idx1 = np.sort(rng.choice(sc.n, m1, replace=False))
    t0 = time.perf_counter()
    oracle.cells(sc.x, sc.y, sc.z, psi, idx=idx1, threads=1)
    dt1 = time.perf_counter() - t0
    oracle.cells(sc.x, sc.y, sc.z, psi, idx=idx1[:1], threads=cores)  # back to all threads
    return {"value": reps * m / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"{what} of the {sc.n}-site workload at the start weights, brute-force "
                      f"neighbours, FP64 ({dt:.1f} s)",
            "single_core": {"value": m1 / dt1, "sample": f"{m1} random cells on 1 thread ({dt1:.1f} s)"}}, \
        c.work.mean(axis=0)


def batched_section(ctx, L, scenes, reps: int = 3):
    """256 independent instances (N log-uniform in [500, 50000], slab or sphere cluster) in one
    lagot_solve_batched call, against the same instances solved one at a time."""
    import torch
    insts = scenes.batch_instances(256)
    offs = np.concatenate([[0], np.cumsum([s.n for s in insts])]).astype(np.int64)
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    cat = lambda f: np.concatenate([f(s) for s in insts])
    x, y, z = (t(cat(lambda s: s.x), torch.float32), t(cat(lambda s: s.y), torch.float32),
               t(cat(lambda s: s.z), torch.float32))
    nu, psi0 = t(cat(lambda s: s.nu), torch.float64), t(cat(lambda s: s.psi0), torch.float64)
    opts = L.default_opts(tol=1e-5, autotune=1)
    p = psi0.clone()
    ctx.solve_batched(offs, x, y, z, nu, p, opts=opts)  # warm-up (and autotuning)
    ms = []
    for _ in range(reps):
        p = psi0.clone()
        torch.cuda.synchronize()
        a = time.perf_counter()
        sts = ctx.solve_batched(offs, x, y, z, nu, p, opts=opts)
        torch.cuda.synchronize()
        ms.append(1000.0 * (time.perf_counter() - a))
    assert all(s.status == 0 for s in sts)
    cell_evals = sum(s.evals * (offs[b + 1] - offs[b]) for b, s in enumerate(sts))
    singles = []
    torch.cuda.synchronize()
    a = time.perf_counter()
    for sc in insts:
        ps = t(sc.psi0, torch.float64)
        ctx.solve(t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64),
                  ps, opts=opts)
    torch.cuda.synchronize()
    singles = 1000.0 * (time.perf_counter() - a)
    med = float(np.median(ms))
    return {"instances": 256, "sites": int(offs[-1]), "ms_per_batched_solve": med,
            "cells_per_s": float(cell_evals / (med / 1000.0)),
            "newton_iters_max": max(s.newton_iters for s in sts),
            "newton_iters_mean": float(np.mean([s.newton_iters for s in sts])),
            "max_rel_err": max(s.max_rel_err for s in sts),
            "ms_one_at_a_time": singles, "speedup_vs_one_at_a_time": singles / med}


def learned_section(ctx, L, scenes, n_seeds: int, train_steps: int, steps: int):
    """Learned warm start: train the network on the solver's own pairs (dam-break seeds
    1..n_seeds, train_steps advect-and-solve steps each), then an advect-and-solve sequence
    of a test scene (seed 77) from the previous step's weights, plain and with the guess."""
    import torch
    from paper_2601_05765_amd import warmstart
    t0 = time.perf_counter()
    F, T = warmstart.generate_pairs(ctx, seeds=range(1, n_seeds + 1), n=100_000, steps=train_steps,
                                    log=lambda *a: None)
    t_pairs = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = warmstart.train(ctx, F, T, epochs=8, batch=4096, lr=1e-3, log=lambda *a: None)
    t_train = time.perf_counter() - t0
    sc = scenes.with_velocity(scenes.dam_break(100_000, 77), seed=777)
    x, y, z = (torch.tensor(a, device="cuda") for a in (sc.x, sc.y, sc.z))
    nu, psi = torch.tensor(sc.nu, device="cuda"), torch.tensor(sc.psi0, device="cuda")
    ctx.solve(x, y, z, nu, psi)
    quiet = lambda *a: None
    warmstart.sequence(ctx, sc, 1, psi_start=psi, use_learned=True, log=quiet)  # warm-up
    a = warmstart.sequence(ctx, sc, steps, psi_start=psi, use_learned=False, log=quiet)
    b = warmstart.sequence(ctx, sc, steps, psi_start=psi, use_learned=True, log=quiet)
    return {"pairs": int(F.shape[0]), "s_pairs": t_pairs, "s_train": t_train, "loss_first": hist[0],
            "loss_last": hist[-1], "target_var": float(T.double().var().item()),
            "steps": steps,
            "ms_per_solve_plain": float(np.mean([r["ms"] for r in a])),
            "ms_per_solve_learned": float(np.mean([r["ms"] for r in b])),
            "newton_iters_plain": [r["newton_iters"] for r in a],
            "newton_iters_learned": [r["newton_iters"] for r in b],
            "guess_accepted": [r["learned_accepted"] for r in b],
            "status_plain": [r["status"] for r in a], "status_learned": [r["status"] for r in b]}


def fluid_section(ctx, L, x, y, z, psi, nu, reps: int = 10, steps: int = 5):
    """The fluid step's velocity update (lagot_fluid_velocity: cells and centroids at the
    converged weights, facet weights, right-hand sides, three Jacobi-PCG solves) on the
    bench workload, per-site viscosity in [0, 2], density 1 (m = nu); then whole fluid
    steps (lagot_fluid_step) from rest under gravity."""
    import torch
    n = x.shape[0]
    g = torch.Generator(device="cuda").manual_seed(3)
    v = torch.randn((n, 3), generator=g, dtype=torch.float64, device="cuda")
    mu = 2.0 * torch.rand(n, generator=g, dtype=torch.float64, device="cuda")
    prm = L.default_fluid_params(dt=2e-3, eps=0.02, gamma=0.05)
    for _ in range(2):
        ctx.fluid_velocity(x, y, z, psi, nu, v, prm, mu=mu)
    torch.cuda.synchronize()
    ms, its = [], None
    for _ in range(reps):
        a = time.perf_counter()
        _, _, its = ctx.fluid_velocity(x, y, z, psi, nu, v, prm, mu=mu)
        torch.cuda.synchronize()
        ms.append(1000.0 * (time.perf_counter() - a))
    # whole steps of the dam break from rest (move, re-solve from the last weights, update
    # the velocities), on copies of the sites
    xs, ys, zs, ps = x.clone(), y.clone(), z.clone(), psi.clone()
    vs = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    step_ms, newton = [], []
    for _ in range(steps):
        a = time.perf_counter()
        st, _ = ctx.fluid_step(xs, ys, zs, nu, ps, nu, vs, prm, opts=L.default_opts(tol=1e-5), mu=mu)
        torch.cuda.synchronize()
        step_ms.append(1000.0 * (time.perf_counter() - a))
        newton.append(st.newton_iters)
    return {"ms_fluid_velocity": float(np.median(ms)), "pcg_iters": its, "dt": prm.dt, "eps": prm.eps,
            "gamma": prm.gamma, "mu": "per site, uniform in [0, 2]", "ms_per_fluid_step": step_ms,
            "newton_iters_per_step": newton}


def splash_section(ctx, L, scenes, n: int, steps: int):
    """The large-scene recipe (slab + 200 over-packed droplets, log-normal nu, random
    velocities) at n sites: the first solve from the Voronoi start, then `steps`
    advect-and-solve steps warm-started from the previous weights. Step sizes use the
    min-volume test alone (Algorithm 1 as printed), which does not stall on the float32
    noise floor near the tolerance."""
    import torch
    sc = scenes.splash(n, 0)
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    nu, psi = t(sc.nu, torch.float64), t(sc.psi0, torch.float64)
    opts = L.default_opts(tol=1e-5, autotune=1, residual_test=0)
    out = {"sites": n, "steps": steps, "ms": [], "newton_iters": [], "evals": [], "status": [], "restarted": [],
           "max_rel_err": []}
    cur = sc
    for k in range(steps + 1):
        if k:
            cur = scenes.advect(cur, 2e-3)
        x, y, z = t(cur.x, torch.float32), t(cur.y, torch.float32), t(cur.z, torch.float32)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = ctx.solve(x, y, z, nu, psi, opts=opts, check=False)
        torch.cuda.synchronize()
        out["ms"].append(1000.0 * (time.perf_counter() - a))
        out["newton_iters"].append(st.newton_iters)
        out["evals"].append(st.evals)
        out["status"].append(st.status)
        out["restarted"].append(st.default_start)
        out["max_rel_err"].append(st.max_rel_err)
    out["ms_settle"] = out["ms"][0]
    out["ms_per_step"] = float(np.mean(out["ms"][1:])) if steps else None
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eval-reps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched solve")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--learned-seeds", type=int, default=6, help="training scenes (100k sites each)")
    ap.add_argument("--learned-steps", type=int, default=4, help="advect-and-solve steps per training scene")
    ap.add_argument("--sequence-steps", type=int, default=5)
    ap.add_argument("--no-splash", action="store_true", help="skip the over-packed splash sequence")
    ap.add_argument("--no-fluid", action="store_true", help="skip the fluid-step velocity update")
    ap.add_argument("--splash-n", type=int, default=200_000)
    ap.add_argument("--splash-steps", type=int, default=5)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is not "
              f"built", file=sys.stderr)
        return 2

    import torch
    import paper_2601_05765_amd as L
    from paper_2601_05765_amd import scenes
    if not os.path.exists(L.LIB_PATH):
        from paper_2601_05765_amd import build
        build.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    sc = scenes.dam_break(args.n, 0)
    dev = "cuda"
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    x, y, z, nu = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64)
    psi0 = t(sc.psi0, torch.float64)
    ctx = L.Context()
    # the autotuner picks lanes per cell and the PCG block shape during the warm-up
    opts = L.default_opts(tol=1e-5, autotune=1)

    for _ in range(args.warmup):
        p = psi0.clone()
        ctx.solve(x, y, z, nu, p, opts=opts)
    psis = [psi0.clone() for _ in range(args.steps)]
    torch.cuda.synchronize()
    stats = []
    per_solve = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        stats.append(ctx.solve(x, y, z, nu, psis[k], opts=opts))  # returns after the stream is synchronised
        per_solve.append(1000.0 * (time.perf_counter() - a))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    evals = sum(s.evals for s in stats)
    value = args.n * evals / wall
    launches = sum(s.cell_launches for s in stats)
    ms_kernel = sum(s.ms_cell_kernel for s in stats) / max(launches, 1)
    s0 = stats[-1]

    # evaluation alone (lagot_cells: validation, grid build, cells, outputs), at the start
    # weights and at the converged ones; and with centroids (lagot_centroids)
    def eval_times(psi_eval, fn):
        for _ in range(3):
            fn(psi_eval)
        torch.cuda.synchronize()
        ev, kk = [], []
        for _ in range(args.eval_reps):
            a = time.perf_counter()
            fn(psi_eval)
            torch.cuda.synchronize()
            ev.append(1000.0 * (time.perf_counter() - a))
            kk.append(ctx.last_cell_kernel_ms())
        return float(np.median(ev)), float(np.median(kk))

    cells_fn = lambda p: ctx.cells(x, y, z, p, csr=False, walls=False)
    ev0, k0 = eval_times(psi0, cells_fn)
    ev1, k1 = eval_times(psis[-1], cells_fn)
    evc, kc = eval_times(psis[-1], lambda p: ctx.centroids(x, y, z, p))

    line = {
        "metric": "cells/s (Laguerre∩ball eval); ms per OT solve to 1e-5 vol err, plain vs learned",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dam_break_{args.n}: jittered cubic lattice in the lower 40% of the unit box, "
                               f"nu=0.35/N, one plain OT solve to 1e-5 relative volume error",
                   "n_sites": args.n, "tol": 1e-5},
        "solve": {"ms_per_solve_plain": ms_per_step, "ms_per_solve_median": float(np.median(per_solve)),
                  "newton_iters": s0.newton_iters, "evals": s0.evals,
                  "halvings": s0.halvings, "cg_iters": s0.cg_iters, "max_rel_err": s0.max_rel_err,
                  "fallback_cells": s0.fallback_cells, "ms_eval": s0.ms_eval, "ms_linear": s0.ms_linear},
        "eval_only": {"cells_per_s_with_grid": args.n / (ev0 / 1000.0), "cells_per_s_kernel": args.n / (k0 / 1000.0),
                      "ms_lagot_cells": ev0, "ms_cell_kernel": k0,
                      "converged": {"cells_per_s_with_grid": args.n / (ev1 / 1000.0),
                                    "cells_per_s_kernel": args.n / (k1 / 1000.0), "ms_lagot_cells": ev1,
                                    "ms_cell_kernel": k1},
                      "centroids_converged": {"ms_lagot_centroids": evc, "ms_cell_kernel": kc,
                                              "cells_per_s_kernel": args.n / (kc / 1000.0)}},
    }
    if not args.no_fluid:
        line["fluid"] = fluid_section(ctx, L, x, y, z, psis[-1], nu)
    if not args.no_batched:
        line["batched"] = batched_section(ctx, L, scenes)
    if not args.no_splash:
        line["splash"] = splash_section(ctx, L, scenes, args.splash_n, args.splash_steps)
    if not args.no_learned:
        line["learned"] = learned_section(ctx, L, scenes, args.learned_seeds, args.learned_steps,
                                          args.sequence_steps)
    work_mean = None
    if not args.no_cpu_baseline:
        cb, work_start = cpu_baseline(sc, sc.psi0, args.cpu_seconds)
        line["cpu_baseline"] = cb
        # the solve evaluates cells from the start weights to the converged ones: average the
        # oracle's work units at both ends (a 2,000-cell sample at the converged weights)
        import oracle
        idx = np.sort(np.random.default_rng(8).choice(sc.n, min(2000, sc.n), replace=False))
        cw = oracle.cells(sc.x, sc.y, sc.z, psis[-1].cpu().numpy(), idx=idx, work=True)
        work_mean = 0.5 * (work_start + cw.work.mean(axis=0))
    if work_mean is not None:
        fpc = flops_per_cell(work_mean)
        achieved = fpc * args.n / (ms_kernel / 1000.0) / 1e12
        line["roofline"] = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": counter_record().get("bytes_per_launch"),
                            "valu_issue_frac": counter_record().get("valu_issue_frac"),
                            "kernel": "k_cells_fast<32, false> (fused clip + ball integration, float32)",
                            "flops_per_cell": fpc, "ms_per_launch": ms_kernel,
                            "work_units_per_cell": dict(zip(["cand", "tests", "newv", "faces", "edges", "cross"],
                                                            [float(v) for v in work_mean]))}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
