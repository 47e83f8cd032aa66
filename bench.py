#!/usr/bin/env python3
"""Benchmark of the analytic partial-OT solver on one MI355X.

Workload (the measured configuration, the largest single-GPU one): the 2M-site
splash scene -- a jittered lattice slab (60% of the sites) and 200 droplets of
log-normal radius packed 1.72x denser than their prescribed volumes, log-normal
prescribed volumes summing to 0.3, random velocities N(0, 0.5^2) per axis. The
scene is settled from its Voronoi start (path following on the prescribed
volumes), then advected by dt = 2e-3 per step (mirror reflection at the walls)
and solved again, each solve warm-started from the previous step's weights.
float32 geometry, float64 weights, reductions and CG.

A step is one advect-and-solve step of that sequence: every Newton evaluation of
all cells (including the crowded-cell passes), Hessian assembly, Jacobi-PCG and
KMT step control, to max |V_i - nu_i| / nu_i <= 1e-5. The positions of every step
are computed before timing and are resident in HBM. Warm-up: the settle, then
W - 1 untimed steps; the K timed steps follow.

Printed (one JSON line):
  value          Laguerre cell evaluations per second over the timed steps
                 (N x evaluations / wall time)
  ms_per_step    ms per advect-and-solve step (one OT solve)
  roofline       the dominant kernel of the step (see the design doc for the model)
  cpu_baseline   the FP64 oracle on the host cores, brute-force neighbours, on a
                 bounded sample of cells of the settled scene, in cells/s
  c3             settle time, per-step ms, Newton iterations, evaluations, and the
                 oracle-sampled error of the final weights (heaviest sites + random)
Sections: dam_break (the 100k-site configuration), batched, fluid, learned.

Profiling modes (no JSON line): --profile c3 | cells | fluid runs a short piece of
the workload for rocprofv3 (c3: settle and two steps; cells: one dam-break solve
and a 256 MiB device copy that calibrates the byte counters; fluid: five velocity
updates of the dam break).
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

# VALU peaks of MI355X (published): 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz
# for FP32; FP64 vector is half of it
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
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


def flops_per_cell_minimal_clip(work_mean: np.ndarray) -> float:
    """The cost model with the clip term of a minimal clipper: each of the cell's own F
    planes (facets and walls) set up and clipped once against a polytope of at most 2F
    vertices (F^2 vertex tests, 2F new vertices), plus the integration units of the final
    cell. For crowded cells the oracle's candidate counts (every bisector that cuts the
    ball, thousands there) measure its brute force, not the work the method needs."""
    _, _, _, faces, edges, cross = work_mean
    return (COST["cand"] * faces + COST["test"] * faces * faces + COST["newv"] * 2.0 * faces
            + COST["face"] * faces + COST["edge"] * edges + COST["cross"] * cross + COST["cell"])


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


def sample_idx(n, psi, seed, k_top=100, k_rand=300):
    """The heaviest sites (the most crowded cells) and a random sample."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.argsort(-psi)[:k_top], rng.choice(n, min(k_rand, n), replace=False)]))


def oracle_error(x, y, z, psi, nu, idx):
    """max and p99 over the sampled cells of |V_i - nu_i| / nu_i, the volumes V_i of the
    returned weights evaluated by the FP64 oracle (brute-force neighbours)."""
    import oracle
    c = oracle.cells(x, y, z, psi, idx=idx)
    e = np.abs(c.V - nu[idx]) / nu[idx]
    return {"cells": int(len(idx)), "max_rel_err": float(e.max()), "p99_rel_err": float(np.percentile(e, 99))}


def c3_sequence(ctx, L, scenes, n: int, warmup: int, steps: int, log):
    """The settle and the advect-and-solve steps of the 2M-site splash scene. Positions of
    every step are computed and uploaded before the timed steps."""
    import torch
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    sc = scenes.splash(n, 0)
    seq, cur = [], sc
    for _ in range(max(warmup, 1) - 1 + steps):
        cur = scenes.advect(cur, 2e-3)
        seq.append(cur)
    pos = [(t(s.x, torch.float32), t(s.y, torch.float32), t(s.z, torch.float32)) for s in seq]
    nu, psi = t(sc.nu, torch.float64), t(sc.psi0, torch.float64)
    x0, y0, z0 = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32)
    settle_opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1)
    step_opts = L.default_opts(tol=1e-5, residual_test=0)
    torch.cuda.synchronize()
    a = time.perf_counter()
    st = ctx.solve(x0, y0, z0, nu, psi, opts=settle_opts, check=False)
    torch.cuda.synchronize()
    settle_ms = 1000.0 * (time.perf_counter() - a)
    if st.status != 0:
        raise RuntimeError(f"settle of the splash scene failed: {st.as_dict()}")
    log(f"c3 settle: {settle_ms:.0f} ms, {st.newton_iters} Newton iterations, {st.stages} stages")
    settle = {"ms": settle_ms, "newton_iters": st.newton_iters, "evals": st.evals, "stages": st.stages,
              "halvings": st.halvings, "cg_iters": st.cg_iters, "max_rel_err": st.max_rel_err}
    prev = torch.empty_like(psi)

    def step(k):
        x, y, z = pos[k]
        prev.copy_(psi)
        s1 = ctx.solve(x, y, z, nu, psi, opts=step_opts, check=False)
        kt = ctx.last_kernel_times()
        retried = False
        if s1.status != 0:  # Algorithm 1 stalled: the same step again with path following
            psi.copy_(prev)
            s1 = ctx.solve(x, y, z, nu, psi, opts=settle_opts, check=False)
            kt = ctx.last_kernel_times()
            retried = True
        if s1.status != 0:
            raise RuntimeError(f"step {k} of the splash sequence failed: {s1.as_dict()}")
        return s1, kt, retried

    for k in range(max(warmup, 1) - 1):
        step(k)
    k0 = max(warmup, 1) - 1
    out = {"ms": [], "newton_iters": [], "evals": [], "halvings": [], "cg_iters": [], "restarted": [],
           "retried": [], "parts": [], "ms_eval": [], "ms_linear": [], "kernel_times": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(k0, k0 + steps):
        a = time.perf_counter()
        s1, kt, retried = step(k)  # returns after the stream is synchronised
        out["ms"].append(1000.0 * (time.perf_counter() - a))
        out["newton_iters"].append(s1.newton_iters)
        out["evals"].append(s1.evals)
        out["halvings"].append(s1.halvings)
        out["cg_iters"].append(s1.cg_iters)
        out["restarted"].append(s1.default_start)
        out["retried"].append(int(retried))
        out["parts"].append(s1.stages)  # continuation stages of a retried step
        out["ms_eval"].append(s1.ms_eval)
        out["ms_linear"].append(s1.ms_linear)
        out["kernel_times"].append(kt)
        log(f"c3 step {k + 1}: {out['ms'][-1]:.0f} ms, {s1.newton_iters} Newton iterations, {s1.evals} evaluations")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"scene": seq[k0 + steps - 1], "nu": sc.nu, "psi": psi, "settle": settle, "steps": out, "wall": wall,
            "n": n}


def copy_calibration():
    """A 256 MiB device-to-device copy (256 MiB read, 256 MiB written): the byte counters'
    reading for a known number of bytes."""
    import torch
    copy_bytes = 256 * 1024 * 1024
    a = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile: copy of {copy_bytes} bytes done", flush=True)


def profile_mode(which: str) -> int:
    """Short runs for rocprofv3 (no JSON line)."""
    import torch
    import paper_2601_05765_amd as L
    from paper_2601_05765_amd import scenes
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    ctx = L.Context()
    if which == "c3":
        r = c3_sequence(ctx, L, scenes, 2_000_000, 1, 2, lambda m: print("profile c3:", m, flush=True))
        print(f"profile c3: done, {r['steps']['evals']} evaluations per step", flush=True)
        copy_calibration()
    elif which in ("cells", "fluid"):
        n = 100_000
        sc = scenes.dam_break(n, 0)
        x, y, z, nu = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64)
        psi = t(sc.psi0, torch.float64)
        ctx.set_threads_per_cell(32)
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5))
        print(f"profile {which}: dam_break {n} solve, {st.evals} evaluations, status {st.status}", flush=True)
        if which == "cells":
            copy_calibration()
        else:
            g = torch.Generator(device="cuda").manual_seed(3)
            v = torch.randn((n, 3), generator=g, dtype=torch.float64, device="cuda")
            mu = 2.0 * torch.rand(n, generator=g, dtype=torch.float64, device="cuda")
            prm = L.default_fluid_params(dt=2e-3, eps=0.02, gamma=0.05)
            for k in range(5):
                _, _, its = ctx.fluid_velocity(x, y, z, psi, nu, v, prm, mu=mu)
                print(f"profile fluid: velocity update {k}: PCG iterations {its}", flush=True)
    else:
        print(f"unknown profile mode {which}", file=sys.stderr)
        return 2
    torch.cuda.synchronize()
    return 0


def dam_break_section(ctx, L, scenes, n: int, steps: int, warmup: int, eval_reps: int):
    """The 100k-site dam break: plain OT solves from the start weights (autotuned shapes),
    one evaluation alone (with and without the grid build) at the start and converged
    weights, and with centroids."""
    import torch
    sc = scenes.dam_break(n, 0)
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    x, y, z, nu = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64)
    psi0 = t(sc.psi0, torch.float64)
    opts = L.default_opts(tol=1e-5, autotune=1)
    for _ in range(warmup):
        p = psi0.clone()
        ctx.solve(x, y, z, nu, p, opts=opts)
    psis = [psi0.clone() for _ in range(steps)]
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for k in range(steps):
        stats.append(ctx.solve(x, y, z, nu, psis[k], opts=opts))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s0 = stats[-1]
    launches = sum(s.cell_launches for s in stats)
    ms_kernel = sum(s.ms_cell_kernel for s in stats) / max(launches, 1)

    def eval_times(psi_eval, fn):
        for _ in range(3):
            fn(psi_eval)
        torch.cuda.synchronize()
        ev, kk = [], []
        for _ in range(eval_reps):
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
    p_last = psis[-1].cpu().numpy()
    err = oracle_error(sc.x, sc.y, sc.z, p_last, sc.nu, sample_idx(n, p_last, 5, k_top=0, k_rand=300))
    sec = {"workload": f"dam_break_{n}: jittered cubic lattice in the lower 40% of the unit box, nu=0.35/N, one "
                       f"plain OT solve from the start weights to 1e-5",
           "cells_per_s": n * sum(s.evals for s in stats) / wall, "ms_per_solve": 1000.0 * wall / steps,
           "newton_iters": s0.newton_iters, "evals": s0.evals, "halvings": s0.halvings, "cg_iters": s0.cg_iters,
           "max_rel_err": s0.max_rel_err, "ms_eval": s0.ms_eval, "ms_linear": s0.ms_linear,
           "ms_cell_kernel": ms_kernel, "oracle_error": err,
           "eval_only": {"cells_per_s_with_grid": n / (ev0 / 1000.0), "cells_per_s_kernel": n / (k0 / 1000.0),
                         "ms_lagot_cells": ev0, "ms_cell_kernel": k0,
                         "converged": {"cells_per_s_with_grid": n / (ev1 / 1000.0),
                                       "cells_per_s_kernel": n / (k1 / 1000.0), "ms_lagot_cells": ev1,
                                       "ms_cell_kernel": k1},
                         "centroids_converged": {"ms_lagot_centroids": evc, "ms_cell_kernel": kc,
                                                 "cells_per_s_kernel": n / (kc / 1000.0)}}}
    return sec, (sc, x, y, z, nu, psis[-1])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed advect-and-solve steps of the 2M-site sequence")
    ap.add_argument("--warmup", type=int, default=2, help="the settle, then warmup - 1 untimed steps")
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--profile", choices=["c3", "cells", "fluid"], default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eval-reps", type=int, default=20)
    ap.add_argument("--no-dam-break", action="store_true", help="skip the 100k dam-break section")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched solve")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start comparison")
    ap.add_argument("--learned-seeds", type=int, default=6, help="training scenes (100k sites each)")
    ap.add_argument("--learned-steps", type=int, default=4, help="advect-and-solve steps per training scene")
    ap.add_argument("--sequence-steps", type=int, default=5)
    ap.add_argument("--no-fluid", action="store_true", help="skip the fluid-step velocity update")
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
    if args.profile:
        return profile_mode(args.profile)
    log = lambda m: print(m, file=sys.stderr, flush=True)

    ctx = L.Context()
    r = c3_sequence(ctx, L, scenes, args.n, args.warmup, args.steps, log)
    st3 = r["steps"]
    wall = r["wall"]
    n = args.n
    evals = sum(st3["evals"])
    value = n * evals / wall
    ms_per_step = 1000.0 * wall / args.steps
    fin = r["scene"]
    p_fin = r["psi"].cpu().numpy()
    c3_err = oracle_error(fin.x, fin.y, fin.z, p_fin, r["nu"], sample_idx(n, p_fin, 3))
    kt = st3["kernel_times"]
    fast_ms = sum(k["fast_ms"] for k in kt) / max(sum(k["fast_launches"] for k in kt), 1)
    crowd_launches = sum(k["crowd_launches"] for k in kt)
    crowd_ms = sum(k["crowd_ms"] for k in kt) / max(crowd_launches, 1)
    crowd_cells = sum(k["crowd_cells"] for k in kt) / max(crowd_launches, 1)
    # roofline of the dominant kernel, the crowded-cell pass (float64): algorithmic FLOPs per
    # cell from the oracle's geometry of a sample of the cells it finishes at the final state
    xf, yf, zf = (torch.tensor(np.ascontiguousarray(a), device="cuda") for a in (fin.x, fin.y, fin.z))
    ctx.cells(xf, yf, zf, r["psi"], csr=False, walls=False)
    deferred = ctx.last_deferred()
    import oracle
    rs = np.random.default_rng(11)
    samp = np.sort(rs.choice(deferred, min(300, len(deferred)), replace=False)) if len(deferred) else None
    roofline = None
    if samp is not None and crowd_ms > 0:
        w = oracle.cells(fin.x, fin.y, fin.z, p_fin, idx=samp, work=True).work.mean(axis=0)
        fpc = flops_per_cell_minimal_clip(w)
        achieved = fpc * crowd_cells / (crowd_ms / 1000.0) / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                    "kernel": "k_cells_overflow (crowded cells: box-overlap candidates, clip rounds, integration; "
                              "float64)",
                    "flops_per_cell": fpc, "cells_per_launch": crowd_cells, "ms_per_launch": crowd_ms,
                    "launches": crowd_launches,
                    "work_units_per_cell": dict(zip(["cand", "tests", "newv", "faces", "edges", "cross"],
                                                    [float(v) for v in w])),
                    "model": "cost model with a minimal clip term (each facet plane clipped once), oracle units "
                             "of 300 sampled crowded cells"}
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
        "config": {"workload": f"splash_{n}: 60% jittered-lattice slab + 200 log-normal droplets packed 1.72x, "
                               f"log-normal nu summing to 0.3, random velocities N(0, 0.5^2); settled from the "
                               f"Voronoi start, then advect (dt 2e-3) and solve to 1e-5 per step, warm-started "
                               f"from the previous weights",
                   "n_sites": n, "tol": 1e-5, "dt": 2e-3},
        "c3": {"settle": r["settle"], "ms_per_step": ms_per_step, "ms_steps": st3["ms"],
               "newton_iters": st3["newton_iters"], "evals": st3["evals"], "halvings": st3["halvings"],
               "cg_iters": st3["cg_iters"], "restarted": st3["restarted"], "retried": st3["retried"],
               "stages": st3["parts"],
               "ms_eval": st3["ms_eval"], "ms_linear": st3["ms_linear"],
               "ms_fast_kernel_per_eval": fast_ms, "ms_crowded_pass_per_eval": crowd_ms,
               "crowded_cells_per_eval": crowd_cells, "oracle_error": c3_err},
    }
    if roofline is not None:
        line["roofline"] = roofline
    if not args.no_dam_break:
        sec, dam = dam_break_section(ctx, L, scenes, 100_000, 10, 3, args.eval_reps)
        line["dam_break"] = sec
        if not args.no_fluid:
            _, x, y, z, nu, psi = dam
            line["fluid"] = fluid_section(ctx, L, x, y, z, psi, nu)
    if not args.no_batched:
        line["batched"] = batched_section(ctx, L, scenes)
    if not args.no_learned:
        line["learned"] = learned_section(ctx, L, scenes, args.learned_seeds, args.learned_steps,
                                          args.sequence_steps)
    if not args.no_cpu_baseline:
        cb, work = cpu_baseline(fin, p_fin, args.cpu_seconds)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
