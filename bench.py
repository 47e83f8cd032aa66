#!/usr/bin/env python3
"""Benchmark of the analytic partial-OT solver on one MI355X.

Workload (the measured configuration, the largest single-GPU one): the 2M-site
splash scene -- a jittered lattice slab (60% of the sites) and 200 droplets of
log-normal radius packed 1.72x denser than their prescribed volumes, log-normal
prescribed volumes summing to 0.3, random velocities N(0, 0.5^2) per axis. The
scene is settled from its Voronoi start (path following on the prescribed
volumes), then advected by dt = 2e-3 per step (mirror reflection at the walls)
and solved again, each solve from the previous step's weights (repaired where they
leave cells empty, else the default start) with the same path following.
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
  roofline       the dominant kernel of the step, the crowded-cell pass: algorithmic
                 FLOPs per launch (cost model over the oracle's work units) / launch
                 time against the FP64 peak, with its counter record (HBM bytes per
                 launch, VALU issue fraction) when the sources match
  cpu_baseline   the FP64 oracle on the host cores, brute-force neighbours, on a
                 bounded sample of cells of the settled scene, in cells/s
  c3             settle time, per-step ms, Newton iterations, evaluations, and the
                 oracle-sampled error of the final weights (heaviest sites + random)
Sections: dam_break (the 100k-site configuration), paper_k_route (the A/B pair of the
spherical area on its converged cells), batched, fluid, learned; each carries its
error against the FP64 oracle (oracle_error), computed after all GPU timing.

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

# Newton directions to a relative PCG residual of 1e-3 (inexact Newton): the stop test is
# on the volumes (max |V_i - nu_i| / nu_i <= 1e-5) whatever the direction's accuracy; on
# the workloads here the Newton iterations and evaluations are those of 1e-6 directions
CG_RTOL = 1e-3

# HBM bytes per launch of the crowded-cell pass from FETCH_SIZE / WRITE_SIZE counters and its
# VALU issue fraction from SQ_INSTS_VALU / GRBM_GUI_ACTIVE (profiles/; written by
# --counters-summary from the rocprofv3 runs the record names), valid only for the kernel
# sources they were taken with
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cells_overflow_splash_2m_counters.json")
TRAFFIC_SOURCES = ("paper_2601_05765_amd/csrc/cells.hip", "paper_2601_05765_amd/csrc/lagot_internal.h")


def kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_record():
    """The committed counter profile of the crowded-cell pass (HBM bytes per launch, VALU
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
            "sample": f"{what} of the {sc.n}-site workload at the weights of the last step, brute-force "
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
    opts = L.default_opts(tol=1e-5, autotune=1, cg_rtol=CG_RTOL)
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
    # the same call with the launch sequences captured as HIP graphs (opts.use_graph)
    gopts = L.default_opts(tol=1e-5, autotune=1, cg_rtol=CG_RTOL, use_graph=1)
    pg = psi0.clone()
    ctx.solve_batched(offs, x, y, z, nu, pg, opts=gopts)  # capture
    ms_graph = []
    for _ in range(reps):
        pg = psi0.clone()
        torch.cuda.synchronize()
        a = time.perf_counter()
        sg = ctx.solve_batched(offs, x, y, z, nu, pg, opts=gopts)
        torch.cuda.synchronize()
        ms_graph.append(1000.0 * (time.perf_counter() - a))
    assert all(s.status == 0 for s in sg)
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
    p_fin = p.cpu().numpy()

    def check():
        # eight instances spread over the size range: the heaviest sites and a random sample of each
        order = np.argsort([sc.n for sc in insts])
        errs = []
        for k, b in enumerate(order[np.linspace(0, len(insts) - 1, 8).astype(int)]):
            sc, pb = insts[b], p_fin[offs[b]:offs[b + 1]]
            errs.append(cell_errors(sc.x, sc.y, sc.z, pb, sc.nu, sample_idx(sc.n, pb, 40 + k, k_top=5, k_rand=40)))
        return summarize(np.concatenate(errs), "8 instances spread over the sizes, 5 heaviest + 40 random cells each")

    return {"instances": 256, "sites": int(offs[-1]), "ms_per_batched_solve": med,
            "cells_per_s": float(cell_evals / (med / 1000.0)),
            "newton_iters_max": max(s.newton_iters for s in sts),
            "newton_iters_mean": float(np.mean([s.newton_iters for s in sts])),
            "max_rel_err": max(s.max_rel_err for s in sts),
            "ms_one_at_a_time": singles, "speedup_vs_one_at_a_time": singles / med,
            "ms_per_batched_solve_graphs": float(np.median(ms_graph))}, check


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
    warmstart.sequence(ctx, sc, 1, psi_start=psi, use_learned=True, log=quiet, cg_rtol=CG_RTOL)  # warm-up
    a = warmstart.sequence(ctx, sc, steps, psi_start=psi, use_learned=False, log=quiet, cg_rtol=CG_RTOL)
    last = {}
    b = warmstart.sequence(ctx, sc, steps, psi_start=psi, use_learned=True, log=quiet, cg_rtol=CG_RTOL, state=last)
    fin, p_fin = last["scene"], last["psi"].cpu().numpy()
    check = lambda: oracle_error(fin.x, fin.y, fin.z, p_fin, fin.nu, sample_idx(fin.n, p_fin, 13, k_top=0),
                                 "300 random cells of the learned sequence's last step")
    return {"pairs": int(F.shape[0]), "s_pairs": t_pairs, "s_train": t_train, "loss_first": hist[0],
            "loss_last": hist[-1], "target_var": float(T.double().var().item()),
            "steps": steps,
            "ms_per_solve_plain": float(np.mean([r["ms"] for r in a])),
            "ms_per_solve_learned": float(np.mean([r["ms"] for r in b])),
            "newton_iters_plain": [r["newton_iters"] for r in a],
            "newton_iters_learned": [r["newton_iters"] for r in b],
            "guess_accepted": [r["learned_accepted"] for r in b],
            "ms_guess": [r["ms_learned"] for r in b],  # inputs, network and trial evaluations per solve
            "status_plain": [r["status"] for r in a], "status_learned": [r["status"] for r in b]}, check


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
    ms, its, vn = [], None, None
    for _ in range(reps):
        a = time.perf_counter()
        vn, _, its = ctx.fluid_velocity(x, y, z, psi, nu, v, prm, mu=mu)
        torch.cuda.synchronize()
        ms.append(1000.0 * (time.perf_counter() - a))
    # whole steps of the dam break from rest (move, re-solve from the last weights, update
    # the velocities), on copies of the sites
    xs, ys, zs, ps = x.clone(), y.clone(), z.clone(), psi.clone()
    vs = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    step_ms, newton = [], []
    for _ in range(steps):
        a = time.perf_counter()
        st, _ = ctx.fluid_step(xs, ys, zs, nu, ps, nu, vs, prm, opts=L.default_opts(tol=1e-5, cg_rtol=CG_RTOL), mu=mu)
        torch.cuda.synchronize()
        step_ms.append(1000.0 * (time.perf_counter() - a))
        newton.append(st.newton_iters)
    data = [a.cpu().numpy() for a in (x, y, z, psi, nu, v, mu, vn)]

    def check():
        import oracle
        xs_, ys_, zs_, ps_, nus_, v_, mu_, vn_ = data
        xyz = np.stack([xs_, ys_, zs_], 1).astype(np.float64)
        o = oracle.fluid_velocity(xyz, ps_, v_, nus_, mu_, dt=prm.dt, eps=prm.eps, gamma=prm.gamma,
                                  gravity=tuple(prm.gravity), solver="cg")
        e = np.linalg.norm(vn_ - o.v, axis=1) / np.linalg.norm(o.v, axis=1)
        return summarize(e, f"|v_i - v_i(oracle)| / |v_i(oracle)| over all {len(e)} sites (oracle: every cell, "
                            f"eq. (4) by FP64 Jacobi-PCG to 1e-13)")

    return {"ms_fluid_velocity": float(np.median(ms)), "pcg_iters": its, "dt": prm.dt, "eps": prm.eps,
            "gamma": prm.gamma, "mu": "per site, uniform in [0, 2]", "ms_per_fluid_step": step_ms,
            "newton_iters_per_step": newton}, check


def paper_k_section(ctx, x, y, z, psi, reps: int = 5):
    """The A/B pair of the spherical area: lagot_cells (signed solid angles at p_i, float32
    fast pass) against lagot_cells_paper_k (section 3.3's own route: interior point,
    projected facets, Gauss-Bonnet; every cell on the float64 path), on the same cells."""
    import torch

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        wall, kern = [], []
        for _ in range(reps):
            a = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            wall.append(1000.0 * (time.perf_counter() - a))
            kern.append(ctx.last_cell_kernel_ms())
        return out, float(np.median(wall)), float(np.median(kern))

    sg, w_sg, k_sg = timed(lambda: ctx.cells(x, y, z, psi, csr=False, walls=False)["sph"])
    (_, kr), w_kr, k_kr = timed(lambda: ctx.cells_paper_k(x, y, z, psi))
    area = 4.0 * math.pi * psi
    d = ((kr - sg).abs() / area).max().item()
    data = [a.cpu().numpy() for a in (x, y, z, psi, kr)]

    def check():
        import oracle
        xs, ys, zs, ps, kk = data
        idx = sample_idx(len(ps), ps, 9, k_top=0, k_rand=300)
        c = oracle.cells(xs, ys, zs, ps, idx=idx, paper_k=True)
        e = np.abs(kk[idx] - c.Kp) / (4.0 * math.pi * ps[idx])
        return summarize(e, "|K_i(route) - K_i(oracle route)| / 4 pi r_i^2, 300 random cells")

    return {"ms_lagot_cells": w_sg, "ms_cell_kernel_signed": k_sg, "ms_lagot_cells_paper_k": w_kr,
            "ms_cell_kernel_paper_k": k_kr, "kernel_ratio": k_kr / max(k_sg, 1e-9),
            "max_rel_diff_K": d, "diff_normalised_by": "4 pi r_i^2"}, check


def domain_section(ctx, L, scenes, n: int = 100_000, reps: int = 3):
    """A non-convex domain: n sites in the L-shaped prism (the unit box less the quarter
    x, y > 1/2) given as 3 convex pieces. Evaluation time against the same sites in the
    unit box (one convex domain), and a solve from the default start to 1e-5."""
    import torch
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    sc = scenes.l_shape_sites(n, 0)
    pieces = scenes.l_shape_pieces()
    x, y, z = t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32)
    psi0 = scenes.default_psi0(sc.nu)
    nu = t(sc.nu, torch.float64)

    def eval_ms():
        p = t(psi0, torch.float64)
        ctx.cells(x, y, z, p, csr=False, walls=False)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a = time.perf_counter()
            ctx.cells(x, y, z, p, csr=False, walls=False)
            torch.cuda.synchronize()
            ms.append(1000.0 * (time.perf_counter() - a))
        return float(np.median(ms))

    ms_box = eval_ms()
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        ms_l = eval_ms()
        psi = t(psi0, torch.float64)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5), check=False)
        torch.cuda.synchronize()
        ms_solve = 1000.0 * (time.perf_counter() - a)
    finally:
        ctx.set_domain(None)
    if st.status != 0:
        raise RuntimeError(f"solve in the L prism failed: {st.as_dict()}")
    data = (sc.x, sc.y, sc.z, psi.cpu().numpy(), sc.nu)

    def check():
        import oracle
        xs, ys, zs, ps, nus = data
        idx = np.sort(np.random.default_rng(13).choice(len(ps), 300, replace=False))
        c = oracle.cells_pieces(xs, ys, zs, ps, pieces, scenes.L_WALLS, idx=idx)
        return summarize(np.abs(c.V - nus[idx]) / nus[idx], "|V_i - nu_i| / nu_i of 300 random cells")

    return {"workload": f"{n} sites uniform in the L-shaped prism [0,1]^3 less x, y > 1/2, 3 convex pieces, "
                        f"nu = 0.375 / n, default start", "n_sites": n, "pieces": len(pieces),
            "ms_lagot_cells_l_prism": ms_l, "ms_lagot_cells_unit_box": ms_box, "eval_ratio": ms_l / ms_box,
            "solve": {"ms": ms_solve, "newton_iters": st.newton_iters, "evals": st.evals,
                      "halvings": st.halvings, "max_rel_err": st.max_rel_err}}, check


def sample_idx(n, psi, seed, k_top=100, k_rand=300):
    """The heaviest sites (the most crowded cells) and a random sample."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.argsort(-psi)[:k_top], rng.choice(n, min(k_rand, n), replace=False)]))


def cell_errors(x, y, z, psi, nu, idx):
    """|V_i - nu_i| / nu_i of the sampled cells, the volumes V_i of the returned weights
    evaluated by the FP64 oracle (brute-force neighbours)."""
    import oracle
    c = oracle.cells(x, y, z, psi, idx=idx)
    return np.abs(c.V - nu[idx]) / nu[idx]


def summarize(e, what):
    return {"count": int(len(e)), "max_rel_err": float(np.max(e)), "p99_rel_err": float(np.percentile(e, 99)),
            "sample": what}


def oracle_error(x, y, z, psi, nu, idx, what="heaviest sites + random cells"):
    return summarize(cell_errors(x, y, z, psi, nu, idx), what)


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
    # every solve follows the path on the prescribed volumes (opts.continuation), with loose
    # intermediate stages (stage_tol 0.1: 38 evaluations per step against 41 at 1e-2) and the
    # step search of each iteration started at twice the last accepted step (step_start 1: 33
    # evaluations per step against 36, the same Newton iterations), each stage's first search at
    # the stage before's first accepted step (step_start 2: 31 against 34 evaluations over 8
    # steps, 2,242 against 2,445 ms per step), and each intermediate stage also ends when ||nu(s) - V||
    # has fallen to 10% of its start value (stage_gtol: 25 against 31 evaluations over 8 steps, 1,814
    # against 2,234 ms per step, with stalled final iterations sent to the float64 path); the first
    # step in s stays at
    # 1/4 (1/3 saves evaluations on most steps but over 20 steps averages the same): at this size
    # the advected previous weights leave ~20% of the cells empty, the repair does not
    # recover them, and the solve restarts from the default weights, from which the path
    # takes fewer evaluations than Algorithm 1 alone (41 against 57 per step)
    settle_opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1, cg_rtol=CG_RTOL, stage_tol=0.1,
                                 step_start=2, stage_gtol=0.1)
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

    def step(k):
        x, y, z = pos[k]
        s1 = ctx.solve(x, y, z, nu, psi, opts=settle_opts, check=False)
        kt = ctx.last_kernel_times()
        if s1.status != 0:
            raise RuntimeError(f"step {k} of the splash sequence failed: {s1.as_dict()}")
        return s1, kt

    for k in range(max(warmup, 1) - 1):
        step(k)
    k0 = max(warmup, 1) - 1
    out = {"ms": [], "newton_iters": [], "evals": [], "halvings": [], "cg_iters": [], "restarted": [],
           "repaired": [], "stages": [], "ms_eval": [], "ms_linear": [], "kernel_times": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(k0, k0 + steps):
        a = time.perf_counter()
        s1, kt = step(k)  # returns after the stream is synchronised
        out["ms"].append(1000.0 * (time.perf_counter() - a))
        out["newton_iters"].append(s1.newton_iters)
        out["evals"].append(s1.evals)
        out["halvings"].append(s1.halvings)
        out["cg_iters"].append(s1.cg_iters)
        out["restarted"].append(s1.default_start)
        out["repaired"].append(s1.repaired_start)
        out["stages"].append(s1.stages)
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
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, cg_rtol=CG_RTOL))
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


def counters_summary(fetch_dir: str, write_dir: str, sq_dir: str, kernel: str = "k_cells_overflow") -> int:
    """Writes the counter record of one kernel (TRAFFIC_FILE and a markdown table beside it)
    from three rocprofv3 --pmc runs of ``--profile c3`` (FETCH_SIZE; WRITE_SIZE;
    SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE). Byte counters are scaled by what they read for
    the 256 MiB device copy at the end of the run; GRBM_GUI_ACTIVE sums the eight XCDs, and
    a CU issues at most one wave64 VALU instruction per cycle."""
    import csv
    import re
    from collections import defaultdict

    def load(d):
        out = defaultdict(lambda: defaultdict(list))
        with open(os.path.join(d, "pmc_counter_collection.csv")) as f:
            for row in csv.DictReader(f):
                m = re.search(r"(k_\w+|copyBuffer\w*)", row["Kernel_Name"])
                if m:
                    out[m.group(1)][row["Counter_Name"]].append(float(row["Counter_Value"]))
        return out

    F, W, S = load(fetch_dir), load(write_dir), load(sq_dir)
    cp = next(k for k in F if k.startswith("copyBuffer"))
    copy_kib = 256 * 1024
    ff = copy_kib / max(F[cp]["FETCH_SIZE"])
    wf = copy_kib / max(W[cp]["WRITE_SIZE"])
    mean = lambda v: sum(v) / len(v)
    fk, wk = mean(F[kernel]["FETCH_SIZE"]), mean(W[kernel]["WRITE_SIZE"])
    valu, waves, gui = (mean(S[kernel][c]) for c in ("SQ_INSTS_VALU", "SQ_WAVES", "GRBM_GUI_ACTIVE"))
    cycles = gui / 8.0
    rec = {"kernel": kernel, "workload": "splash_2000000: settle and two advect-and-solve steps (--profile c3)",
           "dispatches": len(F[kernel]["FETCH_SIZE"]), "fetch_kib_per_dispatch": fk,
           "write_kib_per_dispatch": wk, "fetch_factor": ff, "write_factor": wf,
           "bytes_per_launch": 1024.0 * (fk * ff + wk * wf), "valu_insts_per_dispatch": valu,
           "waves_per_dispatch": waves, "cycles_per_dispatch": cycles,
           "valu_issue_frac": valu / (256.0 * cycles), "sources_sha256": kernel_sources_digest(),
           "source": os.path.relpath(TRAFFIC_FILE.replace(".json", ".md"), ROOT)}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))
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
    opts = L.default_opts(tol=1e-5, autotune=1, cg_rtol=CG_RTOL)
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
    sec = {"workload": f"dam_break_{n}: jittered cubic lattice in the lower 40% of the unit box, nu=0.35/N, one "
                       f"plain OT solve from the start weights to 1e-5",
           "cells_per_s": n * sum(s.evals for s in stats) / wall, "ms_per_solve": 1000.0 * wall / steps,
           "newton_iters": s0.newton_iters, "evals": s0.evals, "halvings": s0.halvings, "cg_iters": s0.cg_iters,
           "max_rel_err": s0.max_rel_err, "ms_eval": s0.ms_eval, "ms_linear": s0.ms_linear,
           "ms_cell_kernel": ms_kernel,
           "eval_only": {"cells_per_s_with_grid": n / (ev0 / 1000.0), "cells_per_s_kernel": n / (k0 / 1000.0),
                         "ms_lagot_cells": ev0, "ms_cell_kernel": k0,
                         "converged": {"cells_per_s_with_grid": n / (ev1 / 1000.0),
                                       "cells_per_s_kernel": n / (k1 / 1000.0), "ms_lagot_cells": ev1,
                                       "ms_cell_kernel": k1},
                         "centroids_converged": {"ms_lagot_centroids": evc, "ms_cell_kernel": kc,
                                                 "cells_per_s_kernel": n / (kc / 1000.0)}}}
    check = lambda: oracle_error(sc.x, sc.y, sc.z, p_last, sc.nu, sample_idx(n, p_last, 5, k_top=0, k_rand=300),
                                 "300 random cells of the last solve")
    return sec, (sc, x, y, z, nu, psis[-1]), check


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed advect-and-solve steps of the 2M-site sequence")
    ap.add_argument("--warmup", type=int, default=2, help="the settle, then warmup - 1 untimed steps")
    ap.add_argument("--n", type=int, default=2_000_000)
    ap.add_argument("--profile", choices=["c3", "cells", "fluid"], default=None)
    ap.add_argument("--counters-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "SQ_DIR"), default=None,
                    help="write the crowded pass's counter record from three rocprofv3 --pmc runs of --profile c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--eval-reps", type=int, default=20)
    ap.add_argument("--no-dam-break", action="store_true", help="skip the 100k dam-break section")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched solve")
    ap.add_argument("--no-domain", action="store_true", help="skip the non-convex (L-shaped) domain section")
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

    if args.counters_summary:
        return counters_summary(*args.counters_summary)

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
    kt = st3["kernel_times"]
    fast_ms = sum(k["fast_ms"] for k in kt) / max(sum(k["fast_launches"] for k in kt), 1)
    crowd_launches = sum(k["crowd_launches"] for k in kt)
    crowd_ms = sum(k["crowd_ms"] for k in kt) / max(crowd_launches, 1)
    crowd_cells = sum(k["crowd_cells"] for k in kt) / max(crowd_launches, 1)
    # the cells the crowded pass finishes at the final state (for the roofline's work units)
    xf, yf, zf = (torch.tensor(np.ascontiguousarray(a), device="cuda") for a in (fin.x, fin.y, fin.z))
    ctx.cells(xf, yf, zf, r["psi"], csr=False, walls=False)
    deferred = ctx.last_deferred()
    rec = counter_record()
    traffic = rec.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": None, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": traffic,
                "kernel": "k_cells_overflow (crowded cells: box-overlap candidates, clip rounds, integration; "
                          "float64)",
                "cells_per_launch": crowd_cells, "ms_per_launch": crowd_ms, "launches": crowd_launches,
                "valu_issue_frac": rec.get("valu_issue_frac"),
                "traffic_bytes_per_cell": None if traffic is None else traffic / max(crowd_cells, 1.0),
                "counters": rec.get("source"),
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
                               f"Voronoi start, then advect (dt 2e-3) and solve to 1e-5 per step from the previous "
                               f"weights (repaired, else the default start) with path following on the volumes",
                   "n_sites": n, "tol": 1e-5, "dt": 2e-3},
        "c3": {"settle": r["settle"], "ms_per_step": ms_per_step, "ms_steps": st3["ms"],
               "newton_iters": st3["newton_iters"], "evals": st3["evals"], "halvings": st3["halvings"],
               "cg_iters": st3["cg_iters"], "restarted": st3["restarted"], "repaired": st3["repaired"],
               "stages": st3["stages"],
               "ms_eval": st3["ms_eval"], "ms_linear": st3["ms_linear"],
               "ms_fast_kernel_per_eval": fast_ms, "ms_crowded_pass_per_eval": crowd_ms,
               "crowded_cells_per_eval": crowd_cells},
        "roofline": roofline,
    }
    # every oracle call of the run is in the leg at the end: the error of each section's result
    # against the FP64 oracle, the roofline's work units, and the oracle's own rate (cpu_baseline)
    checks = {"c3": lambda: oracle_error(fin.x, fin.y, fin.z, p_fin, r["nu"], sample_idx(n, p_fin, 3),
                                         "100 heaviest sites + 300 random cells of the last step")}
    if not args.no_dam_break:
        sec, dam, checks["dam_break"] = dam_break_section(ctx, L, scenes, 100_000, 10, 3, args.eval_reps)
        line["dam_break"] = sec
        _, x, y, z, nu, psi = dam
        line["paper_k_route"], checks["paper_k_route"] = paper_k_section(ctx, x, y, z, psi)
        if not args.no_fluid:
            line["fluid"], checks["fluid"] = fluid_section(ctx, L, x, y, z, psi, nu)
    if not args.no_batched:
        line["batched"], checks["batched"] = batched_section(ctx, L, scenes)
    if not args.no_domain:
        line["domain_pieces"], checks["domain_pieces"] = domain_section(ctx, L, scenes)
    if not args.no_learned:
        line["learned"], checks["learned"] = learned_section(ctx, L, scenes, args.learned_seeds,
                                                             args.learned_steps, args.sequence_steps)
    if not args.no_cpu_baseline:
        for key, fn in checks.items():
            line[key]["oracle_error"] = fn()
            log(f"oracle error of {key}: {line[key]['oracle_error']}")
        import oracle
        if len(deferred) and crowd_ms > 0:
            rs = np.random.default_rng(11)
            samp = np.sort(rs.choice(deferred, min(300, len(deferred)), replace=False))
            w = oracle.cells(fin.x, fin.y, fin.z, p_fin, idx=samp, work=True).work.mean(axis=0)
            fpc = flops_per_cell_minimal_clip(w)
            achieved = fpc * crowd_cells / (crowd_ms / 1000.0) / 1e12
            roofline.update({"achieved": achieved, "frac": achieved / PEAK_FP64_TFLOPS, "flops_per_cell": fpc,
                             "work_units_per_cell": dict(zip(["cand", "tests", "newv", "faces", "edges", "cross"],
                                                             [float(v) for v in w]))})
        cb, work = cpu_baseline(fin, p_fin, args.cpu_seconds)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
