"""Learned warm start: training pairs from the solver's own solves, training on
the GPU through the C-ABI (lagot_features, lagot_mlp_train_step), and the
comparison against the previous-step warm start.

A training pair is (inputs of a state, target): the state is a dam-break scene one
advection step (dt, velocities N(0, sigma^2) per axis) after a converged solve psi_a,
taken along an advect-and-solve sequence (so that later, more disordered states are
in the training distribution too); the target is (psi_b - psi_a) / s_i^2 where psi_b
is the converged weight vector at the advected positions and s_i = nu_i^(1/3). The network's guess is only
ever a start for Newton: lagot_solve accepts it when every cell keeps positive
volume and the residual norm drops, and runs to the tolerance either way.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import scenes


def _t(a, dt, dev="cuda"):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal hidden layers, small output layer (float32, flat layout of lagot.h)."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in [(64, 128), (128, 128), (128, 128), (128, 1)]:
        W = rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b))
        if b == 1:
            W *= 0.1
        out += [W.ravel(), np.zeros(b)]
    return np.concatenate(out).astype(np.float32)


def generate_pairs(ctx, seeds, n: int = 100_000, dt: float = 2e-3, sigma: float = 0.5, tol: float = 1e-5,
                   steps: int = 1, log=print):
    """For each seed: solve cold, then `steps` times advect and solve warm from the previous
    weights; every warm solve gives one pair per site. Returns device (inputs int16 [M,64],
    targets float32 [M])."""
    import torch
    import paper_2601_05765_amd as L
    feats, targets = [], []
    opts = L.default_opts(tol=tol)
    for seed in seeds:
        sc = scenes.with_velocity(scenes.dam_break(n, seed), seed=10_000 + seed, sigma=sigma)
        nu = _t(sc.nu, torch.float64)
        s2 = np.cbrt(sc.nu) ** 2
        psi = _t(sc.psi0, torch.float64)
        ctx.solve(_t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32), nu, psi, opts=opts)
        cur = sc
        for k in range(steps):
            cur = scenes.advect(cur, dt)
            x1, y1, z1 = _t(cur.x, torch.float32), _t(cur.y, torch.float32), _t(cur.z, torch.float32)
            psi_a = psi.clone()
            st = ctx.solve(x1, y1, z1, nu, psi, opts=opts, check=False)
            if st.status != 0:
                break
            _, f = ctx.features(x1, y1, z1, psi_a, nu, want_nbr=False)
            tgt = (psi.cpu().numpy() - psi_a.cpu().numpy()) / s2
            feats.append(f)
            targets.append(_t(tgt, torch.float32))
            log(f"pairs seed {seed} step {k + 1}: warm solve {st.newton_iters} iterations, "
                f"target rms {np.sqrt(np.mean(tgt ** 2)):.3e}")
    return torch.cat(feats), torch.cat(targets)


def train(ctx, feats, targets, epochs: int = 6, batch: int = 4096, lr: float = 1e-3, seed: int = 0, log=print):
    """Adam on the mean squared error, cosine-decayed learning rate; returns the loss history."""
    import torch
    m = feats.shape[0]
    rng = np.random.default_rng(seed)
    ctx.mlp_set_params(_t(init_params(seed), torch.float32))
    steps = epochs * (m // batch)
    hist = []
    k = 0
    for ep in range(epochs):
        perm = _t(rng.permutation(m).astype(np.int32), torch.int32)
        for b in range(m // batch):
            frac = k / max(steps - 1, 1)
            cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * frac)))
            want = (b % 50 == 0)
            loss = ctx.mlp_train_step(feats, targets, perm[b * batch:(b + 1) * batch], cur, want_loss=want)
            if want:
                hist.append(loss)
            k += 1
        log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


def sequence(ctx, sc, steps: int, dt: float = 2e-3, use_learned: bool = False, tol: float = 1e-5, psi_start=None,
             log=print, cg_rtol: float = 1e-6, state: dict | None = None):
    """Advect-and-solve sequence from converged weights; per-step solve statistics (a failed
    solve is recorded and the sequence goes on from its last accepted weights). ``state``
    receives the last scene and weights."""
    import torch
    import paper_2601_05765_amd as L
    nu = _t(sc.nu, torch.float64)
    psi = psi_start.clone()
    cur = sc
    out = []
    for k in range(steps):
        cur = scenes.advect(cur, dt)
        x, y, z = _t(cur.x, torch.float32), _t(cur.y, torch.float32), _t(cur.z, torch.float32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=tol, use_learned=int(use_learned), cg_rtol=cg_rtol),
                       check=False)
        torch.cuda.synchronize()
        ms = 1000 * (time.perf_counter() - t0)
        out.append({"step": k + 1, "ms": ms, "status": st.status, "newton_iters": st.newton_iters,
                    "evals": st.evals, "cg_iters": st.cg_iters, "learned_accepted": st.learned_accepted,
                    "max_rel_err": st.max_rel_err, "ms_learned": st.ms_learned})
        log(f"step {k + 1}: {'learned' if use_learned else 'plain'} {ms:.1f} ms, {st.newton_iters} it, "
            f"accepted={st.learned_accepted}")
    if state is not None:
        state["scene"] = cur
        state["psi"] = psi
    return out
