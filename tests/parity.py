"""Comparison of GPU cell outputs with the FP64 oracle, element by element.

Tolerances (float32 geometry against the float64 oracle), normalised so that
tiny, cancellation-dominated quantities are compared on the scale of the ball:
  |dV_i| <= tol * max(V_i, 1e-3 * 4/3 pi r_i^3)
  |dK_i| <= tol * 4 pi r_i^2
  |dA_ij|, |dW_iw| <= tol * pi r_i^2
Connectivity must be identical away from ties; a facet is a tie when its oracle
area is below 1e-6 pi r_i^2 (zero-area contact, e.g. exact lattice corners).
"""
from __future__ import annotations

import math

import numpy as np

TOL = 1e-5


def gpu_facets(out, n):
    rp = out["row_ptr"].cpu().numpy()
    col = out["col"].cpu().numpy()
    area = out["area"].cpu().numpy()
    return rp, col, area


def compare(out, orc, psi, idx=None, tol=TOL, tie=1e-6):
    """Returns a dict of max normalised errors and mismatch counts; idx = evaluated sites."""
    n = out["vol"].shape[0]
    idx = np.arange(n) if idx is None else np.asarray(idx)
    V = out["vol"].cpu().numpy()[idx]
    K = out["sph"].cpu().numpy()[idx]
    W = out["walls"].cpu().numpy()[idx]
    rp, col, area = gpu_facets(out, n)
    r = np.sqrt(np.maximum(psi[idx], 0))
    ball = 4.0 / 3.0 * math.pi * r ** 3
    eV = np.abs(V - orc.V) / np.maximum(np.maximum(orc.V, 1e-3 * ball), 1e-300)
    eK = np.abs(K - orc.K) / np.maximum(4 * math.pi * r * r, 1e-300)
    eW = np.abs(W - orc.walls).max(axis=1) / np.maximum(math.pi * r * r, 1e-300)
    eA = np.zeros(len(idx))
    conn_bad = 0
    for c, i in enumerate(idx):
        disk = math.pi * r[c] * r[c]
        g = dict(zip(col[rp[i]:rp[i + 1]].tolist(), area[rp[i]:rp[i + 1]].tolist()))
        o = orc.facets(c)
        for j in set(g) | set(o):
            a_g, a_o = g.get(j, 0.0), o.get(j, 0.0)
            eA[c] = max(eA[c], abs(a_g - a_o) / disk)
            if (j in g) != (j in o) and a_o >= tie * disk:
                conn_bad += 1
    return {"V": float(eV.max(initial=0)), "K": float(eK.max(initial=0)), "W": float(eW.max(initial=0)),
            "A": float(eA.max(initial=0)), "conn": conn_bad, "worst_V": int(idx[int(np.argmax(eV))]) if len(idx) else -1}


def assert_close(rep, tol=TOL):
    assert rep["conn"] == 0, rep
    assert rep["V"] <= tol, rep
    assert rep["K"] <= tol, rep
    assert rep["A"] <= tol, rep
    assert rep["W"] <= tol, rep


def newton_direction_bound(oracle_mod, P, psi, c, Hd, g, u, cg_rtol, tol=TOL):
    """Bound on ||u_gpu - u||_2 for a Newton direction u of (-Hess K) u = g (eq. (2)) that the
    GPU solves with float32 facet areas and a PCG stopped at ||r|| <= cg_rtol ||g||:
      ||e||_2 <= (cg_rtol ||g||_2 + ||dH||_2 ||u||_2) / lambda_min(-Hess K),
    first order in dH, where ||dH||_2 <= max row sum of |dH| (symmetric) and the entries of
    dH are bounded by the cell tolerances (|dA_ij| <= tol pi r_i^2 on both sides' areas of
    w_ij = Abar_ij / 2d_ij, |dK_i| <= tol 4 pi r_i^2 in K_i / 2r_i)."""
    r = np.sqrt(np.maximum(psi, 0.0))
    W = oracle_mod.p1_weights(P, c).tocoo()
    d = np.linalg.norm(P[W.row] - P[W.col], axis=1)
    rowb = np.zeros(len(psi))
    np.add.at(rowb, W.row, tol * math.pi * np.maximum(r[W.row], r[W.col]) ** 2 / (2.0 * d))
    dH = float((2.0 * rowb + tol * 4.0 * math.pi * r * r / (2.0 * np.maximum(r, 1e-300))).max())
    lam_min = float(np.linalg.eigvalsh(Hd)[0])
    return (cg_rtol * float(np.linalg.norm(g)) + dH * float(np.linalg.norm(u))) / lam_min
