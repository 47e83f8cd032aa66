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
