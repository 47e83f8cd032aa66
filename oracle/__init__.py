"""FP64 CPU oracle for the analytic partial-optimal-transport solver.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the HIP path.

Contents
  cells(...)          restricted cell volumes, spherical areas, facet areas, centroids
                      (C routine in lagot_oracle.c; eq. (1), section 3.2, 3.3, Alg. 2;
                      centroids: the cell centroid of the pressure model, section 5)
  hessian(...)        gradient nu - V and the sparse matrix -Hess K (eq. (2))
  newton_solve(...)   damped Newton with KMT step control (Alg. 1)
Parity pins for every function live in tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lagot_oracle.c")
_LIB = os.path.join(_HERE, "liblagot_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc, -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_cells.argtypes = [ctypes.c_long, P, P, P, P, P, P, ctypes.c_long, P, P, P, P, P, ctypes.c_int,
                                     P, P, P, ctypes.c_int, P, P, P, ctypes.c_int]
        lib.oracle_cells.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Cells:
    V: np.ndarray            # [m] volumes
    K: np.ndarray            # [m] spherical (free-surface) areas
    walls: np.ndarray        # [m,6] wall facet areas (-x,+x,-y,+y,-z,+z), or [m,P] per domain plane
    fcount: np.ndarray       # [m] neighbour facet counts
    fj: np.ndarray           # [m,fcap] neighbour ids (valid up to fcount)
    fA: np.ndarray           # [m,fcap] facet areas
    ncand: np.ndarray        # [m] bisector planes that cut the ball
    status: np.ndarray       # [m] 0 ok, 1 empty, 2 facet capacity exceeded
    idx: np.ndarray          # [m] evaluated site indices
    work: np.ndarray | None = None  # [m,6] work units (see lagot_oracle.c) when requested
    C: np.ndarray | None = None     # [m,3] centroids (the site itself for an empty cell)

    def facets(self, c: int) -> dict:
        k = int(self.fcount[c])
        return {int(j): float(a) for j, a in zip(self.fj[c, :k], self.fA[c, :k])}


def cells(x, y, z, psi, box=((0, 0, 0), (1, 1, 1)), idx=None, fcap: int = 96, threads: int = 0,
          work: bool = False, domain=None) -> Cells:
    """Evaluate the restricted Laguerre cells of the sites ``idx`` (default: all).

    ``domain``: optional [P, 4] array of planes (n, c), unit outward normals n, for the
    convex domain {x : n.x <= c} in place of the box walls.

    Positions are promoted to float64 exactly; ``psi`` must be float64.
    Neighbours are found by brute force over all sites (O(N) per cell)."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    z = np.ascontiguousarray(z, np.float64)
    psi = np.ascontiguousarray(psi, np.float64)
    n = x.shape[0]
    b = np.ascontiguousarray(np.concatenate([np.asarray(box[0], np.float64), np.asarray(box[1], np.float64)]))
    if idx is None:
        idx_arr = np.arange(n, dtype=np.int64)
        m = n
        idx_p = None
    else:
        idx_arr = np.ascontiguousarray(idx, np.int64)
        m = idx_arr.shape[0]
        idx_p = _ptr(idx_arr)
    V = np.zeros(m)
    K = np.zeros(m)
    dom = None if domain is None else np.ascontiguousarray(domain, np.float64).reshape(-1, 4)
    nwall = 6 if dom is None else dom.shape[0]
    W = np.zeros((m, nwall))
    fj = np.full((m, fcap), -1, np.int64)
    fA = np.zeros((m, fcap))
    fc = np.zeros(m, np.int32)
    nc = np.zeros(m, np.int32)
    st = np.zeros(m, np.int32)
    wk = np.zeros((m, 6), np.int64) if work else None
    C = np.zeros((m, 3))
    lib.oracle_cells(n, _ptr(x), _ptr(y), _ptr(z), _ptr(psi), _ptr(b), idx_p, m, _ptr(V), _ptr(K), _ptr(W),
                     _ptr(fj), _ptr(fA), fcap, _ptr(fc), _ptr(nc), _ptr(st), int(threads),
                     _ptr(wk) if work else None, _ptr(C), _ptr(dom) if dom is not None else None,
                     0 if dom is None else int(dom.shape[0]))
    if (st == 2).any():
        raise RuntimeError("oracle facet capacity exceeded; raise fcap")
    return Cells(V, K, W, fc, fj, fA, nc, st, idx_arr, wk, C)


def hessian(xyz: np.ndarray, psi: np.ndarray, c: Cells):
    """Assemble -Hess K (eq. (2)) as a scipy CSR matrix, from a full evaluation ``c``.

    Off-diagonal (i,j): -w_ij with w_ij = Abar_ij / (2 |p_j - p_i|), Abar the mean of
    the two sides' facet areas (union pattern: a one-sided facet keeps its value).
    Diagonal: sum_j w_ij + K_i / (2 sqrt(psi_i)); box walls do not move with psi and
    do not enter. Empty cells give an empty row and column."""
    import scipy.sparse as sp
    n = xyz.shape[0]
    assert c.idx.shape[0] == n and (c.idx == np.arange(n)).all(), "hessian needs all cells"
    rows, cols, vals = [], [], []
    for i in range(n):
        k = int(c.fcount[i])
        rows.append(np.full(k, i))
        cols.append(c.fj[i, :k])
        vals.append(c.fA[i, :k])
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = np.concatenate(vals) if vals else np.zeros(0)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    At = A.T.tocsr()
    S = (A + At).tocsr()
    both = ((A != 0).astype(np.int8) + (At != 0).astype(np.int8)).tocsr()
    S = S.tocoo()
    both = both.tocoo()
    # union pattern: average where both sides have the facet, keep the single side otherwise
    cnt = dict(zip(zip(both.row.tolist(), both.col.tolist()), both.data.tolist()))
    Abar = np.array([v / cnt[(i, j)] for i, j, v in zip(S.row.tolist(), S.col.tolist(), S.data.tolist())])
    d = np.linalg.norm(xyz[S.row] - xyz[S.col], axis=1)
    w = Abar / (2.0 * d)
    W = sp.coo_matrix((w, (S.row, S.col)), shape=(n, n)).tocsr()
    r = np.sqrt(np.maximum(psi, 0.0))
    kterm = np.where(r > 0, c.K / (2.0 * np.where(r > 0, r, 1.0)), 0.0)
    diag = np.asarray(W.sum(axis=1)).ravel() + kterm
    H = (sp.diags(diag) - W).tocsr()
    return H, diag


@dataclass
class NewtonStats:
    status: str
    iters: int
    evals: int
    halvings: int
    max_rel_err: float
    history: list


def _residuals(V, nu):
    g = nu - V
    return g, float(np.max(np.abs(g) / nu)), float(np.linalg.norm(g))


def newton_solve(xyz: np.ndarray, nu: np.ndarray, psi0: np.ndarray, box=((0, 0, 0), (1, 1, 1)),
                 tol: float = 1e-5, max_newton: int = 100, max_halvings: int = 30, dense_max: int = 3000,
                 cg_rtol: float = 1e-12, threads: int = 0):
    """Damped Newton for the weights (Alg. 1) with KMT step control, FP64.

    Stop when max_i |V_i - nu_i| / nu_i <= tol. Direction: solve (-Hess K) u = nu - V
    (dense Cholesky up to ``dense_max`` sites, else Jacobi-PCG to ``cg_rtol``).
    Step: alpha = 1, halved until min V(psi + alpha u) >= eps0 and
    ||g(psi + alpha u)|| <= (1 - alpha/2) ||g(psi)||, with
    eps0 = 1/2 min(min nu, min V(psi0)) (KMT)."""
    import scipy.linalg as sla
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    psi = np.array(psi0, np.float64, copy=True)
    c = cells(x, y, z, psi, box, threads=threads)
    evals = 1
    V = c.V
    eps0 = 0.5 * min(float(nu.min()), float(V.min()))
    if not eps0 > 0:
        return psi, NewtonStats("empty", 0, evals, 0, float("inf"), [])
    g, err, gn = _residuals(V, nu)
    hist = [dict(it=0, max_rel_err=err, gnorm=gn, alpha=None)]
    halv_total = 0
    for it in range(1, max_newton + 1):
        if err <= tol:
            return psi, NewtonStats("ok", it - 1, evals, halv_total, err, hist)
        H, diag = hessian(xyz, psi, c)
        if xyz.shape[0] <= dense_max:
            u = sla.cho_solve(sla.cho_factor(H.toarray()), g)
        else:
            u = pcg(H, g, diag, rtol=cg_rtol)
        alpha = 1.0
        for h in range(max_halvings + 1):
            trial = psi + alpha * u
            ct = cells(x, y, z, trial, box, threads=threads)
            evals += 1
            gt, errt, gnt = _residuals(ct.V, nu)
            if ct.V.min() >= eps0 and gnt <= (1.0 - 0.5 * alpha) * gn:
                break
            alpha *= 0.5
            halv_total += 1
        else:
            return psi, NewtonStats("linesearch", it, evals, halv_total, err, hist)
        psi, c, g, err, gn = trial, ct, gt, errt, gnt
        hist.append(dict(it=it, max_rel_err=err, gnorm=gn, alpha=alpha))
    status = "ok" if err <= tol else "noconv"
    return psi, NewtonStats(status, max_newton, evals, halv_total, err, hist)


def pcg(H, b, diag, rtol=1e-12, maxit=100000):
    """Jacobi-preconditioned conjugate gradients in FP64 (plain textbook form)."""
    Minv = np.where(diag > 0, 1.0 / np.where(diag > 0, diag, 1.0), 1.0)
    x = np.zeros_like(b)
    r = b.copy()
    zv = Minv * r
    p = zv.copy()
    rz = float(r @ zv)
    bn = float(np.linalg.norm(b))
    if bn == 0:
        return x
    for _ in range(maxit):
        q = H @ p
        a = rz / float(p @ q)
        x += a * p
        r -= a * q
        if np.linalg.norm(r) <= rtol * bn:
            break
        zv = Minv * r
        rz_new = float(r @ zv)
        p = zv + (rz_new / rz) * p
        rz = rz_new
    return x


def ball_volume(r):
    return 4.0 / 3.0 * math.pi * r ** 3
