"""FP64 CPU oracle for the analytic partial-optimal-transport solver.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no code
with the HIP path.

Contents
  cells(...)          restricted cell volumes, spherical areas, facet areas, centroids
                      (C routine in lagot_oracle.c; eq. (1), section 3.2, 3.3, Alg. 2;
                      centroids: the cell centroid of the pressure model, section 5)
  cells_pieces(...)   the same in a non-convex domain given as a union of convex pieces
                      (section 6: cells in polyhedral domains; sums of the per-piece parts)
  hessian(...)        gradient nu - V and the sparse matrix -Hess K (eq. (2))
  newton_solve(...)   damped Newton with KMT step control (Alg. 1)
  p1_weights(...)     facet weights w_ij = |V_ij| / (2 |p_j - p_i|) of the P1 Laplacian (eq. (3))
  p1_rows(...)        the same weights for a few rows only (sampled checks at full size)
  p1_laplacian(...)   the P1 (cotan) Laplacian of a per-site field, optional mu_ij (eq. (3))
  fluid_velocity(...) the semi-implicit velocity update with pressure spring, gravity,
                      surface tension and viscosity (section 5, eq. (4))
  advect(...)         the position update x + dt v of the fluid step, kept inside the domain
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
                                     P, P, P, ctypes.c_int, P, P, P, ctypes.c_int, P, P]
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
    Kp: np.ndarray | None = None    # [m] |K| by section 3.3's own route (paper_k=True)
    cin: np.ndarray | None = None   # [m,3] that route's interior point c (paper_k=True)

    def facets(self, c: int) -> dict:
        k = int(self.fcount[c])
        return {int(j): float(a) for j, a in zip(self.fj[c, :k], self.fA[c, :k])}


def cells(x, y, z, psi, box=((0, 0, 0), (1, 1, 1)), idx=None, fcap: int = 96, threads: int = 0,
          work: bool = False, domain=None, paper_k: bool = False) -> Cells:
    """Evaluate the restricted Laguerre cells of the sites ``idx`` (default: all).

    ``paper_k``: also compute |K| by section 3.3's own route (interior point c from
    rays cast from the restricted facets, each facet projected from c onto the sphere,
    the projected areas by Gauss-Bonnet; Algorithm 2), independently of the signed
    solid-angle form that gives ``K``.

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
    Kp = np.zeros(m) if paper_k else None
    cin = np.zeros((m, 3)) if paper_k else None
    lib.oracle_cells(n, _ptr(x), _ptr(y), _ptr(z), _ptr(psi), _ptr(b), idx_p, m, _ptr(V), _ptr(K), _ptr(W),
                     _ptr(fj), _ptr(fA), fcap, _ptr(fc), _ptr(nc), _ptr(st), int(threads),
                     _ptr(wk) if work else None, _ptr(C), _ptr(dom) if dom is not None else None,
                     0 if dom is None else int(dom.shape[0]), _ptr(Kp) if paper_k else None,
                     _ptr(cin) if paper_k else None)
    if (st == 2).any():
        raise RuntimeError("oracle facet capacity exceeded; raise fcap")
    return Cells(V, K, W, fc, fj, fA, nc, st, idx_arr, wk, C, Kp, cin)


def cells_pieces(x, y, z, psi, pieces, nwalls: int, box=((0, 0, 0), (1, 1, 1)), idx=None, fcap: int = 96,
                 threads: int = 0, paper_k: bool = False) -> Cells:
    """Restricted cells in a non-convex domain, the union of convex pieces with disjoint
    interiors (section 6 evaluates cells in polyhedral domains). ``pieces`` is a list of
    (planes [P_k, 4] (unit outward normal n, c: piece {x : n.x <= c}), wall_id [P_k]) with
    wall_id the wall a plane belongs to, or -1 for a plane between two pieces.

    The restricted cell L_i ∩ B_i ∩ Ω is the disjoint union of L_i ∩ B_i ∩ Ω_k over the
    pieces Ω_k, so every measure of it is the sum of the pieces' measures: volume,
    spherical area, the area of each facet (by neighbour), the area on each wall (by wall
    id; a plane between pieces bounds no wall), and the first moment (the centroid is
    their sum over the total volume; an empty cell keeps the site). With ``paper_k`` the
    second route's |K| (section 3.3) is summed over the pieces too (``Kp``)."""
    parts = [cells(x, y, z, psi, box=box, idx=idx, fcap=fcap, threads=threads, domain=np.asarray(pl, np.float64),
                   paper_k=paper_k) for pl, _ in pieces]
    m = parts[0].V.shape[0]
    V = np.zeros(m)
    K = np.zeros(m)
    W = np.zeros((m, nwalls))
    mom = np.zeros((m, 3))
    fac = [dict() for _ in range(m)]
    nc = np.zeros(m, np.int32)
    for (pl, wid), c in zip(pieces, parts):
        V += c.V
        K += c.K
        mom += c.V[:, None] * c.C
        nc = np.maximum(nc, c.ncand)
        for w, wi in enumerate(np.asarray(wid).reshape(-1)):
            if wi >= 0:
                W[:, wi] += c.walls[:, w]
        for i in range(m):
            for j, a in c.facets(i).items():
                fac[i][j] = fac[i].get(j, 0.0) + a
    fc = np.array([len(f) for f in fac], np.int32)
    if (fc > fcap).any():
        raise RuntimeError("oracle facet capacity exceeded; raise fcap")
    fj = np.full((m, fcap), -1, np.int64)
    fA = np.zeros((m, fcap))
    for i, f in enumerate(fac):
        for s, j in enumerate(sorted(f)):
            fj[i, s] = j
            fA[i, s] = f[j]
    site = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64), np.asarray(z, np.float64)], 1)
    site = site[parts[0].idx]
    C = np.where(V[:, None] > 0, mom / np.where(V > 0, V, 1.0)[:, None], site)
    st = np.where(V > 0, 0, 1).astype(np.int32)
    Kp = sum(c.Kp for c in parts) if paper_k else None
    return Cells(V, K, W, fc, fj, fA, nc, st, parts[0].idx, None, C, Kp)


def hessian(xyz: np.ndarray, psi: np.ndarray, c: Cells):
    """Assemble -Hess K (eq. (2)) as a scipy CSR matrix, from a full evaluation ``c``.

    Off-diagonal (i,j): -w_ij with w_ij = Abar_ij / (2 |p_j - p_i|), Abar the mean of
    the two sides' facet areas (union pattern: a one-sided facet keeps its value).
    Diagonal: sum_j w_ij + K_i / (2 sqrt(psi_i)); box walls do not move with psi and
    do not enter. Empty cells give an empty row and column."""
    W = p1_weights(xyz, c)
    r = np.sqrt(np.maximum(psi, 0.0))
    kterm = np.where(r > 0, c.K / (2.0 * np.where(r > 0, r, 1.0)), 0.0)
    diag = np.asarray(W.sum(axis=1)).ravel() + kterm
    import scipy.sparse as sp
    H = (sp.diags(diag) - W).tocsr()
    return H, diag


def p1_weights(xyz: np.ndarray, c: Cells):
    """Symmetric sparse matrix of the facet weights w_ij = Abar_ij / (2 |p_j - p_i|)
    over the restricted Laguerre facets, from a full evaluation ``c``.

    These are the off-diagonal weights of -Hess K (eq. (2)) and the weights of the P1
    Laplacian of the fluid model (eq. (3)). Abar is the mean of the facet area seen
    from the two cells; a facet that only one side lists keeps that side's value."""
    import scipy.sparse as sp
    n = xyz.shape[0]
    assert c.idx.shape[0] == n and (c.idx == np.arange(n)).all(), "weights need all cells"
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
    return sp.coo_matrix((w, (S.row, S.col)), shape=(n, n)).tocsr()


def p1_rows(xyz: np.ndarray, psi: np.ndarray, rows, box=((0, 0, 0), (1, 1, 1)), domain=None) -> dict:
    """The rows ``rows`` of the facet-weight matrix of p1_weights, without evaluating every
    cell: the cells of those rows and of all their neighbours are evaluated (brute force),
    and each weight uses both sides' areas as p1_weights does. Returns {i: {j: w_ij}}."""
    xyz = np.asarray(xyz, np.float64)
    psi = np.asarray(psi, np.float64)
    rows = np.unique(np.asarray(rows, np.int64))
    r = np.sqrt(np.maximum(psi, 0.0))
    # a cell can list i only if its ball meets ball i: evaluate the rows and every such site
    near = set(rows.tolist())
    for i in rows.tolist():
        d = np.linalg.norm(xyz - xyz[i], axis=1)
        near.update(np.nonzero(d < r + r[i])[0].tolist())
    ev = np.asarray(sorted(near), np.int64)
    c = cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi, box, idx=ev, domain=domain)
    side = {int(i): c.facets(k) for k, i in enumerate(ev)}
    out = {}
    for i in rows.tolist():
        # row i holds every j that lists i or that i lists (union pattern)
        js = set(side[i]) | {j for j in side if j != i and i in side[j]}
        row = {}
        for j in sorted(js):
            a, b = side[i].get(j), side[j].get(i)
            abar = a if b is None else (b if a is None else 0.5 * (a + b))
            row[j] = abar / (2.0 * float(np.linalg.norm(xyz[j] - xyz[i])))
        out[i] = row
    return out


def _mu_scaled(W, mu):
    """W with entry (i,j) multiplied by mu_ij = (mu_i + mu_j) / 2 (mu: scalar or [n])."""
    if np.ndim(mu) == 0:
        return (W * float(mu)).tocsr()
    mu = np.asarray(mu, np.float64)
    C = W.tocoo()
    import scipy.sparse as sp
    return sp.coo_matrix((C.data * 0.5 * (mu[C.row] + mu[C.col]), (C.row, C.col)), shape=W.shape).tocsr()


def p1_laplacian(W, u: np.ndarray, mu=1.0) -> np.ndarray:
    """(Lap u)_i = sum_j mu_ij w_ij (u_j - u_i) for every column of u ([n] or [n,k]),
    the P1 Laplacian of eq. (3); mu_ij = (mu_i + mu_j) / 2."""
    Wm = _mu_scaled(W, mu)
    u = np.asarray(u, np.float64)
    deg = np.asarray(Wm.sum(axis=1)).ravel()
    if u.ndim == 1:
        return Wm @ u - deg * u
    return Wm @ u - deg[:, None] * u


ADVECT_MARGIN = 1e-6


def _keep_in_planes(p, planes, pm):
    """The convex rule: a site with n.x - c + pm > 0 is moved by that amount along -n, in
    two passes over the planes in order (every product and sum rounded separately)."""
    for _ in range(2):
        for nx, ny, nz, c in planes:
            s = ((nx * p[:, 0] + ny * p[:, 1]) + nz * p[:, 2]) - c
            e = s + pm
            out = e > 0
            p[out, 0] -= e[out] * nx
            p[out, 1] -= e[out] * ny
            p[out, 2] -= e[out] * nz
    return p


def advect(xyz32: np.ndarray, v: np.ndarray, dt: float, box=((0, 0, 0), (1, 1, 1)), domain=None,
           pieces=None) -> np.ndarray:
    """Position update of the fluid step (section 5, numerical integration):
    x + dt v in float64, kept inside the domain, rounded once to float32.

    Reading (the paper does not say how sites are kept in the domain): each coordinate
    is clamped to [lo + m_a, hi - m_a] with m_a = max(1e-6 (hi_a - lo_a), u), u = 4
    float32 spacings at the largest |bound| (so that the final rounding to float32 keeps
    a clamped coordinate strictly inside); then, for convex domain planes n.x <= c, a
    site with n.x - c + m > 0 (m = max(1e-6 times the largest box extent, u)) is moved
    by that amount along -n, in two passes over the planes in order. Every product and
    sum is rounded separately.

    With ``pieces`` (a non-convex domain, the union of convex pieces given as in
    ``cells_pieces``): a site stays where it is if the plane rule with the planes of some
    piece leaves it in place (it lies inside that piece by the margin); else it takes the
    nearest, in squared distance ((dx^2 + dy^2) + dz^2), of the places the rule gives with
    each piece's planes, ties to the first piece."""
    lo = np.asarray(box[0], np.float64)
    hi = np.asarray(box[1], np.float64)
    u = 4.0 * float(np.spacing(np.float32(max(np.max(np.abs(lo)), np.max(np.abs(hi))))))
    m = np.maximum(ADVECT_MARGIN * (hi - lo), u)
    p = np.asarray(xyz32, np.float32).astype(np.float64) + dt * np.asarray(v, np.float64)
    p = np.minimum(np.maximum(p, lo + m), hi - m)
    pm = max(ADVECT_MARGIN * float(np.max(hi - lo)), u)
    if pieces is not None:
        best = p.copy()
        bestd = np.full(p.shape[0], np.inf)
        done = np.zeros(p.shape[0], bool)
        for planes, _ in pieces:
            q = _keep_in_planes(p.copy(), np.asarray(planes, np.float64).reshape(-1, 4), pm)
            dq = q - p
            d = (dq[:, 0] * dq[:, 0] + dq[:, 1] * dq[:, 1]) + dq[:, 2] * dq[:, 2]
            take = ~done & (d < bestd)
            best[take] = q[take]
            bestd[take] = d[take]
            done |= d == 0.0
        p = best
    elif domain is not None:
        p = _keep_in_planes(p, np.asarray(domain, np.float64).reshape(-1, 4), pm)
    return p.astype(np.float32)


@dataclass
class FluidStep:
    v: np.ndarray      # [n,3] velocities v^{k+1}
    Fp: np.ndarray     # [n,3] pressure spring (c_i - p_i) / eps^2
    Ft: np.ndarray     # [n,3] surface tension gamma Lap p
    Fg: np.ndarray     # [n,3] gravity m_i g
    cells: Cells
    W: object          # P1 weights (scipy CSR)


def fluid_velocity(xyz: np.ndarray, psi: np.ndarray, v: np.ndarray, mass: np.ndarray, mu, dt: float,
                   eps: float, gamma: float, gravity=(0.0, 0.0, 0.0), box=((0, 0, 0), (1, 1, 1)),
                   domain=None, solver: str = "direct", pieces=None, nwalls: int = 0) -> FluidStep:
    """Velocity update of the fluid step, section 5: with the cells at the sites ``xyz``
    and weights ``psi`` (normally the OT solution there),

      F_p = m_i (c_i - p_i) / eps^2    pressure spring to the cell centroid
      F_g = m_i g                      gravity
      F_t = gamma Lap p                surface tension, P1 Laplacian of the positions
      (m_i/dt) v_i - (Lap_mu v)_i = (m_i/dt) v^k_i + F_p + F_g + F_t     (eq. (4))

    solved exactly (sparse direct solve), or with ``solver="cg"`` by Jacobi-PCG to a
    relative residual of 1e-13 (the matrix is symmetric positive definite: m/dt on the
    diagonal plus a graph Laplacian; for large scenes, where the direct factorisation
    fills in). Lap_mu is the P1 Laplacian with mu_ij = (mu_i + mu_j) / 2. Boundary
    (wall) terms do not enter.

    The spring is read with the particle's mass, as in Gallouet-Merigot's scheme that
    the paper follows (the pull of the OT distance on site i is m_i (c_i - p_i)); the
    paper prints it without m_i, for equal masses absorbed in eps."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    xyz = np.asarray(xyz, np.float64)
    n = xyz.shape[0]
    if pieces is not None:  # a non-convex domain (cells_pieces)
        c = cells_pieces(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi, pieces, nwalls, box)
    else:
        c = cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi, box, domain=domain)
    W = p1_weights(xyz, c)
    m = np.asarray(mass, np.float64)
    Fp = m[:, None] * (c.C - xyz) / (eps * eps)
    Ft = gamma * p1_laplacian(W, xyz)
    Fg = m[:, None] * np.asarray(gravity, np.float64)[None, :]
    Wm = _mu_scaled(W, mu)
    A = (sp.diags(m / dt + np.asarray(Wm.sum(axis=1)).ravel()) - Wm).tocsc()
    b = (m / dt)[:, None] * np.asarray(v, np.float64) + Fp + Fg + Ft
    if solver == "direct":
        vn = np.stack([sla.spsolve(A, b[:, k]) for k in range(3)], axis=1)
    elif solver == "cg":
        A = A.tocsr()
        vn = np.stack([pcg(A, b[:, k], A.diagonal(), rtol=1e-13) for k in range(3)], axis=1)
    else:
        raise ValueError(f"unknown solver {solver!r}")
    return FluidStep(vn, Fp, Ft, Fg, c, W)


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
