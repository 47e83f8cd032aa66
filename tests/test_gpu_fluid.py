"""The fluid model's P1 Laplacian (eq. (3)) and semi-implicit velocity update (eq. (4))
against the FP64 oracle, through the C-ABI (lagot_p1_laplacian, lagot_fluid_velocity).

Tolerances follow from the cell parity bounds (float32 geometry): a facet area is within
1e-5 pi r^2 of the oracle's and a centroid within 1e-5 r, so a row of the Laplacian is
within T_i = 2e-5 sum_j mu_ij pi max(r_i, r_j)^2 |u_j - u_i| / (2 d_ij); the velocity
system is an M-matrix with diagonal excess m_i/dt, so ||dv||_inf <= max(dt/m) times the
largest row error of the right-hand side and of the matrix applied to v."""
import dataclasses
import math
import sys

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2601_05765_amd as L
    assert torch.cuda.is_available()
    return L.Context()


def _t(a, dt):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _sites(sc):
    import torch
    return _t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32)


def _xyz(sc):
    # the float32 positions are the input of both sides
    return np.stack([np.float32(sc.x), np.float32(sc.y), np.float32(sc.z)], 1).astype(np.float64)


def _row_tol(W, psi, xyz, u, mu, rel=2e-5):
    """T_i = rel * sum_j mu_ij pi max(r_i, r_j)^2 |u_j - u_i| / (2 d_ij) for every row."""
    C = W.tocoo()
    r = np.sqrt(np.maximum(psi, 0))
    mu = np.broadcast_to(np.asarray(mu, np.float64), (xyz.shape[0],))
    muij = 0.5 * (mu[C.row] + mu[C.col])
    d = np.linalg.norm(xyz[C.row] - xyz[C.col], axis=1)
    rr = np.maximum(r[C.row], r[C.col])
    du = np.abs(u[C.col] - u[C.row]).max(axis=1) if u.ndim == 2 else np.abs(u[C.col] - u[C.row])
    t = muij * math.pi * rr * rr * du / (2 * d)
    return rel * np.bincount(C.row, weights=t, minlength=xyz.shape[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_p1_laplacian_parity(ctx, oracle_mod, seed):
    import torch
    n = 2500
    _say(f"case: P1 Laplacian, dam_break {n}, seed {seed}")
    sc = scenes.dam_break(n, seed)
    xyz = _xyz(sc)
    rng = np.random.default_rng(10 + seed)
    u = rng.normal(size=(n, 3))
    mu = rng.uniform(0.0, 3.0, n)
    x, y, z = _sites(sc)
    psi = _t(sc.psi0, torch.float64)
    got = ctx.p1_laplacian(x, y, z, psi, _t(u, torch.float64), mu=_t(mu, torch.float64)).cpu().numpy()
    got_p = ctx.p1_laplacian(x, y, z, psi, _t(xyz, torch.float64)).cpu().numpy()
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], sc.psi0)
    W = oracle_mod.p1_weights(xyz, c)
    want = oracle_mod.p1_laplacian(W, u, mu)
    want_p = oracle_mod.p1_laplacian(W, xyz)
    tol = _row_tol(W, sc.psi0, xyz, u, mu) + 1e-14
    tol_p = _row_tol(W, sc.psi0, xyz, xyz, 1.0) + 1e-14
    e = np.abs(got - want).max(axis=1) / tol
    e_p = np.abs(got_p - want_p).max(axis=1) / tol_p
    _say(f"  max err / bound: field {e.max():.3f}, positions {e_p.max():.3f}")
    assert e.max() <= 1.0 and e_p.max() <= 1.0


def test_p1_laplacian_two_balls_closed_form(ctx):
    import torch
    r, d = 0.1, 0.12
    x = _t([0.4, 0.4 + d], torch.float32)
    y = _t([0.5, 0.5], torch.float32)
    z = _t([0.5, 0.5], torch.float32)
    xs = np.array([np.float32(0.4), np.float32(0.4 + d)], np.float64)
    dd = xs[1] - xs[0]
    psi = _t([r * r, r * r], torch.float64)
    P = np.stack([xs, [np.float32(0.5)] * 2, [np.float32(0.5)] * 2], 1)
    got = ctx.p1_laplacian(x, y, z, psi, _t(P, torch.float64)).cpu().numpy()
    a2 = r * r - dd * dd / 4
    assert np.allclose(got[0], [math.pi * a2 / 2, 0, 0], rtol=1e-5, atol=1e-9)
    assert np.allclose(got[1], -got[0], rtol=0, atol=1e-12)


def _fluid_case(n, seed):
    sc = scenes.dam_break(n, seed)
    rng = np.random.default_rng(100 + seed)
    v = rng.normal(size=(n, 3))
    mu = rng.uniform(0.0, 0.5, n)
    mass = np.asarray(sc.nu, np.float64)
    return sc, v, mu, mass


@pytest.mark.parametrize("seed,eps,gamma", [(0, 0.01, 0.05), (1, 0.02, 0.0), (2, float("inf"), 0.3)])
def test_fluid_velocity_parity(ctx, oracle_mod, seed, eps, gamma):
    import torch
    import paper_2601_05765_amd as L
    n = 2500
    _say(f"case: fluid velocity, dam_break {n}, seed {seed}, eps {eps}, gamma {gamma}")
    sc, v, mu, mass = _fluid_case(n, seed)
    xyz = _xyz(sc)
    dt = 2e-3
    prm = L.default_fluid_params(dt=dt, eps=eps, gamma=gamma, gravity=(0.0, 0.0, -9.81))
    x, y, z = _sites(sc)
    got, cen, its = ctx.fluid_velocity(x, y, z, _t(sc.psi0, torch.float64), _t(mass, torch.float64),
                                       _t(v, torch.float64), prm, mu=_t(mu, torch.float64))
    got = got.cpu().numpy()
    st = oracle_mod.fluid_velocity(xyz, sc.psi0, v, mass, mu, dt=dt, eps=eps, gamma=gamma, gravity=(0, 0, -9.81))
    r = np.sqrt(sc.psi0)
    inv_e2 = 0.0 if math.isinf(eps) else 1.0 / (eps * eps)
    rhs_err = 1e-5 * r * mass * inv_e2 + gamma * _row_tol(st.W, sc.psi0, xyz, xyz, 1.0)
    mat_err = _row_tol(st.W, sc.psi0, xyz, st.v, mu)
    bound = 2.0 * (dt / mass.min()) * (rhs_err + mat_err).max() + 1e-8 * np.abs(st.v).max()
    err = np.abs(got - st.v).max()
    _say(f"  PCG iterations {its}, max |dv| {err:.3e}, bound {bound:.3e}, max |v| {np.abs(st.v).max():.3f}")
    assert err <= bound
    assert np.abs(cen.cpu().numpy() - st.cells.C).max() <= 1e-5 * r.max()


def test_fluid_velocity_explicit_when_mu_is_zero(ctx, oracle_mod):
    import torch
    import paper_2601_05765_amd as L
    n = 1500
    sc, v, _, mass = _fluid_case(n, 3)
    xyz = _xyz(sc)
    dt = 1e-3
    prm = L.default_fluid_params(dt=dt, eps=0.02, gamma=0.2, mu=0.0)
    x, y, z = _sites(sc)
    got, _, its = ctx.fluid_velocity(x, y, z, _t(sc.psi0, torch.float64), _t(mass, torch.float64),
                                     _t(v, torch.float64), prm)
    st = oracle_mod.fluid_velocity(xyz, sc.psi0, v, mass, 0.0, dt=dt, eps=0.02, gamma=0.2, gravity=(0, 0, -9.81))
    r = np.sqrt(sc.psi0)
    bound = 2.0 * (dt / mass) * (1e-5 * r * mass / 0.02 ** 2 + 0.2 * _row_tol(st.W, sc.psi0, xyz, xyz, 1.0)) + 1e-12
    err = np.abs(got.cpu().numpy() - st.v).max(axis=1)
    _say(f"  PCG iterations {its}, max err / bound {np.max(err / bound):.3f}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("per_site", [False, True])
def test_fluid_velocity_full_size_invariants(ctx, per_site):
    """100,000-site dam break (the measured workload): a constant velocity field with no
    forces is kept, and with gravity and surface tension only the total momentum grows by
    dt g sum m (the P1 Laplacian's rows and columns sum to zero)."""
    import torch
    import paper_2601_05765_amd as L
    n = 100_000
    _say(f"case: fluid velocity invariants, dam_break {n}, per-site mu {per_site}")
    sc = scenes.dam_break(n, 0)
    rng = np.random.default_rng(7)
    mu = _t(rng.uniform(0.0, 2.0, n), torch.float64) if per_site else None
    mass = _t(sc.nu, torch.float64)
    x, y, z = _sites(sc)
    psi = _t(sc.psi0, torch.float64)
    U = torch.tensor([0.3, -1.2, 0.45], dtype=torch.float64, device="cuda").repeat(n, 1).contiguous()
    prm = L.default_fluid_params(dt=2e-3, eps=float("inf"), gamma=0.0, mu=1.0, gravity=(0.0, 0.0, 0.0))
    v1, _, its = ctx.fluid_velocity(x, y, z, psi, mass, U, prm, mu=mu)
    e = (v1 - U).abs().max().item()
    _say(f"  constant field: PCG iterations {its}, max |v - U| {e:.2e}")
    assert e <= 1e-8
    v0 = _t(rng.normal(size=(n, 3)), torch.float64)
    prm = L.default_fluid_params(dt=2e-3, eps=float("inf"), gamma=0.5, mu=1.0, gravity=(0.0, 0.0, -9.81))
    v2, _, its = ctx.fluid_velocity(x, y, z, psi, mass, v0, prm, mu=mu)
    m = mass[:, None]
    got = (m * v2).sum(0).cpu().numpy()
    want = (m * v0).sum(0).cpu().numpy() + 2e-3 * np.array([0, 0, -9.81]) * float(mass.sum())
    scale = float((m * v0.abs()).sum())
    _say(f"  momentum: PCG iterations {its}, error {np.abs(got - want).max() / scale:.2e} (relative)")
    assert np.abs(got - want).max() <= 1e-8 * scale
    # kinetic energy of the viscous part does not grow
    prm0 = L.default_fluid_params(dt=2e-3, eps=float("inf"), gamma=0.0, mu=1.0, gravity=(0.0, 0.0, 0.0))
    v3, _, _ = ctx.fluid_velocity(x, y, z, psi, mass, v0, prm0, mu=mu)
    assert float((m * v3 * v3).sum()) < float((m * v0 * v0).sum())


def test_fluid_velocity_single_site(ctx):
    import torch
    import paper_2601_05765_amd as L
    x = _t([0.5], torch.float32)
    y = _t([0.5], torch.float32)
    z = _t([0.5], torch.float32)
    psi = _t([0.1 ** 2], torch.float64)
    mass = _t([2e-3], torch.float64)
    v = _t([[1.0, 2.0, 3.0]], torch.float64)
    prm = L.default_fluid_params(dt=0.01, eps=0.1, gamma=1.0, mu=5.0, gravity=(0.0, 0.0, -9.81))
    out, cen, its = ctx.fluid_velocity(x, y, z, psi, mass, v, prm)
    # one isolated ball: centroid = site, no facets, so v + dt g
    assert np.allclose(out.cpu().numpy(), [[1.0, 2.0, 3.0 - 0.0981]], rtol=0, atol=1e-12)
    assert np.allclose(cen.cpu().numpy(), [[0.5, 0.5, 0.5]], atol=0)


def test_fluid_velocity_rejects_bad_input(ctx):
    import torch
    import paper_2601_05765_amd as L
    sc, v, _, mass = _fluid_case(500, 4)
    x, y, z = _sites(sc)
    psi = _t(sc.psi0, torch.float64)
    bad = mass.copy()
    bad[17] = 0.0
    with pytest.raises(L.LagotError) as ei:
        ctx.fluid_velocity(x, y, z, psi, _t(bad, torch.float64), _t(v, torch.float64))
    assert ei.value.code == L.EINVAL
    with pytest.raises(L.LagotError) as ei:
        ctx.fluid_velocity(x, y, z, psi, _t(mass, torch.float64), _t(v, torch.float64),
                           L.default_fluid_params(dt=0.0))
    assert ei.value.code == L.EINVAL
    # the context still works after the rejected calls
    out, _, _ = ctx.fluid_velocity(x, y, z, psi, _t(mass, torch.float64), _t(v, torch.float64))
    assert torch.isfinite(out).all()


@pytest.mark.parametrize("seed,planes", [(0, False), (1, False), (2, True)])
def test_fluid_step_parity(ctx, oracle_mod, seed, planes):
    """One whole step: positions bit-exact against the oracle's update (same clamp
    reading), weights valid under the oracle's own cell evaluation (the stop test holds),
    velocities within the bound of the velocity test at the new cells."""
    import torch
    import paper_2601_05765_amd as L
    n = 2500
    _say(f"case: fluid step, dam_break {n}, seed {seed}, domain planes {planes}")
    sc, v, mu, mass = _fluid_case(n, seed)
    v[:, 2] -= 1.0  # falling: the bottom layer reaches the floor and is clamped
    dt, eps, gamma = 0.03, 0.05, 0.05
    dom = None
    if planes:
        nrm = np.array([1.0, 0.0, 1.0]) / math.sqrt(2.0)
        P = [[-1, 0, 0, 0], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1],
             [nrm[0], nrm[1], nrm[2], float(nrm @ [0.9, 0, 0.45])]]
        dom = np.asarray(P, np.float32).astype(np.float64)
        xyz0 = _xyz(sc)
        keep = np.all(xyz0 @ dom[:, :3].T < dom[:, 3] - 1e-4, axis=1)
        sc = dataclasses.replace(sc, x=sc.x[keep], y=sc.y[keep], z=sc.z[keep], nu=sc.nu[keep], psi0=sc.psi0[keep])
        v, mu, mass = v[keep], mu[keep], mass[keep]
        n = int(keep.sum())
        ctx.set_domain(dom)
    try:
        xyz0 = _xyz(sc)
        x, y, z = _sites(sc)
        psi = _t(sc.psi0, torch.float64)
        vt = _t(v, torch.float64)
        prm = L.default_fluid_params(dt=dt, eps=eps, gamma=gamma, gravity=(0.0, 0.0, -9.81))
        st, its = ctx.fluid_step(x, y, z, _t(sc.nu, torch.float64), psi, _t(mass, torch.float64), vt, prm,
                                 opts=L.default_opts(tol=1e-5), mu=_t(mu, torch.float64))
    finally:
        if planes:
            ctx.set_domain(None)
    x1 = np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)
    want = oracle_mod.advect(xyz0.astype(np.float32), v, dt, domain=dom)
    moved = np.abs(want.astype(np.float64) - (xyz0 + dt * v)).max(axis=1) > 1e-6
    _say(f"  {int(moved.sum())} sites clamped; solve status {st.status}, {st.newton_iters} Newton iterations; "
         f"PCG {its}")
    assert moved.sum() > 0
    assert np.array_equal(x1, want)
    assert st.status == 0
    xyz1 = x1.astype(np.float64)
    p1 = psi.cpu().numpy()
    c = oracle_mod.cells(xyz1[:, 0], xyz1[:, 1], xyz1[:, 2], p1, domain=dom)
    err = float(np.max(np.abs(c.V - sc.nu) / sc.nu))
    _say(f"  oracle max rel volume error at the new weights {err:.2e}")
    assert err <= 1e-5
    so = oracle_mod.fluid_velocity(xyz1, p1, v, mass, mu, dt=dt, eps=eps, gamma=gamma, gravity=(0, 0, -9.81),
                                   domain=dom)
    r = np.sqrt(p1)
    rhs_err = 1e-5 * r * mass / (eps * eps) + gamma * _row_tol(so.W, p1, xyz1, xyz1, 1.0)
    mat_err = _row_tol(so.W, p1, xyz1, so.v, mu)
    bound = 2.0 * (dt / mass.min()) * (rhs_err + mat_err).max() + 1e-8 * np.abs(so.v).max()
    e = np.abs(vt.cpu().numpy() - so.v).max()
    _say(f"  max |dv| {e:.3e}, bound {bound:.3e}")
    assert e <= bound


def test_fluid_steps_dam_break_100k(ctx):
    """Three steps of the 100,000-site dam break from rest under gravity (the measured
    workload): every solve meets its tolerance and every site stays strictly inside the box."""
    import torch
    import paper_2601_05765_amd as L
    n = 100_000
    _say(f"case: fluid steps, dam_break {n}")
    sc = scenes.dam_break(n, 0)
    x, y, z = _sites(sc)
    nu = _t(sc.nu, torch.float64)
    psi = _t(sc.psi0, torch.float64)
    v = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    mu = _t(np.random.default_rng(5).uniform(0.0, 2.0, n), torch.float64)
    prm = L.default_fluid_params(dt=2e-3, eps=0.02, gamma=0.05)
    for k in range(3):
        st, its = ctx.fluid_step(x, y, z, nu, psi, nu, v, prm, opts=L.default_opts(tol=1e-5), mu=mu)
        _say(f"  step {k}: status {st.status}, {st.newton_iters} Newton iterations, max rel err "
             f"{st.max_rel_err:.2e}, PCG {its}, max |v| {v.abs().max().item():.3f}")
        assert st.status == 0 and st.max_rel_err <= 1e-5
    P = torch.stack([x, y, z], 1).double()
    assert float(P.min()) > 0.0 and float(P.max()) < 1.0
    assert float(v[:, 2].mean()) < 0  # the column falls


def test_fluid_step_rejects_bad_parameters_before_moving(ctx):
    import torch
    import paper_2601_05765_amd as L
    sc, v, _, mass = _fluid_case(500, 6)
    x, y, z = _sites(sc)
    x0 = x.clone()
    psi = _t(sc.psi0, torch.float64)
    for bad in (dict(eps=-1.0), dict(dt=0.0), dict(gamma=float("nan")), dict(cg_rtol=2.0)):
        with pytest.raises(L.LagotError) as ei:
            ctx.fluid_step(x, y, z, _t(sc.nu, torch.float64), psi, _t(mass, torch.float64), _t(v, torch.float64),
                           L.default_fluid_params(**bad))
        assert ei.value.code == L.EINVAL
        assert torch.equal(x, x0)
    # invalid per-site inputs and options are found before the sites move too
    m_bad = mass.copy()
    m_bad[7] = 0.0
    v_bad = v.copy()
    v_bad[11, 2] = float("inf")
    nu_bad = sc.nu.copy()
    nu_bad[3] = -1.0
    cases = [(sc.nu, m_bad, v, None, None), (sc.nu, mass, v_bad, None, None), (nu_bad, mass, v, None, None),
             (sc.nu, mass, v, -np.ones(sc.n), None), (sc.nu, mass, v, None, L.default_opts(tol=-1.0))]
    for nu_c, m_c, v_c, mu_c, opts in cases:
        with pytest.raises(L.LagotError) as ei:
            ctx.fluid_step(x, y, z, _t(nu_c, torch.float64), psi, _t(m_c, torch.float64), _t(v_c, torch.float64),
                           L.default_fluid_params(), opts=opts,
                           mu=None if mu_c is None else _t(mu_c, torch.float64))
        assert ei.value.code == L.EINVAL
        assert torch.equal(x, x0)


def test_p1_laplacian_dam_break_100k_sampled(ctx, oracle_mod):
    """The measured workload at full size: 200 sampled rows of the Laplacian against the
    oracle's rows (their cells and every overlapping cell evaluated by brute force)."""
    import scipy.sparse as sp
    import torch
    n = 100_000
    _say(f"case: P1 Laplacian, dam_break {n}, 200 sampled rows")
    sc = scenes.dam_break(n, 0)
    xyz = _xyz(sc)
    rng = np.random.default_rng(21)
    u = rng.normal(size=(n, 3))
    mu = rng.uniform(0.0, 3.0, n)
    x, y, z = _sites(sc)
    got = ctx.p1_laplacian(x, y, z, _t(sc.psi0, torch.float64), _t(u, torch.float64),
                           mu=_t(mu, torch.float64)).cpu().numpy()
    rows = np.sort(rng.choice(n, 200, replace=False))
    R = oracle_mod.p1_rows(xyz, sc.psi0, rows)
    ri = [i for i in rows for _ in R[int(i)]]
    rj = [j for i in rows for j in R[int(i)]]
    rv = [w for i in rows for w in R[int(i)].values()]
    W = sp.coo_matrix((rv, (ri, rj)), shape=(n, n)).tocsr()
    want = oracle_mod.p1_laplacian(W, u, mu)[rows]
    tol = _row_tol(W, sc.psi0, xyz, u, mu)[rows] + 1e-14
    e = np.abs(got[rows] - want).max(axis=1) / tol
    _say(f"  max err / bound {e.max():.3f}")
    assert e.max() <= 1.0


def test_fluid_step_in_the_l_prism(ctx, oracle_mod):
    """One whole step in a non-convex domain (the L-shaped prism, 3 convex pieces): sites
    pushed towards the removed quarter; positions bit-exact against the oracle's update
    (sites that enter the quarter go to the nearest piece), the new weights valid under
    the oracle's cells in the pieces, velocities within the bound of the velocity test."""
    import torch
    import paper_2601_05765_amd as L
    n = 2500
    _say(f"case: fluid step in the L prism, {n} sites")
    sc = scenes.l_shape_sites(n, 6)
    rng = np.random.default_rng(7)
    v = rng.normal(size=(n, 3)) + np.array([1.5, 1.5, 0.0])
    mu = rng.uniform(0.0, 0.5, n)
    mass = np.asarray(sc.nu, np.float64)
    dt, eps, gamma = 0.03, 0.05, 0.05
    pieces = scenes.l_shape_pieces()
    xyz0 = _xyz(sc)
    x, y, z = _sites(sc)
    psi = _t(sc.psi0, torch.float64)
    vt = _t(v, torch.float64)
    prm = L.default_fluid_params(dt=dt, eps=eps, gamma=gamma, gravity=(0.0, 0.0, -9.81))
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        st, its = ctx.fluid_step(x, y, z, _t(sc.nu, torch.float64), psi, _t(mass, torch.float64), vt, prm,
                                 opts=L.default_opts(tol=1e-5), mu=_t(mu, torch.float64))
    finally:
        ctx.set_domain(None)
    x1 = np.stack([x.cpu().numpy(), y.cpu().numpy(), z.cpu().numpy()], 1)
    want = oracle_mod.advect(xyz0.astype(np.float32), v, dt, pieces=pieces)
    free = xyz0 + dt * v
    moved = np.abs(want.astype(np.float64) - free).max(axis=1) > 1e-6
    quarter = (free[:, 0] > 0.5) & (free[:, 1] > 0.5)
    _say(f"  {int(moved.sum())} sites kept in the domain ({int(quarter.sum())} from the removed quarter); "
         f"solve status {st.status}, {st.newton_iters} Newton iterations; PCG {its}")
    assert quarter.sum() > 20
    assert np.array_equal(x1, want)
    assert st.status == 0
    xyz1 = x1.astype(np.float64)
    p1 = psi.cpu().numpy()
    c = oracle_mod.cells_pieces(xyz1[:, 0], xyz1[:, 1], xyz1[:, 2], p1, pieces, scenes.L_WALLS)
    err = float(np.max(np.abs(c.V - sc.nu) / sc.nu))
    _say(f"  oracle max rel volume error at the new weights {err:.2e}")
    assert err <= 1e-5
    so = oracle_mod.fluid_velocity(xyz1, p1, v, mass, mu, dt=dt, eps=eps, gamma=gamma, gravity=(0, 0, -9.81),
                                   pieces=pieces, nwalls=scenes.L_WALLS)
    r = np.sqrt(p1)
    rhs_err = 1e-5 * r * mass / (eps * eps) + gamma * _row_tol(so.W, p1, xyz1, xyz1, 1.0)
    mat_err = _row_tol(so.W, p1, xyz1, so.v, mu)
    bound = 2.0 * (dt / mass.min()) * (rhs_err + mat_err).max() + 1e-8 * np.abs(so.v).max()
    e = np.abs(vt.cpu().numpy() - so.v).max()
    _say(f"  max |dv| {e:.3e}, bound {bound:.3e}")
    assert e <= bound
