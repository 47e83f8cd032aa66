"""Pins of the oracle's fluid-model pieces (section 5): the P1 Laplacian of eq. (3) and
the semi-implicit velocity update of eq. (4).

The pins use facts the oracle's own formulas do not restate: the lens geometry of two
balls (disc area), the closed-polytope identity sum_j |V_ij| n_ij = 0 (with the box walls
read from the clipper's wall areas), the cubic lattice, the two-particle system solved
by hand, and the invariants of the linear system (constants are kept, momentum is
conserved, kinetic energy does not grow, mu = 0 is the explicit update)."""
import math

import numpy as np
import pytest


def _two_balls(r, d):
    xyz = np.array([[0.4, 0.5, 0.5], [0.4 + d, 0.5, 0.5]])
    return xyz, np.array([r * r, r * r])


@pytest.mark.parametrize("r,d", [(0.1, 0.12), (0.08, 0.05), (0.15, 0.29)])
def test_two_balls_weight_and_laplacian(oracle_mod, r, d):
    """Equal balls at distance d < 2r meet in a disc of radius a = sqrt(r^2 - d^2/4):
    w_12 = pi a^2 / (2 d), and Lap p_1 = w_12 (p_2 - p_1) = (pi a^2 / 2) e_x."""
    xyz, psi = _two_balls(r, d)
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi)
    W = oracle_mod.p1_weights(xyz, c)
    a2 = r * r - d * d / 4
    assert W[0, 1] == pytest.approx(math.pi * a2 / (2 * d), rel=1e-12)
    assert W[1, 0] == W[0, 1]
    L = oracle_mod.p1_laplacian(W, xyz)
    assert np.allclose(L[0], [math.pi * a2 / 2, 0, 0], rtol=1e-12, atol=1e-15)
    assert np.allclose(L[1], [-math.pi * a2 / 2, 0, 0], rtol=1e-12, atol=1e-15)


def test_closed_cells_laplacian_of_positions(oracle_mod):
    """For a cell with no spherical part, its boundary is closed by neighbour facets and
    wall facets, and the outward area vectors sum to zero. With n_ij = (p_j - p_i)/d_ij,
    Lap p_i = 1/2 sum_j |V_ij| n_ij = -1/2 sum_walls A_w n_w. Every wall area comes from
    the clipper, not from the weights."""
    rng = np.random.default_rng(5)
    n = 200
    xyz = rng.uniform(0.02, 0.98, (n, 3))
    psi = np.full(n, 0.5 ** 2)  # balls far larger than the cells: plain power diagram
    psi += rng.uniform(0, 2e-3, n)
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi)
    assert np.abs(c.K).max() < 1e-12  # no spherical part (up to rounding)
    W = oracle_mod.p1_weights(xyz, c)
    L = oracle_mod.p1_laplacian(W, xyz)
    normals = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.float64)
    wall_vec = c.walls @ normals
    assert np.abs(wall_vec).max() > 1e-3  # the identity is not trivially zero
    assert np.allclose(L, -0.5 * wall_vec, atol=1e-12)


def test_cubic_lattice_laplacian_of_a_quadratic(oracle_mod):
    """Sites on a cubic lattice of spacing h, cells are cubes: w = h^2 / (2h) = h/2 for
    the six face neighbours, so an interior site has Lap x^2 = (h/2)((x+h)^2 + (x-h)^2 - 2x^2)
    = h^3 = |C_i| * 2, the cell integral of the continuous Laplacian of x^2."""
    k = 6
    h = 1.0 / k
    g = (np.arange(k) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    psi = np.full(xyz.shape[0], 1.0)
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi)
    W = oracle_mod.p1_weights(xyz, c)
    L = oracle_mod.p1_laplacian(W, xyz[:, 0] ** 2 + 3 * xyz[:, 1] - xyz[:, 2])
    inner = np.all((xyz > h) & (xyz < 1 - h), axis=1)
    assert inner.sum() == (k - 2) ** 3
    assert np.allclose(L[inner], h ** 3, rtol=1e-11)


def _blob(n, seed):
    rng = np.random.default_rng(seed)
    xyz = 0.5 + 0.22 * (rng.uniform(-1, 1, (n, 3)))
    psi = np.full(n, (0.6 * 0.44 / n ** (1 / 3)) ** 2 * 4)
    return xyz, psi, rng


def test_explicit_update_when_mu_is_zero(oracle_mod):
    xyz, psi, rng = _blob(120, 1)
    v = rng.normal(size=(120, 3))
    m = rng.uniform(0.5, 2.0, 120) * 1e-3
    st = oracle_mod.fluid_velocity(xyz, psi, v, m, 0.0, dt=0.01, eps=0.3, gamma=0.7, gravity=(0, 0, -9.81))
    want = v + 0.01 / m[:, None] * (st.Fp + st.Fg + st.Ft)
    assert np.allclose(st.v, want, rtol=1e-12, atol=1e-12)
    assert np.allclose(st.Fg[:, 2], -9.81 * m)
    assert np.allclose(st.Fp, m[:, None] * (st.cells.C - xyz) / 0.09)


@pytest.mark.parametrize("mu", [0.3, "site"])
def test_constant_velocity_is_kept(oracle_mod, mu):
    xyz, psi, rng = _blob(150, 2)
    m = rng.uniform(0.5, 2.0, 150) * 1e-3
    muv = rng.uniform(0.0, 5.0, 150) if mu == "site" else mu
    U = np.array([0.3, -1.2, 0.45])
    v = np.tile(U, (150, 1))
    st = oracle_mod.fluid_velocity(xyz, psi, v, m, muv, dt=0.02, eps=1e30, gamma=0.0)
    assert np.allclose(st.v, v, rtol=1e-12, atol=1e-13)


def test_momentum_and_energy(oracle_mod):
    """Lap_mu has zero row and column sums when mu_ij is symmetric, so total momentum
    changes only by dt * sum of the forces; with no forces the update is a contraction
    in the mass-weighted norm (kinetic energy does not grow)."""
    xyz, psi, rng = _blob(180, 3)
    m = rng.uniform(0.5, 2.0, 180) * 1e-3
    muv = rng.uniform(0.0, 3.0, 180)
    v = rng.normal(size=(180, 3))
    dt = 0.01
    st = oracle_mod.fluid_velocity(xyz, psi, v, m, muv, dt=dt, eps=0.2, gamma=0.4, gravity=(0, 0, -9.81))
    F = st.Fp + st.Fg + st.Ft
    assert np.allclose((m[:, None] * st.v).sum(0), (m[:, None] * v).sum(0) + dt * F.sum(0), rtol=0, atol=1e-12)
    st0 = oracle_mod.fluid_velocity(xyz, psi, v, m, muv, dt=dt, eps=1e30, gamma=0.0)
    e0 = (m[:, None] * v * v).sum()
    e1 = (m[:, None] * st0.v * st0.v).sum()
    assert e1 < e0 * (1 - 1e-3)
    # the viscous step moves velocities toward their neighbours' (it damps the jump)
    assert np.abs(st0.v - st0.v.mean(0)).max() < np.abs(v - v.mean(0)).max()


def test_cg_solver_matches_the_direct_solve(oracle_mod):
    """The iterative solve of eq. (4) (Jacobi-PCG, for scenes too large to factorise)
    reaches the sparse direct solution; it also keeps the momentum balance, which the
    direct solve satisfies exactly."""
    xyz, psi, rng = _blob(180, 5)
    m = rng.uniform(0.5, 2.0, 180) * 1e-3
    muv = rng.uniform(0.0, 3.0, 180)
    v = rng.normal(size=(180, 3))
    dt = 0.01
    kw = dict(dt=dt, eps=0.2, gamma=0.4, gravity=(0, 0, -9.81))
    a = oracle_mod.fluid_velocity(xyz, psi, v, m, muv, **kw)
    b = oracle_mod.fluid_velocity(xyz, psi, v, m, muv, solver="cg", **kw)
    assert np.abs(b.v - a.v).max() <= 1e-10 * np.abs(a.v).max()
    F = b.Fp + b.Fg + b.Ft
    assert np.allclose((m[:, None] * b.v).sum(0), (m[:, None] * v).sum(0) + dt * F.sum(0), rtol=0, atol=1e-10)
    with pytest.raises(ValueError):
        oracle_mod.fluid_velocity(xyz, psi, v, m, muv, solver="lu", **kw)


@pytest.mark.parametrize("mu1,mu2,m1,m2", [(1.0, 1.0, 1e-3, 1e-3), (0.2, 3.0, 1e-3, 4e-3)])
def test_two_particle_system_by_hand(oracle_mod, mu1, mu2, m1, m2):
    """Two cells sharing one facet: with k = mu_12 w_12 dt, mu_12 = (mu1 + mu2)/2,
    m1 v1 + k (v1 - v2) = m1 u1 and m2 v2 + k (v2 - v1) = m2 u2, so the relative velocity
    is divided by 1 + k (1/m1 + 1/m2) and the momentum m1 v1 + m2 v2 is kept."""
    r, d, dt = 0.1, 0.12, 0.05
    xyz, psi = _two_balls(r, d)
    u = np.array([[0.5, -0.2, 0.1], [-0.3, 0.4, 0.0]])
    st = oracle_mod.fluid_velocity(xyz, psi, u, np.array([m1, m2]), np.array([mu1, mu2]), dt=dt, eps=1e30,
                                   gamma=0.0)
    w = math.pi * (r * r - d * d / 4) / (2 * d)
    k = 0.5 * (mu1 + mu2) * w * dt
    rel = (u[0] - u[1]) / (1 + k * (1 / m1 + 1 / m2))
    mom = m1 * u[0] + m2 * u[1]
    assert np.allclose(st.v[0] - st.v[1], rel, rtol=1e-12)
    assert np.allclose(m1 * st.v[0] + m2 * st.v[1], mom, rtol=1e-12)


def test_surface_tension_pulls_the_pair_together(oracle_mod):
    xyz, psi = _two_balls(0.1, 0.12)
    st = oracle_mod.fluid_velocity(xyz, psi, np.zeros((2, 3)), np.array([1e-3, 1e-3]), 0.0, dt=0.01, eps=1e30,
                                   gamma=2.0)
    assert st.Ft[0, 0] > 0 and st.Ft[1, 0] < 0
    assert st.v[0, 0] > 0 and st.v[1, 0] < 0


def test_advect_inside_is_the_plain_update(oracle_mod):
    rng = np.random.default_rng(9)
    x = rng.uniform(0.3, 0.7, (50, 3)).astype(np.float32)
    v = rng.normal(size=(50, 3))
    got = oracle_mod.advect(x, v, 0.01)
    assert np.array_equal(got, (x.astype(np.float64) + 0.01 * v).astype(np.float32))


def test_advect_clamps_to_the_box_margin(oracle_mod):
    box = ((0.0, -1.0, 2.0), (1.0, 3.0, 2.5))
    x = np.array([[0.5, 0.0, 2.2], [0.999, 2.9, 2.49]], np.float32)
    v = np.array([[-100.0, -100.0, -100.0], [100.0, 100.0, 100.0]])
    got = oracle_mod.advect(x, v, 1.0, box).astype(np.float64)
    lo, hi = np.array(box[0]), np.array(box[1])
    # margin 1e-6 of the extent, at least 4 float32 spacings at the largest bound (3.0)
    m = np.maximum(1e-6 * (hi - lo), 4.0 * 2.0 ** -22)
    assert np.allclose(got[0], lo + m, rtol=0, atol=1e-7 * 4) and np.all(got[0] > lo)
    assert np.allclose(got[1], hi - m, rtol=0, atol=1e-7 * 4) and np.all(got[1] < hi)


def test_advect_margin_survives_float32_rounding_far_from_the_origin(oracle_mod):
    """A box far from the origin, [100, 101]^3: 1e-6 of the extent is below one float32
    spacing at 100 (7.6e-6), so the margin is 4 spacings; clamped sites round to float32
    strictly inside the box (the site validation's strict test passes)."""
    box = ((100.0, 100.0, 100.0), (101.0, 101.0, 101.0))
    x = np.array([[100.5, 100.5, 100.5], [100.9, 100.1, 100.5]], np.float32)
    v = np.array([[-50.0, 50.0, 0.0], [50.0, -50.0, 0.0]])
    got = oracle_mod.advect(x, v, 1.0, box)
    assert np.all(got > np.float32(100.0)) and np.all(got < np.float32(101.0))
    sp = float(np.spacing(np.float32(101.0)))
    assert abs(float(got[0, 0]) - (100.0 + 4 * sp)) <= sp and abs(float(got[0, 1]) - (101.0 - 4 * sp)) <= sp


def test_advect_projects_onto_a_domain_plane(oracle_mod):
    n = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    c = float(n @ [0.6, 0.6, 0.0])
    x = np.array([[0.5, 0.5, 0.5], [0.2, 0.3, 0.5]], np.float32)
    v = np.array([[0.3, 0.2, 0.1], [0.0, 0.0, 0.0]])
    got = oracle_mod.advect(x, v, 1.0, domain=[[n[0], n[1], n[2], c]]).astype(np.float64)
    # the first site crossed the plane: it lands on n.x = c - 1e-6, displaced along -n only
    assert abs(got[0] @ n - (c - 1e-6)) < 2e-7
    d = got[0] - (x[0].astype(np.float64) + v[0])
    assert np.allclose(d - (d @ n) * n, 0, atol=2e-7)
    assert np.array_equal(got[1], x[1])


@pytest.mark.parametrize("m", [1e-4, 3.0])
def test_spring_acceleration_of_a_ball_at_a_wall(oracle_mod, m):
    """One ball of radius r at distance a from the floor: its cell is the ball minus a cap
    of height r - a, whose centroid lies V_cap z_cap / (V_ball - V_cap) above the site
    (closed form). The spring's acceleration (c - p)/eps^2 does not depend on the mass."""
    r, a, eps, dt = 0.2, 0.07, 0.05, 0.01
    p = np.array([[0.5, 0.5, a]])
    h = r - a
    vcap = math.pi * h * h * (3 * r - h) / 3
    zc = 3 * (2 * r - h) ** 2 / (4 * (3 * r - h))
    shift = vcap * zc / (4 / 3 * math.pi * r ** 3 - vcap)
    v0 = np.array([[0.1, -0.2, 0.3]])
    st = oracle_mod.fluid_velocity(p, np.array([r * r]), v0, np.array([m]), 2.0, dt=dt, eps=eps, gamma=1.0,
                                   gravity=(0, 0, -9.81))
    assert np.allclose(st.v[0], v0[0] + dt * np.array([0, 0, shift / eps ** 2 - 9.81]), rtol=1e-12, atol=1e-12)


def test_p1_rows_match_the_full_matrix(oracle_mod):
    """The sampled-row form gives the rows of the full assembly (same union pattern)."""
    rng = np.random.default_rng(11)
    n = 300
    xyz = rng.uniform(0.05, 0.95, (n, 3))
    psi = rng.uniform(0.06, 0.12, n) ** 2
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi)
    W = oracle_mod.p1_weights(xyz, c).tocsr()
    rows = rng.choice(n, 25, replace=False)
    got = oracle_mod.p1_rows(xyz, psi, rows)
    for i in rows:
        lo, hi = W.indptr[i], W.indptr[i + 1]
        want = dict(zip(W.indices[lo:hi].tolist(), W.data[lo:hi].tolist()))
        assert set(got[int(i)]) == set(want)
        for j, w in want.items():
            assert got[int(i)][j] == pytest.approx(w, rel=1e-13)
