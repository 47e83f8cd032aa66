"""Pins of the oracle's cell geometry against closed forms (eq. (1); pyramid
decomposition of section 3.2; occlusion identity of section 3.3).

Every expected value below is an independent textbook formula (ball, spherical
cap, lens, ball-cube intersection), never a call into the oracle."""
import math

import numpy as np
import pytest


def cap_volume(r, t):
    """Volume of {y in B(0,r) : n.y <= t}, -r < t < r (height h = r + t)."""
    h = r + t
    return math.pi * h * h * (3 * r - h) / 3.0


def cap_sphere_area(r, t):
    return 2 * math.pi * r * (r + t)


@pytest.mark.parametrize("r", [0.01, 0.05, 0.2])
def test_isolated_ball(oracle_mod, r):
    c = oracle_mod.cells([0.5], [0.5], [0.5], [r * r])
    assert c.V[0] == pytest.approx(4 / 3 * math.pi * r ** 3, rel=1e-13)
    assert c.K[0] == pytest.approx(4 * math.pi * r * r, rel=1e-13)
    assert c.fcount[0] == 0 and np.all(c.walls[0] == 0)


@pytest.mark.parametrize("wall", range(6))
def test_ball_cut_by_one_wall(oracle_mod, wall):
    r, a = 0.1, 0.037
    p = [0.5, 0.5, 0.5]
    ax = wall // 2
    p[ax] = a if wall % 2 == 0 else 1 - a
    c = oracle_mod.cells([p[0]], [p[1]], [p[2]], [r * r])
    assert c.V[0] == pytest.approx(cap_volume(r, a), rel=1e-12)
    assert c.K[0] == pytest.approx(cap_sphere_area(r, a), rel=1e-12)
    expect = np.zeros(6)
    expect[wall] = math.pi * (r * r - a * a)
    np.testing.assert_allclose(c.walls[0], expect, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("r1,r2,d", [(0.1, 0.1, 0.12), (0.1, 0.13, 0.15), (0.05, 0.14, 0.12), (0.14, 0.05, 0.12)])
def test_two_balls_lens(oracle_mod, r1, r2, d):
    """Two balls: the radical plane at t1 = (d^2 + r1^2 - r2^2)/(2d) from p1; the
    third case puts p1 beyond the plane (t1 < 0), the fourth p2 (t2 < 0)."""
    c = oracle_mod.cells([0.4, 0.4 + d], [0.5, 0.5], [0.5, 0.5], [r1 * r1, r2 * r2])
    t1 = (d * d + r1 * r1 - r2 * r2) / (2 * d)
    t2 = d - t1
    rho2 = r1 * r1 - t1 * t1
    assert abs(rho2 - (r2 * r2 - t2 * t2)) < 1e-15
    assert c.V[0] == pytest.approx(cap_volume(r1, t1), rel=1e-12)
    assert c.V[1] == pytest.approx(cap_volume(r2, t2), rel=1e-12)
    assert c.K[0] == pytest.approx(cap_sphere_area(r1, t1), rel=1e-12)
    assert c.K[1] == pytest.approx(cap_sphere_area(r2, t2), rel=1e-12)
    assert c.facets(0)[1] == pytest.approx(math.pi * rho2, rel=1e-12)
    assert c.facets(1)[0] == pytest.approx(math.pi * rho2, rel=1e-12)


def test_engulfed_ball_is_empty(oracle_mod):
    """d + r1 <= r2: every point of ball 1 has lower power w.r.t. site 2 -> empty cell."""
    r1, r2, d = 0.03, 0.12, 0.05
    c = oracle_mod.cells([0.4, 0.4 + d], [0.5, 0.5], [0.5, 0.5], [r1 * r1, r2 * r2])
    assert c.status[0] == 1 and c.V[0] == 0 and c.K[0] == 0
    assert c.V[1] == pytest.approx(4 / 3 * math.pi * r2 ** 3, rel=1e-12)


def test_disjoint_balls_do_not_interact(oracle_mod):
    r = 0.05
    c = oracle_mod.cells([0.3, 0.3 + 2 * r + 1e-3], [0.5, 0.5], [0.5, 0.5], [r * r, r * r])
    assert c.fcount.tolist() == [0, 0]
    np.testing.assert_allclose(c.V, 4 / 3 * math.pi * r ** 3, rtol=1e-13)


def _lattice(m, h, r):
    g = (np.arange(m) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    return x, y, z, np.full(x.shape, r * r)


@pytest.mark.parametrize("ratio", [0.52, 0.6, 0.7])
def test_lattice_ball_cube(oracle_mod, ratio):
    """Cubic lattice, equal weights, h/2 < r < h/sqrt(2): an interior cell is the cube of
    side h intersected with the ball, i.e. the ball minus six disjoint caps."""
    m, h = 5, 0.2
    r = ratio * h
    x, y, z, psi = _lattice(m, h, r)
    centre = (2 * m + 2) * m + 2  # index of (2,2,2)
    c = oracle_mod.cells(x, y, z, psi, idx=[centre])
    cc = r - h / 2
    V = 4 / 3 * math.pi * r ** 3 - 6 * math.pi * cc * cc * (3 * r - cc) / 3
    K = 4 * math.pi * r * r - 12 * math.pi * r * cc
    assert c.V[0] == pytest.approx(V, rel=1e-12)
    assert c.K[0] == pytest.approx(K, rel=1e-12)
    f = c.facets(0)
    assert len(f) == 6
    for a in f.values():
        assert a == pytest.approx(math.pi * (r * r - h * h / 4), rel=1e-12)


def test_large_radius_tiling(oracle_mod):
    """r > h sqrt(3)/2: every ball covers its lattice cube, so cells tile the box:
    V = h^3, K = 0, interior facets are h^2 squares, volumes sum to the box."""
    m, h = 4, 0.25
    x, y, z, psi = _lattice(m, h, 0.9 * h)
    c = oracle_mod.cells(x, y, z, psi)
    np.testing.assert_allclose(c.V, h ** 3, rtol=1e-12)
    np.testing.assert_allclose(c.K, 0.0, atol=1e-13)
    assert c.V.sum() == pytest.approx(1.0, rel=1e-12)
    # exact lattice: edge and corner neighbours touch in zero-area ties (A ~ 1e-33)
    for i in range(len(x)):
        real = [a for a in c.facets(i).values() if a > 1e-9 * h * h]
        assert len(real) == sum(1 for ax in (x, y, z) for s in (-h, h)
                                if 0 < ax[i] + s < 1)
        for a in real:
            assert a == pytest.approx(h * h, rel=1e-12)
    wall_total = c.walls.sum()
    assert wall_total == pytest.approx(6.0, rel=1e-12)


def test_random_sites_huge_weights_tile_box(oracle_mod):
    """Random sites and large random weights: an unrestricted power diagram of the box."""
    rng = np.random.default_rng(3)
    n = 40
    p = rng.uniform(0.05, 0.95, size=(n, 3))
    psi = 4.0 + rng.uniform(0, 0.02, size=n)
    c = oracle_mod.cells(p[:, 0], p[:, 1], p[:, 2], psi)
    assert c.V.sum() == pytest.approx(1.0, rel=1e-11)
    np.testing.assert_allclose(c.K, 0.0, atol=1e-11)
    assert c.walls.sum() == pytest.approx(6.0, rel=1e-11)
