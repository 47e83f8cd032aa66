"""Pins of the oracle in convex polyhedral domains {x : n_w.x <= c_w} (the paper evaluates
its cells in polyhedral domains, section 6): closed forms for a tilted plane, the box
written as six planes, the tiling of a tetrahedron, and Monte Carlo in a cut box."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

from test_oracle_montecarlo import _uniform_ball


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


BOX_PLANES = np.array([[-1, 0, 0, 0], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]],
                      np.float64)


@pytest.mark.parametrize("normal", [(1, 1, 1), (1, -2, 0.5), (0, 0, 1)])
@pytest.mark.parametrize("a", [0.02, 0.09, 0.15])
def test_tilted_plane_cap(oracle_mod, normal, a):
    """Ball of radius 0.2 whose centre is at distance a from one tilted wall: the cell is the
    ball minus a cap of height r - a; wall area pi (r^2 - a^2); spherical area 4 pi r^2 -
    2 pi r (r - a); centroid moved against the normal by V_cap z_cap / V."""
    r = 0.2
    n = _unit(normal)
    p = np.array([0.5, 0.5, 0.5])
    dom = np.vstack([BOX_PLANES, np.concatenate([n, [n @ p + a]])])
    c = oracle_mod.cells(p[0:1], p[1:2], p[2:3], np.array([r * r]), domain=dom)
    h = r - a
    vcap = math.pi * h * h * (3 * r - h) / 3
    zc = 3 * (2 * r - h) ** 2 / (4 * (3 * r - h))
    V = 4 / 3 * math.pi * r ** 3 - vcap
    assert c.V[0] == pytest.approx(V, rel=1e-12)
    assert c.walls[0, 6] == pytest.approx(math.pi * (r * r - a * a), rel=1e-12)
    assert np.allclose(c.walls[0, :6], 0.0)
    assert c.K[0] == pytest.approx(4 * math.pi * r * r - 2 * math.pi * r * h, rel=1e-12)
    assert np.allclose(c.C[0], p - n * vcap * zc / V, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 2])
def test_box_as_six_planes(oracle_mod, seed):
    sc = scenes.random_small(25, seed)
    a = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0)
    b = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0, domain=BOX_PLANES)
    assert np.allclose(a.V, b.V, rtol=1e-13, atol=1e-16)
    assert np.allclose(a.K, b.K, rtol=1e-12, atol=1e-15)
    assert np.allclose(a.walls, b.walls, rtol=1e-12, atol=1e-15)
    assert np.array_equal(a.fcount, b.fcount)
    assert np.allclose(a.C, b.C, atol=1e-13)


def _tetra():
    v = np.array([[0.1, 0.1, 0.1], [0.9, 0.15, 0.1], [0.2, 0.85, 0.15], [0.3, 0.3, 0.9]])
    planes, areas = [], []
    for k in range(4):
        f = [v[i] for i in range(4) if i != k]
        n = np.cross(f[1] - f[0], f[2] - f[0])
        area = 0.5 * np.linalg.norm(n)
        n = _unit(n)
        if n @ (v[k] - f[0]) > 0:
            n = -n
        planes.append(np.concatenate([n, [n @ f[0]]]))
        areas.append(area)
    vol = abs(np.linalg.det(v[1:] - v[0])) / 6
    return v, np.array(planes), np.array(areas), vol


def test_tetrahedron_tiling(oracle_mod):
    """Huge weights: the cells tile the tetrahedron, so their volumes, first moments and
    wall areas add up to the tetrahedron's volume, centroid and face areas."""
    v, planes, areas, vol = _tetra()
    rng = np.random.default_rng(4)
    w = rng.dirichlet(np.ones(4), size=60)
    P = w @ v
    psi = np.full(len(P), 4.0) + rng.uniform(0, 1e-3, len(P))
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi, domain=planes)
    assert c.V.sum() == pytest.approx(vol, rel=1e-12)
    assert np.allclose((c.V[:, None] * c.C).sum(0) / vol, v.mean(0), atol=1e-12)
    assert np.allclose(c.walls.sum(0), areas, rtol=1e-11)


@pytest.mark.parametrize("seed", [1, 4])
def test_mc_cut_box(oracle_mod, seed):
    """Random overlapping balls in the box cut by two tilted planes: Monte Carlo of eq. (1)
    membership with the domain test."""
    sc = scenes.random_small(10, seed)
    P = sc.xyz64()
    psi = sc.psi0
    extra = np.array([np.concatenate([_unit([1, 1, 0]), [_unit([1, 1, 0]) @ [0.62, 0.62, 0]]]),
                      np.concatenate([_unit([0, -1, 1]), [_unit([0, -1, 1]) @ [0, 0.35, 0.65]]])])
    dom = np.vstack([BOX_PLANES, extra])
    inside = np.all(P @ dom[:, :3].T < dom[:, 3], axis=1)
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi, domain=dom)
    rng = np.random.default_rng(200 + seed)
    m = 300_000
    for i in range(len(P)):
        if not inside[i]:
            continue
        r = math.sqrt(psi[i])
        pts = P[i] + _uniform_ball(rng, m, r)
        d_i = ((pts - P[i]) ** 2).sum(1) - psi[i]
        ok = np.all(pts @ dom[:, :3].T <= dom[:, 3], axis=1) & (d_i <= 0)
        for j in range(len(P)):
            if j != i:
                ok &= d_i <= ((pts - P[j]) ** 2).sum(1) - psi[j]
        f = ok.mean()
        Vb = 4 / 3 * math.pi * r ** 3
        sig = Vb * math.sqrt(max(f * (1 - f), 1e-12) / m)
        assert abs(c.V[i] - f * Vb) <= 5 * sig + 1e-12, (i, c.V[i], f * Vb)
