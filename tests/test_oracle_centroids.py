"""Pins of the oracle's cell centroids (the centroid of the pressure model, section 5),
against closed forms, the tiling invariant and Monte Carlo.

The oracle computes the first moment from facet data by the divergence theorem; the pins
below use only elementary solids (ball, spherical cap), the box's own centroid, or a
point-membership sampler of eq. (1)."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

from test_oracle_montecarlo import BOX, _member, _uniform_ball


def _cap(r, h):
    """Volume of a spherical cap of height h and the distance of its centroid from the
    ball centre."""
    v = math.pi * h * h * (3 * r - h) / 3
    zc = 3 * (2 * r - h) ** 2 / (4 * (3 * r - h))
    return v, zc


def test_isolated_ball_centroid_is_the_site(oracle_mod):
    c = oracle_mod.cells(np.array([0.31]), np.array([0.47]), np.array([0.52]), np.array([0.1 ** 2]))
    assert np.allclose(c.C[0], [0.31, 0.47, 0.52], atol=1e-15)


@pytest.mark.parametrize("wall", range(6))
@pytest.mark.parametrize("a", [0.0, 0.03, 0.11, 0.17])
def test_ball_cut_by_one_wall(oracle_mod, wall, a):
    """Ball of radius 0.2 at distance a from one wall: the cell is the ball minus a cap of
    height r - a; its centroid moves away from the wall by V_cap z_cap / (V_ball - V_cap)."""
    r = 0.2
    ax, hi = wall // 2, wall % 2
    p = np.full(3, 0.5)
    p[ax] = (1.0 - a) if hi else a
    if a == 0.0:
        p[ax] = (1.0 - 1e-12) if hi else 1e-12
        a = 1e-12
    c = oracle_mod.cells(p[0:1], p[1:2], p[2:3], np.array([r * r]))
    vcap, zc = _cap(r, r - a)
    shift = vcap * (zc - 0.0) / (4 / 3 * math.pi * r ** 3 - vcap)
    want = p.copy()
    want[ax] += -shift if hi else shift
    assert np.allclose(c.C[0], want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("r1,r2,d", [(0.1, 0.1, 0.12), (0.1, 0.13, 0.15), (0.05, 0.14, 0.12)])
def test_two_balls_lens(oracle_mod, r1, r2, d):
    """Two overlapping balls: each cell is its ball minus the cap beyond the radical plane
    (distance t = (d^2 + r_i^2 - r_j^2) / 2d from the centre), when t > -r_i."""
    x = np.array([0.4, 0.4 + d])
    y = np.array([0.5, 0.5])
    z = np.array([0.5, 0.5])
    psi = np.array([r1 * r1, r2 * r2])
    c = oracle_mod.cells(x, y, z, psi)
    for i, (ri, rj, sgn) in enumerate([(r1, r2, 1.0), (r2, r1, -1.0)]):
        t = (d * d + ri * ri - rj * rj) / (2 * d)
        vcap, zc = _cap(ri, ri - t)
        vb = 4 / 3 * math.pi * ri ** 3
        shift = -sgn * vcap * zc / (vb - vcap)  # away from the other site
        assert c.C[i][0] == pytest.approx(x[i] + shift, abs=1e-12)
        assert c.C[i][1] == pytest.approx(0.5, abs=1e-14) and c.C[i][2] == pytest.approx(0.5, abs=1e-14)


@pytest.mark.parametrize("seed", [0, 1])
def test_tiling_first_moments_sum_to_the_box(oracle_mod, seed):
    """Huge weights: the cells tile the unit box, so sum_i V_i c_i is the box's first
    moment (1/2, 1/2, 1/2)."""
    rng = np.random.default_rng(seed)
    n = 40
    P = rng.uniform(0.05, 0.95, size=(n, 3))
    psi = 9.0 + rng.uniform(0.0, 0.01, size=n)
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    assert c.V.sum() == pytest.approx(1.0, abs=1e-12)
    assert np.allclose((c.V[:, None] * c.C).sum(0), [0.5, 0.5, 0.5], atol=1e-12)


@pytest.mark.parametrize("seed", [1, 3])
def test_mc_centroids(oracle_mod, seed):
    """Monte Carlo mean of uniform points of each cell (eq. (1) membership)."""
    sc = scenes.random_small(10, seed)
    P = sc.xyz64()
    psi = sc.psi0
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    rng = np.random.default_rng(300 + seed)
    m = 400_000
    for i in range(len(P)):
        r = math.sqrt(psi[i])
        pts = P[i] + _uniform_ball(rng, m, r)
        inside = _member(pts, i, P, psi)
        k = int(inside.sum())
        if k < 1000:
            continue
        mean = pts[inside].mean(0)
        sd = pts[inside].std(0) / math.sqrt(k)
        assert np.all(np.abs(c.C[i] - mean) <= 5 * sd + 1e-12), (i, c.C[i], mean, sd)
