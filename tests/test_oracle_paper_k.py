"""Pins of the oracle's second route to the spherical area |K_i| (section 3.3 and
Algorithm 2: an interior point c from rays cast from the restricted facets, each facet
projected from c onto the sphere, the projected areas by Gauss-Bonnet with the geodesic
curvature read as k_g = e / (r rho)).

The two routes share nothing but the clipped face polygons: the signed solid angles at
p_i (``K``) against the projections from an off-centre point with circle arcs, corner
turning angles and geodesic curvatures (``Kp``). Their agreement on crowded cells, on
cells whose site lies outside its own cell, and on cells cut by the box walls pins both;
closed forms (caps, the lens of two balls, the free ball) and the position of c (inside
the restricted cell) pin the route on its own."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes


def _k_scale(psi):
    return 4.0 * math.pi * np.asarray(psi)


@pytest.mark.parametrize("make", [lambda: scenes.slab_uniform(1000, 0),
                                  lambda: scenes.overpacked_sphere(2500, 1.72, 0),
                                  lambda: scenes.dam_break(1500, 2)])
def test_route_matches_signed_solid_angles(oracle_mod, make):
    sc = make()
    c = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0, paper_k=True)
    err = np.abs(c.Kp - c.K) / _k_scale(sc.psi0)
    assert err.max() <= 1e-10, (err.max(), int(np.argmax(err)))


def test_route_on_sites_outside_their_cells(oracle_mod):
    """Heavy random weights: many sites lie outside their own (non-empty) cells, where
    the signed form subtracts solid angles of facets with t < 0 and the paper's route
    projects from an interior point instead."""
    rng = np.random.default_rng(4)
    n = 400
    xyz = rng.uniform(0.1, 0.9, (n, 3))
    psi = (rng.uniform(0.02, 0.12, n)) ** 2
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], psi, paper_k=True)
    live = c.V > 0
    outside = np.zeros(n, bool)
    for i in np.flatnonzero(live):
        pw = np.sum((xyz - xyz[i]) ** 2, 1) - psi
        pw[i] = np.inf
        outside[i] = (pw < -psi[i]).any()  # p_i is closer (in power) to another site
    assert outside.sum() >= 10
    err = np.abs(c.Kp - c.K) / _k_scale(psi)
    assert err.max() <= 1e-10


@pytest.mark.parametrize("t", [-0.07, 0.0, 0.05, 0.09])
def test_single_plane_cap(oracle_mod, t):
    """A ball of radius 0.1 cut by one bisector at offset t: the remaining sphere is the
    cap of area 2 pi r (r + t)."""
    r = 0.1
    d = 0.06
    # two sites at distance d: t = (d^2 + psi_i - psi_j) / (2 d)
    psi_i = r * r
    psi_j = d * d + psi_i - 2.0 * d * t
    xyz = np.array([[0.5, 0.5, 0.5], [0.5 + d, 0.5, 0.5]])
    c = oracle_mod.cells(xyz[:, 0], xyz[:, 1], xyz[:, 2], np.array([psi_i, psi_j]), idx=[0], paper_k=True)
    assert c.Kp[0] == pytest.approx(2.0 * math.pi * r * (r + t), rel=1e-12, abs=1e-15)


def test_free_ball_and_wall_cap(oracle_mod):
    """A ball with no neighbour and no wall inside it has no facet: K = 4 pi r^2. The
    same ball moved so that one box wall cuts it at distance h from the centre keeps
    the cap 2 pi r (r + h), its facet a full circle (the whole disk inside the wall)."""
    r = 0.1
    c = oracle_mod.cells(np.array([0.5]), np.array([0.5]), np.array([0.5]), np.array([r * r]), paper_k=True)
    assert c.Kp[0] == pytest.approx(4.0 * math.pi * r * r, rel=1e-14)
    h = 0.04
    c = oracle_mod.cells(np.array([h]), np.array([0.5]), np.array([0.5]), np.array([r * r]), paper_k=True)
    assert c.Kp[0] == pytest.approx(2.0 * math.pi * r * (r + h), rel=1e-12)


def test_corner_of_the_box(oracle_mod):
    """A ball at a corner of the box, cut by three orthogonal walls through its centre:
    one eighth of the sphere remains."""
    r = 0.2
    c = oracle_mod.cells(np.array([0.0]), np.array([0.0]), np.array([0.0]), np.array([r * r]), paper_k=True)
    assert c.Kp[0] == pytest.approx(4.0 * math.pi * r * r / 8.0, rel=1e-12)


def test_interior_point_is_inside_the_restricted_cell(oracle_mod):
    """point_in: c lies in the ball, in the box and on the site's side of every
    bisector (brute force over all sites)."""
    sc = scenes.overpacked_sphere(800, 1.72, 1)
    xyz = sc.xyz64()
    c = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0, paper_k=True)
    psi = sc.psi0
    for i in np.flatnonzero(c.V > 1e-3 * np.pi * psi ** 1.5):
        p = c.cin[i]
        assert np.sum((p - xyz[i]) ** 2) < psi[i]
        assert (p > 0).all() and (p < 1).all()
        pw = np.sum((xyz - p) ** 2, 1) - psi
        assert pw[i] < np.delete(pw, i).min()
