"""Pins of the oracle's cells in a non-convex domain given as convex pieces (section 6
evaluates cells in polyhedral domains; ``oracle.cells_pieces`` sums each measure of the
restricted cell over its parts in the pieces).

What pins it: a convex box cut into pieces gives the box's own cells (every output,
including sites that lie outside a piece); two different decompositions of the same
L-shaped prism agree; a ball reaching across the prism's re-entrant edge (its volume and
sphere area against quadratures of the removed wedge, circular segments on the two
re-entrant walls) and a ball that crosses only a plane between pieces (whole); and
tilings whose volumes, wall areas and first moments add up to the domain's. A site
must not lie on a plane of a piece (there the facet's solid angle depends on the side
it is approached from), so every site here lies off the planes."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes


def _halves():
    """The unit box as two pieces split at x = 0.6 (walls 0..5 = -x, +x, -y, +y, -z, +z)."""
    left = (np.array([[-1, 0, 0, 0], [1, 0, 0, 0.6], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]],
                     np.float64), [0, -1, 2, 3, 4, 5])
    right = (np.array([[-1, 0, 0, -0.6], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]],
                      np.float64), [-1, 1, 2, 3, 4, 5])
    return [left, right]


def _same(a, b, psi, tol=1e-12):
    r = np.sqrt(psi)
    ball = 4.0 / 3.0 * math.pi * r ** 3
    assert np.all(np.abs(a.V - b.V) <= tol * ball)
    assert np.all(np.abs(a.K - b.K) <= tol * 4 * math.pi * psi)
    assert np.all(np.abs(a.walls - b.walls) <= tol * math.pi * psi[:, None])
    assert np.all(np.abs(a.C - b.C) <= tol * np.maximum(1.0, r[:, None]))
    for i in range(len(psi)):
        # the same neighbours and areas; a facet may be present on one side only as a
        # rounding-level sliver (area ~1e-19: where its planes meet at a vertex)
        fa, fb = a.facets(i), b.facets(i)
        disk = math.pi * psi[i]
        for j in set(fa) | set(fb):
            assert abs(fa.get(j, 0.0) - fb.get(j, 0.0)) <= tol * disk, (i, j)
            if (j in fa) != (j in fb):
                assert max(fa.get(j, 0.0), fb.get(j, 0.0)) <= 1e-15 * disk, (i, j)


@pytest.mark.parametrize("seed", range(3))
def test_box_split_in_two_is_the_box(oracle_mod, seed):
    """A site in the right half lies outside the left piece (behind its plane at x = 0.6,
    or beyond its ball's reach): its left part must come out exactly as the box clip
    does, so the sums reproduce the box's cells."""
    sc = scenes.random_small(150, seed, lo=0.05, hi=0.95, r_lo=0.05, r_hi=0.25)
    whole = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0)
    parts = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, _halves(), 6)
    # some balls straddle the cut, some lie wholly on one side
    straddle = np.abs(sc.x.astype(np.float64) - 0.6) < np.sqrt(sc.psi0)
    assert straddle.sum() >= 20 and (~straddle).sum() >= 20
    _same(parts, whole, sc.psi0)


def test_two_decompositions_of_the_l_prism_agree(oracle_mod):
    sc = scenes.l_shape_sites(250, 3, spread=0.4)
    a = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, scenes.l_shape_pieces(), scenes.L_WALLS)
    b = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, scenes.l_shape_pieces(split_z=True), scenes.L_WALLS)
    _same(a, b, sc.psi0)
    # the re-entrant walls are reached by some cells
    assert (a.walls[:, 6] > 0).sum() >= 3 and (a.walls[:, 7] > 0).sum() >= 3


def _removed_wedge(r, a, b):
    """Volume and sphere area of a ball of radius r (centre at the origin) in the wedge
    {x > a, y > b} (a, b >= 0), by quadrature over z: the disk of radius rho(z) meets the
    wedge in the area under sqrt(rho^2 - x^2) - b for x in (a, rho); the sphere's ring at
    height z (area 2 pi r dz, Archimedes) lies in the wedge along the arc between the
    angles asin(b / rho) and acos(a / rho)."""
    from scipy.integrate import quad

    def disk_part(z):
        rho2 = r * r - z * z
        if a * a + b * b >= rho2:
            return 0.0
        return quad(lambda x: max(math.sqrt(max(rho2 - x * x, 0.0)) - b, 0.0), a, math.sqrt(rho2),
                    epsabs=0, epsrel=1e-13, limit=200)[0]

    def arc(z):
        rho = math.sqrt(r * r - z * z)
        if a * a + b * b >= rho * rho:
            return 0.0
        return max(math.acos(a / rho) - math.asin(b / rho), 0.0)

    zmax = math.sqrt(r * r - a * a - b * b)
    vol = quad(disk_part, -zmax, zmax, epsabs=0, epsrel=1e-12, limit=200)[0]
    area = r * quad(arc, -zmax, zmax, epsabs=0, epsrel=1e-12, limit=200)[0]
    return vol, area


@pytest.mark.parametrize("split_z", [False, True])
def test_ball_across_the_reentrant_edge(oracle_mod, split_z):
    """One ball of radius 0.2 centred at (0.45, 0.45, 0.5), inside the first piece and 0.05
    from the two planes it shares with the others: the ball reaches both other pieces (the
    site lies outside them) and the removed quarter {x > 1/2, y > 1/2}. V and K are the
    ball's less the removed wedge's (quadrature); each re-entrant wall holds the circular
    segment of the ball's section beyond the edge, R^2 acos(d / R) - d sqrt(R^2 - d^2) with
    R^2 = r^2 - d^2, d = 0.05; no other wall is reached."""
    r, d = 0.2, 0.05
    c = oracle_mod.cells_pieces(np.array([0.5 - d]), np.array([0.5 - d]), np.array([0.5]), np.array([r * r]),
                                scenes.l_shape_pieces(split_z), scenes.L_WALLS)
    v_cut, k_cut = _removed_wedge(r, d, d)
    assert c.V[0] == pytest.approx(4.0 / 3.0 * math.pi * r ** 3 - v_cut, rel=1e-10)
    assert c.K[0] == pytest.approx(4.0 * math.pi * r * r - k_cut, rel=1e-10)
    R2 = r * r - d * d
    seg = R2 * math.acos(d / math.sqrt(R2)) - d * math.sqrt(R2 - d * d)
    w = c.walls[0]
    assert w[6] == pytest.approx(seg, rel=1e-12)
    assert w[7] == pytest.approx(seg, rel=1e-12)
    assert np.all(np.delete(w, [6, 7]) == 0.0)


def test_ball_across_a_plane_between_pieces(oracle_mod):
    """A ball that crosses only a plane between two pieces (x = 1/2 at y < 1/2) is whole:
    V, K and the centroid of the free ball, no wall area."""
    r = 0.15
    c = oracle_mod.cells_pieces(np.array([0.47]), np.array([0.25]), np.array([0.5]), np.array([r * r]),
                                scenes.l_shape_pieces(True), scenes.L_WALLS)
    assert c.V[0] == pytest.approx(4.0 / 3.0 * math.pi * r ** 3, rel=1e-12)
    assert c.K[0] == pytest.approx(4.0 * math.pi * r * r, rel=1e-12)
    assert np.allclose(c.C[0], [0.47, 0.25, 0.5], rtol=0, atol=1e-13)
    assert np.all(c.walls[0] == 0.0)


def test_l_prism_tiling(oracle_mod):
    """Huge weights: the cells tile the prism; volumes and the areas on each wall add up
    to the prism's (the re-entrant walls included, the planes between pieces excluded)."""
    sc = scenes.l_shape_sites(120, 7)
    psi = np.full(sc.n, 4.0)
    c = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, psi, scenes.l_shape_pieces(split_z=True), scenes.L_WALLS)
    assert c.V.sum() == pytest.approx(scenes.L_VOLUME, rel=1e-12)
    assert np.allclose(c.walls.sum(0), scenes.L_WALL_AREAS, rtol=1e-12)
    assert np.all(np.abs(c.K) <= 1e-12 * 4 * math.pi * psi)  # no free surface (up to rounding)
    # first moment of the prism: the unit box's less the removed quarter's
    m = (c.V[:, None] * c.C).sum(0)
    assert np.allclose(m, 1.0 * np.array([0.5, 0.5, 0.5]) - 0.25 * np.array([0.75, 0.75, 0.5]), atol=1e-12)


# ---- the position update in a non-convex domain (fluid step) ----

M = 1e-6  # the plane margin of the unit box: max(1e-6 x extent, 4 float32 spacings at 1)


def _adv(p, pieces=None, domain=None):
    import oracle
    p = np.asarray(p, np.float32).reshape(-1, 3)
    return oracle.advect(p, np.zeros((len(p), 3)), 0.0, pieces=pieces, domain=domain).astype(np.float64)


def test_advect_one_piece_is_the_convex_rule(oracle_mod):
    planes = np.array([[-1, 0, 0, 0], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0],
                       [0, 0, 1, 1], [0.6, 0.0, 0.8, 0.7]], np.float64)
    rng = np.random.default_rng(2)
    p = rng.uniform(0.0, 1.0, (500, 3)).astype(np.float32)
    v = rng.normal(size=(500, 3))
    a = oracle_mod.advect(p, v, 0.05, domain=planes)
    b = oracle_mod.advect(p, v, 0.05, pieces=[(planes, list(range(7)))])
    assert np.array_equal(a, b)
    assert (np.abs(a.astype(np.float64) - (p + 0.05 * v)).max(axis=1) > 1e-6).sum() > 50


def test_advect_sites_inside_pieces_stay(oracle_mod):
    sc = scenes.l_shape_sites(400, 5)
    p = np.stack([sc.x, sc.y, sc.z], 1)
    inner = np.all(np.abs(p.astype(np.float64) - 0.5) > 1e-3, axis=1) & np.all((p > 1e-3) & (p < 1 - 1e-3), axis=1)
    out = _adv(p[inner], pieces=scenes.l_shape_pieces(True))
    assert np.array_equal(out, p[inner].astype(np.float64))


@pytest.mark.parametrize("site,axis", [((0.6, 0.55, 0.45), 1), ((0.52, 0.7, 0.45), 0), ((0.6, 0.6, 0.45), 1)])
def test_advect_into_the_nearest_piece(oracle_mod, site, axis):
    """A site in the removed quarter of the L prism moves onto the nearer re-entrant wall,
    the margin inside: (0.6, 0.55) to y = 1/2 - m (piece 1), (0.52, 0.7) to x = 1/2 - m
    (piece 2), and (0.6, 0.6), as near to both, to the first of them (piece 1)."""
    for split in (False, True):
        q = _adv(site, pieces=scenes.l_shape_pieces(split))[0]
        want = np.array(site, np.float32).astype(np.float64)
        want[axis] = 0.5 - M
        assert np.all(np.abs(q - want) <= 6e-8), (split, q, want)


def test_paper_k_route_summed_over_pieces(oracle_mod):
    """The second |K| route (section 3.3), run in each piece and summed, agrees with the
    signed solid-angle form summed the same way (1e-10 of 4 pi r^2), in the L prism and
    for the box split in two (where it also equals the box's own route)."""
    sc = scenes.l_shape_sites(300, 9, spread=0.3)
    c = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, scenes.l_shape_pieces(True), scenes.L_WALLS,
                                paper_k=True)
    assert np.max(np.abs(c.Kp - c.K) / (4 * math.pi * sc.psi0)) <= 1e-10
    sb = scenes.random_small(120, 4, lo=0.05, hi=0.95, r_lo=0.05, r_hi=0.25)
    h = oracle_mod.cells_pieces(sb.x, sb.y, sb.z, sb.psi0, _halves(), 6, paper_k=True)
    w = oracle_mod.cells(sb.x, sb.y, sb.z, sb.psi0, paper_k=True)
    assert np.max(np.abs(h.Kp - w.Kp) / (4 * math.pi * sb.psi0)) <= 1e-10
