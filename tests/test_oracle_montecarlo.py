"""Monte Carlo pins of the oracle (volumes, facet areas, spherical areas).

The sampler below evaluates the membership test of eq. (1) point by point; it
shares nothing with the oracle's polytope clipping or fan integration. Tiny random
configurations with overlapping balls and nearby walls (N <= 12)."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

BOX = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])


def _member(pts, i, P, psi):
    """Mask of points that belong to C_i per eq. (1): inside the box, inside ball i,
    and power(i) <= power(j) for every j."""
    d_i = ((pts - P[i]) ** 2).sum(1) - psi[i]
    ok = (d_i <= 0) & np.all((pts >= BOX[0]) & (pts <= BOX[1]), axis=1)
    for j in range(len(P)):
        if j != i:
            ok &= d_i <= ((pts - P[j]) ** 2).sum(1) - psi[j]
    return ok


def _uniform_ball(rng, m, r):
    v = rng.normal(size=(m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * (r * rng.uniform(size=(m, 1)) ** (1 / 3))


def _uniform_sphere(rng, m, r):
    v = rng.normal(size=(m, 3))
    return r * v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_mc_volume_sphere_area(oracle_mod, seed):
    sc = scenes.random_small(10, seed)
    P = sc.xyz64()
    psi = sc.psi0
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    rng = np.random.default_rng(100 + seed)
    m = 400_000
    for i in range(len(P)):
        r = math.sqrt(psi[i])
        f = _member(P[i] + _uniform_ball(rng, m, r), i, P, psi).mean()
        Vb = 4 / 3 * math.pi * r ** 3
        sig = Vb * math.sqrt(max(f * (1 - f), 1e-12) / m)
        assert abs(c.V[i] - f * Vb) <= 5 * sig + 1e-12, (i, c.V[i], f * Vb)
        # spherical area: fraction of the sphere inside all half-spaces and the box
        s = P[i] + _uniform_sphere(rng, m, r)
        keep = np.all((s >= BOX[0]) & (s <= BOX[1]), axis=1)
        d_i = ((s - P[i]) ** 2).sum(1) - psi[i]  # == 0 on the sphere (up to rounding)
        for j in range(len(P)):
            if j != i:
                keep &= d_i <= ((s - P[j]) ** 2).sum(1) - psi[j]
        g = keep.mean()
        Ks = 4 * math.pi * r * r
        sigK = Ks * math.sqrt(max(g * (1 - g), 1e-12) / m)
        assert abs(c.K[i] - g * Ks) <= 5 * sigK + 1e-12, (i, c.K[i], g * Ks)


@pytest.mark.parametrize("seed", [5, 6])
def test_mc_facet_areas(oracle_mod, seed):
    """Facet (i,j): sample the disk where the radical plane meets ball i and test eq. (1)
    against every other site; the shared facet is seen identically from i and j."""
    sc = scenes.random_small(8, seed, r_lo=0.12, r_hi=0.25)
    P = sc.xyz64()
    psi = sc.psi0
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    rng = np.random.default_rng(seed)
    m = 300_000
    checked = 0
    for i in range(len(P)):
        r = math.sqrt(psi[i])
        for j in range(len(P)):
            if j == i:
                continue
            dv = P[j] - P[i]
            d = np.linalg.norm(dv)
            t = (d * d + psi[i] - psi[j]) / (2 * d)
            if not (-r < t < r):
                assert j not in c.facets(i)
                continue
            n = dv / d
            rho = math.sqrt(r * r - t * t)
            e1 = np.cross(n, [1.0, 0, 0] if abs(n[0]) < 0.9 else [0, 1.0, 0])
            e1 /= np.linalg.norm(e1)
            e2 = np.cross(n, e1)
            rad = rho * np.sqrt(rng.uniform(size=m))
            th = rng.uniform(0, 2 * math.pi, size=m)
            pts = P[i] + t * n + (rad * np.cos(th))[:, None] * e1 + (rad * np.sin(th))[:, None] * e2
            ok = np.all((pts >= BOX[0]) & (pts <= BOX[1]), axis=1)
            pw = ((pts - P[i]) ** 2).sum(1) - psi[i]
            for k in range(len(P)):
                if k != i and k != j:
                    ok &= pw <= ((pts - P[k]) ** 2).sum(1) - psi[k]
            f = ok.mean()
            D = math.pi * rho * rho
            sig = D * math.sqrt(max(f * (1 - f), 1e-12) / m)
            a = c.facets(i).get(j, 0.0)
            assert abs(a - f * D) <= 5 * sig + 1e-12, (i, j, a, f * D)
            if a > 0:
                assert c.facets(j)[i] == pytest.approx(a, rel=1e-10)
                checked += 1
    assert checked >= 4
