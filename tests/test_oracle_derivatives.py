"""Pins of the gradient/Hessian formulas (section 3.1, eq. (2)) through finite
differences of the oracle's own volumes.

  dV_i/dpsi_j = -A_ij / (2 |p_j - p_i|)                        (j != i)
  dV_i/dpsi_i =  sum_j A_ij / (2 |p_j - p_i|) + K_i / (2 sqrt(psi_i))
  sum_j dV_i/dpsi_j = K_i / (2 sqrt(psi_i))   (shifting every weight moves no
                                                bisector, only the balls grow)
A wrong facet area, a dropped spherical term or a missing factor 1/2 in any of
them breaks one of these identities, because V is pinned independently by the
closed-form and Monte Carlo tests."""
import math

import numpy as np
import pytest

from paper_2601_05765_amd import scenes


def _vols(oracle_mod, P, psi):
    return oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi).V


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_fd_hessian(oracle_mod, seed):
    sc = scenes.random_small(9, seed, r_lo=0.1, r_hi=0.22)
    P, psi = sc.xyz64(), sc.psi0
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    n = len(P)
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * psi[j]
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (_vols(oracle_mod, P, psi + e) - _vols(oracle_mod, P, psi - e)) / (2 * h)
    for i in range(n):
        r = math.sqrt(psi[i])
        f = c.facets(i)
        diag = c.K[i] / (2 * r)
        for j in range(n):
            if j == i:
                continue
            d = np.linalg.norm(P[j] - P[i])
            w = f.get(j, 0.0) / (2 * d)
            diag += w
            assert J[i, j] == pytest.approx(-w, abs=1e-6 * (abs(w) + 1e-3))
        assert J[i, i] == pytest.approx(diag, rel=1e-6)
        assert J[i].sum() == pytest.approx(c.K[i] / (2 * r), abs=1e-6 * (abs(diag) + 1e-3))


def test_hessian_assembly_matches_fd_and_is_spd(oracle_mod):
    sc = scenes.random_small(9, 21, r_lo=0.1, r_hi=0.22)
    P, psi = sc.xyz64(), sc.psi0
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    H, diag = oracle_mod.hessian(P, psi, c)
    Hd = H.toarray()
    n = len(P)
    J = np.zeros((n, n))
    for j in range(n):
        h = 1e-6 * psi[j]
        e = np.zeros(n)
        e[j] = h
        J[:, j] = (_vols(oracle_mod, P, psi + e) - _vols(oracle_mod, P, psi - e)) / (2 * h)
    np.testing.assert_allclose(Hd, J, atol=1e-6 * np.abs(J).max())
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-14)
    assert np.linalg.eigvalsh(Hd).min() > 0
    # row sums of -Hess K equal the spherical term K_i / (2 r_i)
    np.testing.assert_allclose(Hd.sum(1), c.K / (2 * np.sqrt(psi)), rtol=1e-10, atol=1e-14)


def test_walls_do_not_enter_hessian(oracle_mod):
    """A ball cut by a wall: dV/dpsi has only the spherical term (the wall does not move)."""
    r, a = 0.1, 0.04
    P = np.array([[a, 0.5, 0.5]])
    psi = np.array([r * r])
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    h = 1e-7 * psi[0]
    fd = (_vols(oracle_mod, P, psi + h) - _vols(oracle_mod, P, psi - h))[0] / (2 * h)
    assert fd == pytest.approx(c.K[0] / (2 * r), rel=1e-7)
    H, _ = oracle_mod.hessian(P, psi, c)
    assert H.toarray()[0, 0] == pytest.approx(c.K[0] / (2 * r), rel=1e-13)
