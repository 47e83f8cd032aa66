"""Pins of the oracle's damped Newton solve (Alg. 1 with KMT step control).

  * one isolated ball: psi* = (3 nu / 4 pi)^(2/3) and the undamped trajectory
    psi_{k+1} = psi_k + (nu - V_k) / (2 pi sqrt(psi_k)) in closed form;
  * two overlapping balls: the lens/cap closed forms solved by scipy root finding;
  * the 1,000-site slab: convergence, total volume, KMT invariant, uniqueness of
    the weights from two different starts (the solution is unique, section 2.2)."""
import math

import numpy as np
import pytest
from scipy.optimize import fsolve

from paper_2601_05765_amd import scenes


def test_single_ball_closed_form(oracle_mod):
    nu = 3e-3
    psi0 = 0.8 * (3 * nu / (4 * math.pi)) ** (2 / 3)
    P = np.array([[0.5, 0.5, 0.5]])
    psi, st = oracle_mod.newton_solve(P, np.array([nu]), np.array([psi0]), tol=1e-13)
    assert st.status == "ok"
    assert psi[0] == pytest.approx((3 * nu / (4 * math.pi)) ** (2 / 3), rel=1e-12)
    # closed-form undamped trajectory
    p = psi0
    for h in st.history[1:]:
        assert h["alpha"] == 1.0
        V = 4 / 3 * math.pi * p ** 1.5
        p = p + (nu - V) / (2 * math.pi * math.sqrt(p))
        assert abs(4 / 3 * math.pi * p ** 1.5 - nu) / nu == pytest.approx(h["max_rel_err"], rel=1e-6, abs=1e-15)


def _cap(r, t):
    h = r + t
    return math.pi * h * h * (3 * r - h) / 3.0


def test_two_ball_solve_vs_root_finding(oracle_mod):
    d = 0.12
    nu = np.array([3.0e-3, 5.0e-3])
    P = np.array([[0.4, 0.5, 0.5], [0.4 + d, 0.5, 0.5]])

    def F(s):
        p1, p2 = s
        r1, r2 = math.sqrt(p1), math.sqrt(p2)
        t1 = (d * d + p1 - p2) / (2 * d)
        t2 = d - t1
        return [_cap(r1, t1) - nu[0], _cap(r2, t2) - nu[1]]

    ref = fsolve(F, [0.01, 0.012], xtol=1e-15)
    assert np.allclose(F(ref), 0, atol=1e-16)
    psi0 = scenes.default_psi0(nu)
    psi, st = oracle_mod.newton_solve(P, nu, psi0, tol=1e-12)
    assert st.status == "ok"
    np.testing.assert_allclose(psi, ref, rtol=1e-9)


@pytest.fixture(scope="module")
def slab_solution(oracle_mod):
    sc = scenes.slab_uniform(1000, 0)
    P = sc.xyz64()
    psi, st = oracle_mod.newton_solve(P, sc.nu, sc.psi0, tol=1e-5)
    return sc, P, psi, st


def test_slab_1k_converges(oracle_mod, slab_solution):
    sc, P, psi, st = slab_solution
    assert st.status == "ok" and st.max_rel_err <= 1e-5
    c = oracle_mod.cells(P[:, 0], P[:, 1], P[:, 2], psi)
    assert np.max(np.abs(c.V - sc.nu) / sc.nu) <= 1e-5
    assert c.V.sum() == pytest.approx(sc.nu.sum(), rel=1e-5)
    # KMT invariant: residual norm decreases monotonically along accepted iterates
    g = [h["gnorm"] for h in st.history]
    assert all(b < a for a, b in zip(g, g[1:]))


def test_slab_1k_unique_weights(oracle_mod, slab_solution):
    sc, P, psi, st = slab_solution
    psi_b, st_b = oracle_mod.newton_solve(P, sc.nu, scenes.default_psi0(sc.nu, 1.05), tol=1e-9)
    assert st_b.status == "ok"
    psi_a, st_a = oracle_mod.newton_solve(P, sc.nu, psi, tol=1e-9)
    assert st_a.status == "ok"
    np.testing.assert_allclose(psi_a, psi_b, rtol=1e-6)
