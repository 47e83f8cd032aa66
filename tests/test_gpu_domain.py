"""Cells and solves in convex polyhedral domains (lagot_set_domain) against the FP64
oracle, through the C-ABI. The planes are rounded to float32 before they are given to
both sides (the float32 values are the input, as for the positions)."""
import math
import sys

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

from parity import assert_close, compare

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


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def _f32_planes(planes):
    return np.asarray(planes, np.float32).astype(np.float64)


BOX = [[-1, 0, 0, 0], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]]
CUT = _f32_planes(BOX + [list(_unit([1, 1, 0])) + [float(_unit([1, 1, 0]) @ [0.62, 0.62, 0])],
                         list(_unit([0, -1, 1])) + [float(_unit([0, -1, 1]) @ [0, 0.35, 0.65])],
                         list(_unit([-1, 0.3, -1])) + [float(_unit([-1, 0.3, -1]) @ [0.3, 0.5, 0.2])]])


def _inside(P, planes):
    return np.all(P @ planes[:, :3].T < planes[:, 3] - 1e-6, axis=1)


def _dev(x, y, z, psi):
    import torch
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return t(x, torch.float32), t(y, torch.float32), t(z, torch.float32), t(psi, torch.float64)


@pytest.mark.parametrize("seed", range(4))
def test_domain_cells_parity(ctx, oracle_mod, seed):
    _say(f"case: cells in a cut box (9 planes), seed {seed}")
    sc = scenes.random_small(60, seed, r_lo=0.05, r_hi=0.2)
    P = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    keep = _inside(P, CUT)
    x, y, z, psi = sc.x[keep], sc.y[keep], sc.z[keep], sc.psi0[keep]
    ctx.set_domain(CUT)
    try:
        out = ctx.cells(*_dev(x, y, z, psi))
    finally:
        ctx.set_domain(None)
    orc = oracle_mod.cells(x, y, z, psi, domain=CUT)
    rep = compare(out, orc, psi)
    _say(f"  {keep.sum()} sites: {rep}")
    assert out["walls"].shape[1] == CUT.shape[0]
    assert_close(rep)


@pytest.mark.parametrize("seed", range(2))
def test_domain_paper_k_route(ctx, oracle_mod, seed):
    """lagot_cells_paper_k in the cut box: the domain planes are facets of the restricted
    cells like the box walls; K and V against the oracle's route and its signed form. The
    planes are the float32 values both sides are given, whose normals are unit only to
    1.7e-8; the two forms of K read a non-unit normal differently at that level (with the
    normals renormalised in float64 the oracle's two forms agree to 3e-16), hence 1e-7."""
    _say(f"case: paper K route in a cut box (9 planes), seed {seed}")
    sc = scenes.random_small(60, seed, r_lo=0.05, r_hi=0.2)
    P = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    keep = _inside(P, CUT)
    x, y, z, psi = sc.x[keep], sc.y[keep], sc.z[keep], sc.psi0[keep]
    ctx.set_domain(CUT)
    try:
        V, K = ctx.cells_paper_k(*_dev(x, y, z, psi))
    finally:
        ctx.set_domain(None)
    orc = oracle_mod.cells(x, y, z, psi, domain=CUT, paper_k=True)
    area = 4.0 * math.pi * psi
    eK = np.abs(K.cpu().numpy() - orc.Kp) / area
    eK2 = np.abs(orc.Kp - orc.K) / area
    eV = np.abs(V.cpu().numpy() - orc.V) / (area * np.sqrt(psi) / 3.0)
    _say(f"  {keep.sum()} sites: K vs oracle route {eK.max():.2e}, oracle routes {eK2.max():.2e}, V {eV.max():.2e}")
    assert eK.max() <= 1e-7 and eK2.max() <= 1e-7 and eV.max() <= 1e-7


def _tetra():
    v = np.array([[0.1, 0.1, 0.1], [0.9, 0.15, 0.1], [0.2, 0.85, 0.15], [0.3, 0.3, 0.9]])
    planes, areas = [], []
    for k in range(4):
        f = [v[i] for i in range(4) if i != k]
        n = np.cross(f[1] - f[0], f[2] - f[0])
        areas.append(0.5 * np.linalg.norm(n))
        n = _unit(n)
        if n @ (v[k] - f[0]) > 0:
            n = -n
        planes.append(list(n) + [float(n @ f[0])])
    return v, _f32_planes(planes), np.array(areas), abs(np.linalg.det(v[1:] - v[0])) / 6


def test_domain_tetrahedron_tiling(ctx):
    """Huge weights in a tetrahedron: volumes, wall areas and first moments add up to the
    tetrahedron's (float32 planes: to 1e-5)."""
    _say("case: tetrahedron tiled by 3000 cells")
    v, planes, areas, vol = _tetra()
    rng = np.random.default_rng(5)
    P = (rng.dirichlet(np.ones(4), size=3000) @ v).astype(np.float32)
    keep = _inside(P.astype(np.float64), planes)
    P = P[keep]
    psi = np.full(len(P), 0.01)
    ctx.set_domain(planes)
    try:
        out = ctx.cells(*_dev(P[:, 0], P[:, 1], P[:, 2], psi), csr=False)
        vol_g, cen = ctx.centroids(*_dev(P[:, 0], P[:, 1], P[:, 2], psi))
    finally:
        ctx.set_domain(None)
    V = out["vol"].cpu().numpy()
    assert V.sum() == pytest.approx(vol, rel=1e-5)
    assert np.allclose(out["walls"].cpu().numpy().sum(0), areas, rtol=1e-5)
    m = (vol_g.cpu().numpy()[:, None] * cen.cpu().numpy()).sum(0) / vol
    assert np.allclose(m, v.mean(0), atol=1e-5)


def test_domain_solve(ctx, oracle_mod):
    """A slab of sites in the unit box cut by a tilted plane: the solve converges and the
    oracle confirms every sampled volume."""
    _say("case: solve in a cut box")
    import paper_2601_05765_amd as L
    import torch
    planes = _f32_planes(BOX + [list(_unit([1, 0, 1])) + [float(_unit([1, 0, 1]) @ [1.0, 0, 0.2])]])
    sc = scenes.slab_uniform(3000, 8)
    P = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    keep = _inside(P, planes)
    x, y, z = sc.x[keep], sc.y[keep], sc.z[keep]
    n = int(keep.sum())
    nu = np.full(n, 0.25 / n)
    psi0 = scenes.default_psi0(nu)
    xd, yd, zd, pd = _dev(x, y, z, psi0)
    nud = torch.tensor(nu, device="cuda")
    ctx.set_domain(planes)
    try:
        st = ctx.solve(xd, yd, zd, nud, pd, opts=L.default_opts(tol=1e-5))
    finally:
        ctx.set_domain(None)
    _say(f"  {n} sites: {st.as_dict()}")
    assert st.status == 0 and st.max_rel_err <= 1e-5
    idx = np.sort(np.random.default_rng(3).choice(n, 400, replace=False))
    c = oracle_mod.cells(x, y, z, pd.cpu().numpy(), idx=idx, domain=planes)
    assert float(np.max(np.abs(c.V - nu[idx]) / nu[idx])) <= 1e-5


def test_domain_errors_and_reset(ctx):
    _say("case: domain errors, reset to the box")
    import paper_2601_05765_amd as L
    with pytest.raises(L.LagotError):
        ctx.set_domain([[1.0, 1.0, 0.0, 0.5]])  # normal not unit
    sc = scenes.random_small(20, 1)
    args = _dev(sc.x, sc.y, sc.z, sc.psi0)
    ref = ctx.cells(*args, csr=False)["vol"].cpu().numpy()
    ctx.set_domain(_f32_planes(BOX + [[0.0, 0.0, 1.0, 0.3]]))  # most sites lie above z = 0.3
    try:
        with pytest.raises(L.LagotError):
            ctx.cells(*args, csr=False)
    finally:
        ctx.set_domain(None)
    again = ctx.cells(*args, csr=False)["vol"].cpu().numpy()
    assert np.array_equal(ref, again)
    # the box as six planes gives the box's cells
    ctx.set_domain(_f32_planes(BOX))
    try:
        six = ctx.cells(*args, csr=False)["vol"].cpu().numpy()
    finally:
        ctx.set_domain(None)
    assert np.array_equal(ref, six)
