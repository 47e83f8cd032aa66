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


# ---- non-convex domains: unions of convex pieces (lagot_set_domain_pieces) ----

def _halves():
    """The unit box as two pieces split at x = 0.6 (walls 0..5 = -x, +x, -y, +y, -z, +z)."""
    left = (np.array([[-1, 0, 0, 0], [1, 0, 0, 0.6], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]],
                     np.float64), [0, -1, 2, 3, 4, 5])
    right = (np.array([[-1, 0, 0, -0.6], [1, 0, 0, 1], [0, -1, 0, 0], [0, 1, 0, 1], [0, 0, -1, 0], [0, 0, 1, 1]],
                      np.float64), [-1, 1, 2, 3, 4, 5])
    return [(_f32_planes(p), w) for p, w in (left, right)]


@pytest.mark.parametrize("case,split_z", [("uniform", False), ("uniform", True), ("crowded", False)])
def test_l_prism_cells_parity(ctx, oracle_mod, case, split_z):
    """Every cell in the L-shaped prism (3 or 6 pieces) against the oracle: V, K, facet
    areas and connectivity, the 8 walls (re-entrant ones included) and the first moments
    about the sites (on the ball's scale, r times its volume, like the volumes: the
    centroid of a cell empty up to rounding is 0/0). 'crowded' is the over-packed sphere
    next to the planes between pieces, whose cells go through the crowded pass."""
    _say(f"case: cells in the L prism, {6 if split_z else 3} pieces, {case} sites")
    sc = scenes.l_shape_sites(1500, 11) if case == "uniform" else scenes.l_shape_crowded(2500, 0)
    pieces = scenes.l_shape_pieces(split_z)
    args = _dev(sc.x, sc.y, sc.z, sc.psi0)
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        # the first evaluation with crowded cells announces them (they finish on the
        # float64 pass); the later ones take the crowded pass
        first = ctx.cells(*args)
        out = ctx.cells(*args)
        passes = ctx.last_pass_counts()
        crowd = passes["crowded_pass"]
        vol, cen = ctx.centroids(*args)
    finally:
        ctx.set_domain(None)
    orc = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, pieces, scenes.L_WALLS)
    assert_close(compare(first, orc, sc.psi0))
    rep = compare(out, orc, sc.psi0)
    r = np.sqrt(sc.psi0)
    ball = 4.0 / 3.0 * math.pi * r ** 3
    site = np.stack([sc.x, sc.y, sc.z], 1).astype(np.float64)
    V = vol.cpu().numpy()
    eM = np.abs(V[:, None] * (cen.cpu().numpy() - site) - orc.V[:, None] * (orc.C - site)).max(1) / (ball * r)
    _say(f"  {sc.n} sites: {rep}; first moments {eM.max():.2e}; crowded pass {crowd}; "
         f"empty {(orc.V == 0).sum()}")
    assert out["walls"].shape[1] == scenes.L_WALLS
    assert_close(rep)
    assert eM.max() <= 1e-5
    assert np.array_equal(V, out["vol"].cpu().numpy())
    assert (orc.walls[:, 6] > 0).any() and (orc.walls[:, 7] > 0).any() or case == "crowded"
    if case == "crowded":
        # the crowded cells of every piece count (the sum over the pieces turns the pass on)
        _say(f"  crowded cells over the pieces: {passes['crowded']}")
        assert crowd and passes["crowded"] >= sc.n // 2


def test_box_split_in_two_pieces(ctx, oracle_mod):
    """The unit box given as two pieces (cut at x = 0.6): the cells against the oracle's
    box cells; sites lie on both sides of the cut and many balls cross it."""
    _say("case: the unit box as two pieces")
    sc = scenes.random_small(400, 2, lo=0.05, hi=0.95, r_lo=0.05, r_hi=0.25)
    ctx.set_domain_pieces(_halves(), 6)
    try:
        out = ctx.cells(*_dev(sc.x, sc.y, sc.z, sc.psi0))
    finally:
        ctx.set_domain(None)
    orc = oracle_mod.cells(sc.x, sc.y, sc.z, sc.psi0)
    rep = compare(out, orc, sc.psi0)
    _say(f"  {rep}")
    assert_close(rep)


def test_l_prism_solve(ctx, oracle_mod):
    """Algorithm 1 in the L-shaped prism (3 pieces): the solve converges and the oracle
    confirms 300 sampled volumes."""
    _say("case: solve in the L prism")
    import paper_2601_05765_amd as L
    import torch
    sc = scenes.l_shape_sites(2000, 4)
    psi0 = scenes.default_psi0(sc.nu)  # the Voronoi start
    xd, yd, zd, pd = _dev(sc.x, sc.y, sc.z, psi0)
    nud = torch.tensor(sc.nu, device="cuda")
    pieces = scenes.l_shape_pieces()
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        st = ctx.solve(xd, yd, zd, nud, pd, opts=L.default_opts(tol=1e-6))
    finally:
        ctx.set_domain(None)
    _say(f"  {sc.n} sites: {st.as_dict()}")
    assert st.status == 0 and st.max_rel_err <= 1e-6
    idx = np.sort(np.random.default_rng(3).choice(sc.n, 300, replace=False))
    c = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, pd.cpu().numpy(), pieces, scenes.L_WALLS, idx=idx)
    err = float(np.max(np.abs(c.V - sc.nu[idx]) / sc.nu[idx]))
    _say(f"  oracle: max rel volume error {err:.2e}")
    assert err <= 1e-5


def test_pieces_errors_and_reset(ctx):
    _say("case: non-convex domain errors, reset to the box")
    import paper_2601_05765_amd as L
    pieces = scenes.l_shape_pieces()
    with pytest.raises(L.LagotError):
        ctx.set_domain_pieces(pieces, 6)  # wall ids 6 and 7 out of range
    with pytest.raises(L.LagotError):
        ctx.set_domain_pieces([(np.array([[1.0, 1.0, 0.0, 0.5]]), [0])], 1)  # normal not unit
    sc = scenes.l_shape_sites(50, 2)
    args = _dev(sc.x, sc.y, sc.z, sc.psi0)
    ref = ctx.cells(*args, csr=False)["vol"].cpu().numpy()
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        # a site in the removed quarter lies in no piece; a site on a plane between pieces
        # lies strictly inside none
        for p in ([0.75, 0.75, 0.5], [0.5, 0.25, 0.5]):
            x, y, z = sc.x.copy(), sc.y.copy(), sc.z.copy()
            x[0], y[0], z[0] = p
            with pytest.raises(L.LagotError):
                ctx.cells(*_dev(x, y, z, sc.psi0), csr=False)
        ctx.cells(*args, csr=False)
    finally:
        ctx.set_domain(None)
    again = ctx.cells(*args, csr=False)["vol"].cpu().numpy()
    assert np.array_equal(ref, again)


def test_l_prism_batched_solve(ctx, oracle_mod):
    """Three instances of different sizes in the L-shaped prism solved in one batched call
    (the per-piece passes and sums run for the instances in the phase each launch
    selects): every instance converges, and the oracle confirms 150 sampled volumes of
    each."""
    _say("case: batched solve in the L prism, 3 instances")
    import paper_2601_05765_amd as L
    import torch
    parts = [scenes.l_shape_sites(m, 20 + k) for k, m in enumerate((600, 1500, 3000))]
    offs = np.cumsum([0] + [p.n for p in parts])
    cat = lambda f: np.concatenate([f(p) for p in parts])
    x, y, z = cat(lambda p: p.x), cat(lambda p: p.y), cat(lambda p: p.z)
    nu = cat(lambda p: p.nu)
    psi0 = cat(lambda p: scenes.default_psi0(p.nu))
    xd, yd, zd, pd = _dev(x, y, z, psi0)
    nud = torch.tensor(nu, device="cuda")
    pieces = scenes.l_shape_pieces()
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        sts = ctx.solve_batched(offs, xd, yd, zd, nud, pd, opts=L.default_opts(tol=1e-6))
    finally:
        ctx.set_domain(None)
    p = pd.cpu().numpy()
    for k, st in enumerate(sts):
        a, b = int(offs[k]), int(offs[k + 1])
        _say(f"  instance {k} ({b - a} sites): status {st.status}, {st.newton_iters} Newton iterations, "
             f"max rel err {st.max_rel_err:.2e}")
        assert st.status == 0 and st.max_rel_err <= 1e-6
        idx = np.sort(np.random.default_rng(k).choice(b - a, 150, replace=False))
        c = oracle_mod.cells_pieces(x[a:b], y[a:b], z[a:b], p[a:b], pieces, scenes.L_WALLS, idx=idx)
        err = float(np.max(np.abs(c.V - nu[a:b][idx]) / nu[a:b][idx]))
        _say(f"    oracle max rel volume error {err:.2e}")
        assert err <= 1e-5


def test_l_prism_paper_k_route(ctx, oracle_mod):
    """lagot_cells_paper_k in the L-shaped prism (6 pieces): the paper's |K| route run in
    every piece and summed, against the oracle's route summed the same way and its signed
    form (every cell on the float64 path; axis-aligned planes, exact in float32)."""
    _say("case: paper K route in the L prism, 6 pieces")
    sc = scenes.l_shape_sites(1500, 12)
    pieces = scenes.l_shape_pieces(True)
    ctx.set_domain_pieces(pieces, scenes.L_WALLS)
    try:
        V, K = ctx.cells_paper_k(*_dev(sc.x, sc.y, sc.z, sc.psi0))
    finally:
        ctx.set_domain(None)
    orc = oracle_mod.cells_pieces(sc.x, sc.y, sc.z, sc.psi0, pieces, scenes.L_WALLS, paper_k=True)
    area = 4.0 * math.pi * sc.psi0
    eK = np.abs(K.cpu().numpy() - orc.Kp) / area
    eK2 = np.abs(K.cpu().numpy() - orc.K) / area
    eV = np.abs(V.cpu().numpy() - orc.V) / (area * np.sqrt(sc.psi0) / 3.0)
    _say(f"  K vs oracle route {eK.max():.2e}, vs signed form {eK2.max():.2e}, V {eV.max():.2e}")
    assert eK.max() <= 1e-9 and eK2.max() <= 1e-9 and eV.max() <= 1e-9
