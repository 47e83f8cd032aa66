"""GPU parity of lagot_cells (fused cell_clip + ball_cell_integrate, grid search)
against the FP64 oracle, element by element, through the C-ABI."""
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


def _dev(sc_or_arrays, psi=None):
    import torch
    if hasattr(sc_or_arrays, "x"):
        sc = sc_or_arrays
        x, y, z = sc.x, sc.y, sc.z
        psi = sc.psi0 if psi is None else psi
    else:
        x, y, z = [np.asarray(a, np.float32) for a in sc_or_arrays]
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    return t(x, torch.float32), t(y, torch.float32), t(z, torch.float32), t(psi, torch.float64)


def _run(ctx, oracle_mod, x, y, z, psi, idx=None):
    xd, yd, zd, pd = _dev((x, y, z), psi)
    out = ctx.cells(xd, yd, zd, pd)
    orc = oracle_mod.cells(np.float32(x), np.float32(y), np.float32(z), psi, idx=idx)
    return out, orc


def test_isolated_ball_and_wall_cap(ctx, oracle_mod):
    _say("case: isolated ball + wall cap")
    r, a = 0.1, 0.037
    x = np.array([0.5, a], np.float32)
    y = np.array([0.2, 0.8], np.float32)
    z = np.array([0.5, 0.5], np.float32)
    psi = np.array([r * r, r * r])
    out, orc = _run(ctx, oracle_mod, x, y, z, psi)
    V = out["vol"].cpu().numpy()
    assert V[0] == pytest.approx(4 / 3 * math.pi * r ** 3, rel=1e-6)
    a32 = float(np.float32(a))
    h = r - a32
    assert V[1] == pytest.approx(4 / 3 * math.pi * r ** 3 - math.pi * h * h * (3 * r - h) / 3, rel=1e-6)
    assert_close(compare(out, orc, psi))


@pytest.mark.parametrize("r1,r2,d", [(0.1, 0.1, 0.12), (0.1, 0.13, 0.15), (0.05, 0.14, 0.12), (0.03, 0.12, 0.05)])
def test_two_balls(ctx, oracle_mod, r1, r2, d):
    _say(f"case: two balls r1={r1} r2={r2} d={d}")
    x = np.array([0.4, 0.4 + d], np.float32)
    y = np.array([0.5, 0.5], np.float32)
    z = np.array([0.5, 0.5], np.float32)
    psi = np.array([r1 * r1, r2 * r2])
    out, orc = _run(ctx, oracle_mod, x, y, z, psi)
    assert_close(compare(out, orc, psi))


def test_lattice_cells(ctx, oracle_mod):
    _say("case: lattice ball-cube")
    m, h = 6, 1.0 / 6
    g = (np.arange(m) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    for ratio in (0.6, 0.8, 0.9):
        psi = np.full(m ** 3, (ratio * h) ** 2)
        out, orc = _run(ctx, oracle_mod, X.ravel(), Y.ravel(), Z.ravel(), psi)
        assert_close(compare(out, orc, psi))


@pytest.mark.parametrize("seed", range(8))
def test_random_small_configs(ctx, oracle_mod, seed):
    _say(f"case: random small seed={seed}")
    sc = scenes.random_small(40, seed, r_lo=0.05, r_hi=0.2)
    out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0)
    assert_close(compare(out, orc, sc.psi0))


def test_slab_1k_all_cells(ctx, oracle_mod):
    _say("case: slab_uniform 1k, all cells")
    sc = scenes.slab_uniform(1000, 0)
    out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0)
    rep = compare(out, orc, sc.psi0)
    _say(f"  {rep}")
    assert_close(rep)
    # every facet that is not a tie is present on both sides (compare() checks each row)
    assert out["nnz"] <= int(orc.fcount.sum()) + 10


@pytest.mark.parametrize("tpc", [8, 32, 64])
def test_slab_1k_lanes_per_cell(ctx, oracle_mod, tpc):
    _say(f"case: slab_uniform 1k, {tpc} lanes per cell")
    sc = scenes.slab_uniform(1000, 3)
    ctx.set_threads_per_cell(tpc)
    try:
        out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0)
    finally:
        ctx.set_threads_per_cell(32)
    assert_close(compare(out, orc, sc.psi0))


def test_slab_1k_perturbed_weights(ctx, oracle_mod):
    _say("case: slab_uniform 1k, perturbed weights")
    sc = scenes.slab_uniform(1000, 1)
    rng = np.random.default_rng(5)
    psi = sc.psi0 * rng.uniform(0.5, 1.6, size=sc.n)
    out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, psi)
    assert_close(compare(out, orc, psi))


def test_dam_break_100k_sampled(ctx, oracle_mod):
    _say("case: dam_break 100k, 3000 sampled cells")
    sc = scenes.dam_break(100_000, 0)
    idx = np.sort(np.random.default_rng(1).choice(sc.n, 3000, replace=False))
    out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0, idx=idx)
    rep = compare(out, orc, sc.psi0, idx=idx)
    _say(f"  {rep} fallback={ctx.last_fallback_cells()}")
    assert_close(rep)
    # volume total over all cells against the oracle's sample mean is not a pin; check Sum V < box
    assert float(out["vol"].sum()) < 1.0


def test_dam_break_100k_converged_sampled(ctx, oracle_mod):
    """Cells at the converged weights of the 100k dam break (the state every later Newton
    evaluation and the fluid step sees): volumes, spherical and wall areas, facet areas and
    connectivity of 3,000 sampled cells against the oracle."""
    _say("case: dam_break 100k at its converged weights, 3000 sampled cells")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.dam_break(100_000, 0)
    x, y, z, psi = _dev(sc)
    nu = torch.tensor(sc.nu, dtype=torch.float64, device="cuda")
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5))
    assert st.status == 0
    p = psi.cpu().numpy()
    idx = np.sort(np.random.default_rng(4).choice(sc.n, 3000, replace=False))
    out, orc = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, p, idx=idx)
    rep = compare(out, orc, p, idx=idx)
    _say(f"  {rep}")
    assert_close(rep)


def test_empty_cells(ctx, oracle_mod):
    _say("case: empty cells (engulfed ball, psi <= 0)")
    x = np.array([0.4, 0.45, 0.7, 0.2], np.float32)
    y = np.array([0.5, 0.5, 0.5, 0.2], np.float32)
    z = np.array([0.5, 0.5, 0.5, 0.2], np.float32)
    psi = np.array([0.03 ** 2, 0.12 ** 2, -1e-4, 0.0])
    out, orc = _run(ctx, oracle_mod, x, y, z, psi)
    V = out["vol"].cpu().numpy()
    assert V[0] == 0 and V[2] == 0 and V[3] == 0
    assert V[1] == pytest.approx(orc.V[1], rel=1e-6)
    assert out["nnz"] == 0


@pytest.fixture(scope="module")
def overpacked(oracle_mod):
    """A sphere packed 1.72x and its converged weights (oracle): ~500 candidate
    bisectors per cell, far beyond the kernels' candidate capacities."""
    sc = scenes.overpacked_sphere(2500, 1.72, 0)
    psi, st = oracle_mod.newton_solve(sc.xyz64(), sc.nu, sc.psi0, tol=1e-7)
    assert st.status == "ok"
    return sc, psi


@pytest.mark.parametrize("tpc", [16, 32, 64])
def test_overpacked_sphere_cells(ctx, oracle_mod, overpacked, tpc):
    _say(f"case: over-packed sphere at converged weights, lanes per cell {tpc}")
    sc, psi = overpacked
    ctx.set_threads_per_cell(tpc)
    try:
        out, c = _run(ctx, oracle_mod, sc.x, sc.y, sc.z, psi)
    finally:
        ctx.set_threads_per_cell(32)
    _say(f"  oracle candidates per cell: median {int(np.median(c.ncand))} max {int(c.ncand.max())}")
    rep = compare(out, c, psi)
    _say(f"  {rep} fallback {ctx.last_fallback_cells()} flags {ctx.last_flag_counts()}")
    assert_close(rep)


def _centroid_err(ctx, oracle_mod, x, y, z, psi, idx=None, box=((0, 0, 0), (1, 1, 1))):
    """max over non-empty cells of |c_gpu - c_oracle| / (r_i max(1, 1e-3 |B_i| / V_i)),
    through lagot_centroids: the first moment V c is held to 1e-5 r max(V, 1e-3 |B_i|),
    as volumes are to 1e-5 max(V, 1e-3 |B_i|) (a centroid of a vanishing cell is not
    defined to any accuracy)."""
    xd, yd, zd, pd = _dev((x, y, z), psi)
    vol, cen = ctx.centroids(xd, yd, zd, pd, box=box)
    c = oracle_mod.cells(np.float32(x), np.float32(y), np.float32(z), psi, idx=idx, box=box)
    sel = c.idx
    V = vol.cpu().numpy()[sel]
    C = cen.cpu().numpy()[sel]
    r = np.sqrt(np.maximum(psi[sel], 0.0))
    live = c.V > 0
    assert np.all((V > 0) == live)
    # empty cells report the site itself
    site = np.stack([np.float32(x)[sel], np.float32(y)[sel], np.float32(z)[sel]], 1).astype(np.float64)
    assert np.allclose(C[~live], site[~live], atol=0)
    if not live.any():
        return 0.0
    ball = 4.0 / 3.0 * math.pi * r ** 3
    scale = r * np.maximum(1.0, 1e-3 * ball / np.maximum(c.V, 1e-300))
    return float(np.max(np.linalg.norm(C[live] - c.C[live], axis=1) / scale[live]))


@pytest.mark.parametrize("seed", range(6))
def test_centroids_random_small(ctx, oracle_mod, seed):
    _say(f"case: centroids, random small seed={seed}")
    sc = scenes.random_small(40, seed, r_lo=0.05, r_hi=0.2)
    err = _centroid_err(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0)
    _say(f"  max |dc|/r = {err:.2e}")
    assert err <= 1e-5


def test_centroids_slab_1k_and_dam_break_sample(ctx, oracle_mod):
    _say("case: centroids, slab 1k (all cells) and dam_break 100k (3000 sampled)")
    sc = scenes.slab_uniform(1000, 2)
    assert _centroid_err(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0) <= 1e-5
    sc = scenes.dam_break(100_000, 0)
    idx = np.sort(np.random.default_rng(4).choice(sc.n, 3000, replace=False))
    err = _centroid_err(ctx, oracle_mod, sc.x, sc.y, sc.z, sc.psi0, idx=idx)
    _say(f"  dam_break max |dc|/r = {err:.2e}")
    assert err <= 1e-5


def test_centroids_overpacked_sphere(ctx, oracle_mod, overpacked):
    _say("case: centroids of the over-packed sphere (overflow and float64 passes)")
    sc, psi = overpacked
    err = _centroid_err(ctx, oracle_mod, sc.x, sc.y, sc.z, psi)
    _say(f"  max |dc|/r = {err:.2e}")
    assert err <= 1e-5


def test_centroids_tile_the_box(ctx):
    """Huge weights: the cells tile the box, so sum_i V_i c_i is its first moment."""
    _say("case: centroids, box tiling invariant")
    rng = np.random.default_rng(9)
    n = 5000
    P = rng.uniform(0.02, 0.98, size=(n, 3)).astype(np.float32)
    psi = np.full(n, 0.05)
    xd, yd, zd, pd = _dev((P[:, 0], P[:, 1], P[:, 2]), psi)
    vol, cen = ctx.centroids(xd, yd, zd, pd)
    V = vol.cpu().numpy()
    C = cen.cpu().numpy()
    assert V.sum() == pytest.approx(1.0, rel=1e-6)
    assert np.allclose((V[:, None] * C).sum(0), [0.5, 0.5, 0.5], atol=2e-6)


def test_centroids_scaled_box_and_edge_cases(ctx, oracle_mod):
    """Centroids in the box [0, 2]^3 (a similarity of a unit-box scene: centroids scale by
    2), a single site, and an engulfed (empty) cell."""
    _say("case: centroids in a scaled box, one site, an empty cell")
    sc = scenes.random_small(30, 7, r_lo=0.05, r_hi=0.2)
    f = 2.0
    xs, ys, zs = [(np.asarray(a, np.float64) * f).astype(np.float32) for a in (sc.x, sc.y, sc.z)]
    psi = sc.psi0 * f * f
    box = ((0, 0, 0), (f, f, f))
    assert _centroid_err(ctx, oracle_mod, xs, ys, zs, psi, box=box) <= 1e-5
    xd, yd, zd, pd = _dev((xs, ys, zs), psi)
    _, c2 = ctx.centroids(xd, yd, zd, pd, box=box)
    xd, yd, zd, pd = _dev((sc.x, sc.y, sc.z), sc.psi0)
    _, c1 = ctx.centroids(xd, yd, zd, pd)
    assert np.allclose(c2.cpu().numpy(), f * c1.cpu().numpy(), rtol=0, atol=1e-5)
    # one site: a ball cut by two walls
    assert _centroid_err(ctx, oracle_mod, [0.05], [0.93], [0.5], np.array([0.1 ** 2])) <= 1e-5
    # an engulfed ball reports its site
    x = np.array([0.4, 0.45], np.float32)
    y = np.array([0.5, 0.5], np.float32)
    z = np.array([0.5, 0.5], np.float32)
    xd, yd, zd, pd = _dev((x, y, z), np.array([0.03 ** 2, 0.12 ** 2]))
    vol, cen = ctx.centroids(xd, yd, zd, pd)
    assert float(vol[0]) == 0.0
    assert np.allclose(cen.cpu().numpy()[0], [x[0], y[0], z[0]], atol=0)


@pytest.mark.parametrize("seed", range(3))
def test_sites_on_box_edges_and_corners(ctx, oracle_mod, seed):
    """Sites 1e-6 from two or three walls (the corner edges and corners of the box, where a
    clamped position update leaves them) among ordinary ones: two planes pass within a
    tiny distance of p_i, and the cell must still match the oracle."""
    rng = np.random.default_rng(300 + seed)
    n = 400
    p = rng.uniform(0.02, 0.98, (n, 3))
    e = 1e-6
    for k in range(60):
        a, b = rng.choice(3, 2, replace=False)
        p[k, a] = e if rng.random() < 0.5 else 1 - e
        p[k, b] = e if rng.random() < 0.5 else 1 - e
        if k % 4 == 0:
            c = 3 - a - b
            p[k, c] = e if rng.random() < 0.5 else 1 - e
    r = rng.uniform(0.06, 0.12, n)
    psi = r * r
    x, y, z = (np.float32(p[:, i]) for i in range(3))
    _say(f"case: sites on box edges and corners, seed {seed}")
    out, orc = _run(ctx, oracle_mod, x, y, z, psi)
    rep = compare(out, orc, psi)
    _say(f"  {rep}")
    assert_close(rep)
