"""Crowded scenes on the GPU: the box-overlap candidates of section 4 ("Finding
Contributing Neighbors") and the path following on the prescribed volumes, against
the FP64 oracle.

Cells whose search block is crowded (a few balls much larger than the rest) are seeded
with their nearest sites, boxed, and finished with the sites whose boxes overlap their
own; the results must equal the oracle's brute-force cells element by element (the
candidate set is exact, not a heuristic). The large-scene recipe (200 droplets packed
1.72x next to a slab, log-normal prescribed volumes) is solved from its Voronoi start
with opts.continuation, and then advected and solved again as in the 2M-site sequence,
at 200,000 sites so that the oracle can check sampled cells."""
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


def _t(a, dt):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _xyz(sc):
    import torch
    return _t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32)


def _sample(n, psi, seed, k_top=150, k_rand=250):
    """The heaviest sites (the most crowded cells) and a random sample."""
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.argsort(-psi)[:k_top], rng.choice(n, k_rand, replace=False)]))


@pytest.fixture(scope="module")
def splash_settled(ctx):
    """The splash recipe at 200,000 sites solved with path following (continuation)."""
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.splash(200_000, 0)
    x, y, z = _xyz(sc)
    nu, psi = _t(sc.nu, torch.float64), _t(sc.psi0, torch.float64)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, residual_test=0, continuation=1), check=False)
    _say(f"  settle: {st.as_dict()}")
    return sc, st, psi.cpu().numpy()


def test_continuation_settles_splash_200k(ctx, oracle_mod, splash_settled):
    _say("case: splash 200k settled by continuation")
    sc, st, psi = splash_settled
    assert st.status == 0 and st.max_rel_err <= 1e-5 and st.stages >= 1
    idx = _sample(sc.n, psi, 1)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi, idx=idx)
    err = np.abs(c.V - sc.nu[idx]) / sc.nu[idx]
    _say(f"  oracle on {len(idx)} cells: max {err.max():.2e} p99 {np.percentile(err, 99):.2e}")
    assert err.max() <= 1e-5


def test_crowded_cells_match_oracle(ctx, oracle_mod, splash_settled):
    """At the settled weights most droplet cells are crowded (balls of many spacings,
    displaced cells): volumes, spherical areas, facet areas, wall areas and connectivity
    of sampled cells against the oracle, with the crowded pass in use."""
    _say("case: crowded cells at the settled splash weights")
    sc, _, psi = splash_settled
    x, y, z = _xyz(sc)
    import torch
    out = ctx.cells(x, y, z, _t(psi, torch.float64))
    passes = ctx.last_pass_counts()
    _say(f"  passes {passes} flags {ctx.last_flag_counts()['final']}")
    assert passes["crowded"] > 10_000 and passes["crowded_pass"]
    idx = _sample(sc.n, psi, 2)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi, idx=idx)
    rep = compare(out, c, psi, idx=idx)
    _say(f"  {rep}")
    assert_close(rep)


def test_overpacked_sphere_takes_crowded_pass(oracle_mod):
    """The over-packed sphere at its converged weights, in a box [-2, 3]^3 large enough that
    the site grid keeps cells of 2 r_max: most cells' search blocks are crowded. On a fresh
    context the first evaluation finishes the deferred cells on the float64 pass (nothing
    announced crowded cells), the second on the crowded pass (seed, boxes, box-overlap
    candidates); both match the oracle on every cell."""
    _say("case: over-packed sphere, crowded cells on a fresh context")
    import torch
    import paper_2601_05765_amd as L
    fresh = L.Context()
    sc = scenes.overpacked_sphere(2500, 1.72, 0)
    psi, st = oracle_mod.newton_solve(sc.xyz64(), sc.nu, sc.psi0, tol=1e-7)
    assert st.status == "ok"
    x, y, z = _xyz(sc)
    box = ((-2.0, -2.0, -2.0), (3.0, 3.0, 3.0))
    orc = oracle_mod.cells(sc.x, sc.y, sc.z, psi, box=box)
    for k in range(2):
        out = fresh.cells(x, y, z, _t(psi, torch.float64), box=box)
        passes = fresh.last_pass_counts()
        rep = compare(out, orc, psi)
        _say(f"  evaluation {k}: passes {passes} {rep}")
        assert passes["crowded"] >= sc.n // 2
        assert passes["crowded_pass"] == (k == 1)
        assert_close(rep)


def test_advected_steps_200k(ctx, oracle_mod, splash_settled):
    """Two steps of the large-scene sequence at 200,000 sites: sites advected by dt 2e-3
    with their random velocities (mirror reflection at the walls), each solve warm-started
    from the previous weights (with continuation, as the 2M-site sequence runs)."""
    _say("case: splash 200k, two advect-and-solve steps")
    import torch
    import paper_2601_05765_amd as L
    sc, _, psi = splash_settled
    cur = sc
    p = _t(psi, torch.float64)
    nu = _t(sc.nu, torch.float64)
    for k in range(1, 3):
        cur = scenes.advect(cur, 2e-3)
        x, y, z = _xyz(cur)
        st = ctx.solve(x, y, z, nu, p, opts=L.default_opts(tol=1e-5, residual_test=0, continuation=1), check=False)
        _say(f"  step {k}: {st.as_dict()}")
        assert st.status == 0 and st.max_rel_err <= 1e-5
        ph = p.cpu().numpy()
        idx = _sample(cur.n, ph, 10 + k, k_top=80, k_rand=150)
        c = oracle_mod.cells(cur.x, cur.y, cur.z, ph, idx=idx)
        err = np.abs(c.V - cur.nu[idx]) / cur.nu[idx]
        _say(f"  oracle max {err.max():.2e}")
        assert err.max() <= 1e-5


def test_solve_moved_200k(ctx, oracle_mod, splash_settled):
    """lagot_solve_moved on the large-scene sequence at 200,000 sites: the settled weights
    carried with the advected sites (dt 2e-3), split into parts while the carried weights
    leave cells empty; each step converges (oracle re-evaluation of sampled cells), and the
    two steps take fewer Newton iterations in all than lagot_solve from the previous weights."""
    _say("case: splash 200k, lagot_solve_moved")
    import torch
    import paper_2601_05765_amd as L
    sc, _, psi = splash_settled
    nu = _t(sc.nu, torch.float64)
    opts = L.default_opts(tol=1e-5, residual_test=0)
    cur, p = sc, _t(psi, torch.float64)
    its_moved = its_plain = 0
    for k in range(1, 3):
        nxt = scenes.advect(cur, 2e-3)
        x0, y0, z0 = _xyz(cur)
        x1, y1, z1 = _xyz(nxt)
        q = p.clone()
        plain = ctx.solve(x1, y1, z1, nu, q, opts=opts, check=False)
        st = ctx.solve_moved(x0, y0, z0, x1, y1, z1, nu, p, opts=opts, check=False)
        _say(f"  step {k}: moved {st.as_dict()}; plain iterations {plain.newton_iters} evals {plain.evals}")
        assert st.status == 0 and st.max_rel_err <= 1e-5 and st.stages >= 1
        assert plain.status == 0
        its_moved += st.newton_iters
        its_plain += plain.newton_iters
        ph = p.cpu().numpy()
        idx = _sample(nxt.n, ph, 20 + k, k_top=80, k_rand=150)
        c = oracle_mod.cells(nxt.x, nxt.y, nxt.z, ph, idx=idx)
        err = np.abs(c.V - nxt.nu[idx]) / nxt.nu[idx]
        _say(f"  oracle max {err.max():.2e}")
        assert err.max() <= 1e-5
        cur = nxt
    assert its_moved < its_plain


def test_solve_moved_without_motion_keeps_the_solution(ctx, oracle_mod):
    """Sites that do not move: the carried weights are the given ones (d = 0), which already
    solve the problem, so no Newton iteration is taken."""
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(1000, 0)
    x, y, z = _xyz(sc)
    nu = _t(sc.nu, torch.float64)
    p = _t(sc.psi0, torch.float64)
    st = ctx.solve(x, y, z, nu, p, opts=L.default_opts(tol=1e-6), check=False)
    assert st.status == 0
    p0 = p.clone()
    st = ctx.solve_moved(x, y, z, x, y, z, nu, p, opts=L.default_opts(tol=1e-5), check=False)
    assert st.status == 0 and st.newton_iters == 0 and st.stages == 1
    assert torch.equal(p, p0)


def test_continuation_options_rejected(ctx):
    """Invalid continuation options, and continuation in a batched call, are EINVAL."""
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(500, 3)
    x, y, z = _xyz(sc)
    nu = _t(sc.nu, torch.float64)
    for kw in ({"continuation": 2}, {"continuation": 1, "stage_newton": 0}, {"continuation": 1, "stage_tol": 0.0},
               {"continuation": 1, "stage_step": 0.0}, {"continuation": 1, "stage_step": 1.5}):
        p = _t(sc.psi0, torch.float64)
        st = ctx.solve(x, y, z, nu, p, opts=L.default_opts(**kw), check=False)
        assert st.status == L.EINVAL, kw
    offs = np.array([0, 250, 500], dtype=np.int64)
    p = _t(sc.psi0, torch.float64)
    sts = ctx.solve_batched(offs, x, y, z, nu, p, opts=L.default_opts(continuation=1), check=False)
    assert all(s.status == L.EINVAL for s in sts)


def test_continuation_on_easy_problem_matches_plain(ctx, oracle_mod):
    """On the 1,000-site slab the path-following solve converges to the same unique
    weights as the plain one (oracle re-evaluation within tolerance)."""
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(1000, 0)
    x, y, z = _xyz(sc)
    nu = _t(sc.nu, torch.float64)
    p = _t(sc.psi0, torch.float64)
    st = ctx.solve(x, y, z, nu, p, opts=L.default_opts(tol=1e-5, continuation=1), check=False)
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.stages >= 1
    c = oracle_mod.cells(sc.x, sc.y, sc.z, p.cpu().numpy())
    assert float(np.max(np.abs(c.V - sc.nu) / sc.nu)) <= 1e-5


def test_continuation_first_step_one_third(ctx, oracle_mod):
    """Path following with a first step of 1/3 in s (with loose intermediate stages and
    the step search started at twice the last step) on the 200,000-site splash scene from
    its Voronoi start: converges to the oracle's volumes."""
    _say("case: splash 200k, continuation with stage_step 1/3")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.splash(200_000, 0)
    x, y, z = _xyz(sc)
    nu, psi = _t(sc.nu, torch.float64), _t(sc.psi0, torch.float64)
    opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1, stage_step=1.0 / 3.0, stage_tol=0.1,
                          step_start=1, cg_rtol=1e-3)
    st = ctx.solve(x, y, z, nu, psi, opts=opts, check=False)
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.stages >= 1 and st.max_rel_err <= 1e-5
    ph = psi.cpu().numpy()
    idx = _sample(sc.n, ph, 31, k_top=100, k_rand=200)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, ph, idx=idx)
    assert float(np.max(np.abs(c.V - sc.nu[idx]) / sc.nu[idx])) <= 1e-5


def test_continuation_stage_carry(ctx, oracle_mod):
    """opts.step_start = 2 (the bench's setting: each continuation stage after the first
    starts its step search at the first step length accepted in the stage before) on the
    200,000-site splash scene from its Voronoi start: the same unique weights (oracle
    re-evaluation of the heaviest and random cells) as with step_start = 1."""
    _say("case: splash 200k, continuation with the stages' first steps carried")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.splash(200_000, 0)
    x, y, z = _xyz(sc)
    nu = _t(sc.nu, torch.float64)
    res = {}
    for ss in (1, 2):
        psi = _t(sc.psi0, torch.float64)
        opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1, stage_tol=0.1, step_start=ss,
                              cg_rtol=1e-3)
        st = ctx.solve(x, y, z, nu, psi, opts=opts, check=False)
        _say(f"  step_start {ss}: {st.as_dict()}")
        assert st.status == 0 and st.stages >= 2 and st.max_rel_err <= 1e-5
        res[ss] = psi.cpu().numpy()
    ph = res[2]
    idx = _sample(sc.n, ph, 37, k_top=100, k_rand=200)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, ph, idx=idx)
    assert float(np.max(np.abs(c.V - sc.nu[idx]) / sc.nu[idx])) <= 1e-5


def test_continuation_stage_norm_stop(ctx, oracle_mod):
    """opts.stage_gtol = 0.01 (the bench's setting: an intermediate stage also ends when
    ||nu(s) - V||_2 has fallen to 1% of its value at the stage's start) on the 200,000-site
    splash scene from its Voronoi start: converges to the oracle's volumes in no more
    Newton iterations than with stage_tol alone; out-of-range values are EINVAL."""
    _say("case: splash 200k, continuation with the stages' norm stop")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.splash(200_000, 0)
    x, y, z = _xyz(sc)
    nu = _t(sc.nu, torch.float64)
    its = {}
    for gt in (0.0, 0.01, 0.5):
        psi = _t(sc.psi0, torch.float64)
        opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1, stage_tol=0.1, step_start=2,
                              cg_rtol=1e-3, stage_gtol=gt)
        st = ctx.solve(x, y, z, nu, psi, opts=opts, check=False)
        _say(f"  stage_gtol {gt}: {st.as_dict()}")
        assert st.status == 0 and st.stages >= 2 and st.max_rel_err <= 1e-5
        its[gt] = st.newton_iters
    assert its[0.01] <= its[0.0]
    ph = psi.cpu().numpy()
    idx = _sample(sc.n, ph, 41, k_top=100, k_rand=200)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, ph, idx=idx)
    assert float(np.max(np.abs(c.V - sc.nu[idx]) / sc.nu[idx])) <= 1e-5
    small = scenes.slab_uniform(300, 1)
    xs, ys, zs = _xyz(small)
    for bad in (1.0, -0.1, float("nan")):
        st = ctx.solve(xs, ys, zs, _t(small.nu, torch.float64), _t(small.psi0, torch.float64),
                       opts=L.default_opts(continuation=1, stage_gtol=bad), check=False)
        assert st.status == L.EINVAL


def test_solve_below_the_float32_floor(ctx, oracle_mod):
    """A tolerance below the rounding of the float32 cells (1e-7 on the 200,000-site splash
    scene): at a full Newton step that no longer halves ||nu - V||, the cells still off by
    more than tol/4 are marked and finished on the float64 path for the rest of the call,
    so the solve converges instead of stalling (at 1e-5 the same solve sends ~7,000 cells
    to the float64 path in all; here over 100,000 evaluations of cells go there)."""
    _say("case: splash 200k to 1e-7 (float64 marks at stalled iterations)")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.splash(200_000, 0)
    x, y, z = _xyz(sc)
    nu, psi = _t(sc.nu, torch.float64), _t(sc.psi0, torch.float64)
    opts = L.default_opts(tol=1e-7, residual_test=0, continuation=1, stage_tol=0.1, step_start=2, cg_rtol=1e-3,
                          stage_gtol=0.1)
    st = ctx.solve(x, y, z, nu, psi, opts=opts, check=False)
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.max_rel_err <= 1e-7
    assert st.fallback_cells > 100_000
    ph = psi.cpu().numpy()
    idx = _sample(sc.n, ph, 43, k_top=100, k_rand=200)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, ph, idx=idx)
    err = float(np.max(np.abs(c.V - sc.nu[idx]) / sc.nu[idx]))
    _say(f"  oracle max rel volume error {err:.2e}")
    assert err <= 1e-6


def test_hopeless_start_restarts(ctx, oracle_mod, splash_settled):
    """Settled 200,000-site weights at sites advected far (dt 0.05): many more than 1% of the
    cells are empty. The start evaluation counts the certainly empty cells from the boxes
    after the seed pass and skips its crowded and float64 passes; the solve restarts from
    the default weights and converges to the oracle's volumes."""
    _say("case: splash 200k, far-moved sites, start gate and restart")
    import torch
    import paper_2601_05765_amd as L
    sc, _, psi = splash_settled
    cur = scenes.advect(sc, 0.05)
    x, y, z = _xyz(cur)
    nu = _t(sc.nu, torch.float64)
    p = _t(psi, torch.float64)
    opts = L.default_opts(tol=1e-5, residual_test=0, continuation=1, stage_tol=0.1, step_start=2, cg_rtol=1e-3,
                          stage_gtol=0.1)
    st = ctx.solve(x, y, z, nu, p, opts=opts, check=False)
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.default_start == 1 and st.repaired_start == 0 and st.max_rel_err <= 1e-5
    ph = p.cpu().numpy()
    idx = _sample(cur.n, ph, 47, k_top=100, k_rand=200)
    c = oracle_mod.cells(cur.x, cur.y, cur.z, ph, idx=idx)
    err = float(np.max(np.abs(c.V - cur.nu[idx]) / cur.nu[idx]))
    _say(f"  oracle max rel volume error {err:.2e}")
    assert err <= 1e-5
