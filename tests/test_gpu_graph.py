"""Graph mode (opts.use_graph): the launch sequences of a Newton iteration are captured
as HIP graphs once per call and replayed. Every replay must give exactly what eager
launches give, also with eager work and synchronisations between graph calls."""
import sys

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

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


def _dev(sc, psi=None):
    import torch
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    psi = sc.psi0 if psi is None else psi
    return (t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64),
            t(psi, torch.float64))


@pytest.mark.parametrize("name", ["slab_1k", "dam_break_20k"])
def test_graph_replays_match_eager(ctx, oracle_mod, name):
    _say(f"case: graph vs eager solves, {name}")
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(1000, 3) if name == "slab_1k" else scenes.dam_break(20_000, 5)
    x, y, z, nu, psi = _dev(sc)
    st0 = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(use_graph=0))
    ref = psi.cpu().numpy()
    assert st0.status == 0
    for rep in range(3):
        x, y, z, nu, psi = _dev(sc)
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(use_graph=1))
        _say(f"  replay {rep}: {st.newton_iters} it, {st.evals} evals, {st.cg_iters} cg")
        assert st.status == 0
        assert np.array_equal(psi.cpu().numpy(), ref)
        assert (st.newton_iters, st.evals, st.halvings, st.cg_iters) == (st0.newton_iters, st0.evals,
                                                                         st0.halvings, st0.cg_iters)
        # eager work in between
        x2, y2, z2, nu2, p2 = _dev(sc)
        ctx.cells(x2, y2, z2, p2, csr=False)
    if name == "slab_1k":
        c = oracle_mod.cells(sc.x, sc.y, sc.z, ref)
        assert float(np.max(np.abs(c.V - sc.nu) / sc.nu)) <= 1e-5


def test_graph_newton_step_and_batch(ctx):
    _say("case: graph mode for a single Newton step and a batch")
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(1000, 4)
    x, y, z, nu, psi = _dev(sc)
    ctx.newton_step(x, y, z, nu, psi, opts=L.default_opts(use_graph=0))
    ref = psi.cpu().numpy()
    x, y, z, nu, psi = _dev(sc)
    ctx.newton_step(x, y, z, nu, psi, opts=L.default_opts(use_graph=1))
    assert np.array_equal(psi.cpu().numpy(), ref)
    insts = scenes.batch_instances(6, base_seed=7000, n_lo=300, n_hi=3000)
    offs = np.concatenate([[0], np.cumsum([s.n for s in insts])]).astype(np.int64)
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    cat = lambda f: np.concatenate([f(s) for s in insts])
    args = (t(cat(lambda s: s.x), torch.float32), t(cat(lambda s: s.y), torch.float32),
            t(cat(lambda s: s.z), torch.float32), t(cat(lambda s: s.nu), torch.float64))
    psi0 = cat(lambda s: s.psi0)
    p_e = t(psi0, torch.float64)
    ctx.solve_batched(offs, *args, p_e, opts=L.default_opts(use_graph=0))
    for _ in range(2):
        p_g = t(psi0, torch.float64)
        sts = ctx.solve_batched(offs, *args, p_g, opts=L.default_opts(use_graph=1))
        assert all(s.status == 0 for s in sts)
        assert bool((p_g == p_e).all())
