"""lagot_cells_paper_k on the GPU: |K| by section 3.3's own route (interior point c from
rays cast from the restricted facets' centroids, each facet projected from c onto the
sphere, Gauss-Bonnet over the projected arcs), against the FP64 oracle's two routes (the
same route, and the signed solid angles) and against lagot_cells' signed form on the GPU
(the A/B pair)."""
import math
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


def _t(a, dt):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def _run(ctx, sc, psi):
    import torch
    x, y, z = _t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32)
    V, K = ctx.cells_paper_k(x, y, z, _t(psi, torch.float64))
    return V.cpu().numpy(), K.cpu().numpy(), (x, y, z)


@pytest.mark.parametrize("name,make", [("slab_1000", lambda: scenes.slab_uniform(1000, 0)),
                                       ("overpacked_sphere_2500", lambda: scenes.overpacked_sphere(2500, 1.72, 0)),
                                       ("dam_break_3000", lambda: scenes.dam_break(3000, 1))])
def test_route_matches_oracle_on_every_cell(ctx, oracle_mod, name, make):
    """Every cell: K against the oracle's route and its signed form, V against the oracle,
    to 1e-9 of the ball's area / volume (float64 path, float32 sites promoted exactly)."""
    _say(f"case: paper K route, {name}")
    sc = make()
    psi = sc.psi0
    V, K, _ = _run(ctx, sc, psi)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi, paper_k=True)
    area = 4.0 * math.pi * psi
    vol = area * np.sqrt(psi) / 3.0
    eK = np.abs(K - c.Kp) / area
    eK2 = np.abs(K - c.K) / area
    eV = np.abs(V - c.V) / vol
    _say(f"  max |K - Kp(oracle)| / 4 pi r^2 {eK.max():.2e}, vs signed form {eK2.max():.2e}, "
         f"max |V - V(oracle)| / ball {eV.max():.2e}")
    assert eK.max() <= 1e-9 and eK2.max() <= 1e-9 and eV.max() <= 1e-9


def test_route_at_converged_weights_and_ab_pair(ctx, oracle_mod):
    """The converged weights of the 2,500-site over-packed sphere (most cells crowded, sites
    outside their own cells): the route against the oracle on every cell, and against
    lagot_cells' signed solid-angle form on the GPU (float32 fast pass for most cells)."""
    _say("case: paper K route, over-packed sphere at converged weights")
    import torch
    sc = scenes.overpacked_sphere(2500, 1.72, 0)
    psi, st = oracle_mod.newton_solve(sc.xyz64(), sc.nu, sc.psi0, tol=1e-7)
    assert st.status == "ok"
    V, K, (x, y, z) = _run(ctx, sc, psi)
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi)
    area = 4.0 * math.pi * psi
    assert (np.abs(K - c.K) / area).max() <= 1e-9
    out = ctx.cells(x, y, z, _t(psi, torch.float64))
    Kb = out["sph"].cpu().numpy()
    e = np.abs(K - Kb) / area
    _say(f"  A/B: max |K(route) - K(signed)| / 4 pi r^2 {e.max():.2e}")
    assert e.max() <= 1e-5


def test_route_dam_break_100k_sampled(ctx, oracle_mod):
    """100,000 sites: every cell against lagot_cells (A/B), 2,000 sampled cells against the
    oracle."""
    _say("case: paper K route, dam break 100k")
    import torch
    sc = scenes.dam_break(100_000, 0)
    psi = sc.psi0
    V, K, (x, y, z) = _run(ctx, sc, psi)
    ms = ctx.last_cell_kernel_ms()
    out = ctx.cells(x, y, z, _t(psi, torch.float64))
    Kb = out["sph"].cpu().numpy()
    area = 4.0 * math.pi * psi
    e_ab = np.abs(K - Kb) / area
    idx = np.sort(np.random.default_rng(5).choice(sc.n, 2000, replace=False))
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi, idx=idx, paper_k=True)
    e = np.abs(K[idx] - c.Kp) / area[idx]
    _say(f"  route kernel {ms:.3f} ms; A/B max {e_ab.max():.2e}; oracle max {e.max():.2e}")
    assert e.max() <= 1e-9 and e_ab.max() <= 1e-5


def test_route_rejects_bad_arguments(ctx):
    import torch
    import paper_2601_05765_amd as L
    sc = scenes.slab_uniform(100, 0)
    x, y, z = _t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32)
    p = _t(sc.psi0, torch.float64)
    v = torch.empty(100, dtype=torch.float64, device="cuda")
    lib = L.load()
    rc = lib.lagot_cells_paper_k(ctx._h, 100, x.data_ptr(), y.data_ptr(), z.data_ptr(), p.data_ptr(),
                                 L.make_box(((0, 0, 0), (1, 1, 1))), v.data_ptr(), None)
    assert rc == L.EINVAL
    rc = lib.lagot_cells_paper_k(ctx._h, 0, x.data_ptr(), y.data_ptr(), z.data_ptr(), p.data_ptr(),
                                 L.make_box(((0, 0, 0), (1, 1, 1))), v.data_ptr(), v.data_ptr())
    assert rc == L.EINVAL
