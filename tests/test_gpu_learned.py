"""The learned warm start inside lagot_solve (opts.use_learned = 1) against the FP64 oracle.

The network's correction is taken like a Newton step from the start weights, halved up to
twice: psi + beta s^2 out for beta = 1, 1/2, 1/4; the first trial that keeps every cell at
the KMT floor eps0 of the start weights and lowers both the residual norm and the largest
relative volume error is kept (learned_accepted = 1 + the halvings); Newton then runs to
the tolerance from whichever start was kept. The networks have known outcomes:

  * hand-built networks that output a damped Jacobi step k f from their input
    f = (nu - V)/nu: hidden unit 0 carries 16 f + 8 through three GELU layers (GELU is the
    identity to 3e-7 there), the output layer maps it back to k f, so the trial is
    psi + beta k nu^(2/3) (nu - V)/nu. On slab_uniform(1000, 0) from psi0 the oracle gives
    (min V / eps0, ||g|| ratio, max rel err ratio) at beta = 1, 1/2, 1/4:
      k = 0.1: (3.21, 0.77, 0.90) kept at the full step;
      k = 0.4: (0.00, 0.68, 1.16), then (3.37, 0.61, 0.89): kept at beta = 1/2;
      k = 0.8: empty, empty, then (3.37, 0.61, 0.89): kept at beta = 1/4;
      k = 1.6: a cell empties at every beta; k = -0.1: ||g|| grows at every beta (1.24,
      1.12, 1.06): both rejected, after which the solve is the plain solve, bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_2601_05765_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(sc, psi=None):
    import torch
    t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    psi = sc.psi0 if psi is None else psi
    return (t(sc.x, torch.float32), t(sc.y, torch.float32), t(sc.z, torch.float32), t(sc.nu, torch.float64),
            t(psi, torch.float64))


def jacobi_params(k=0.1, a=16.0, c=8.0) -> np.ndarray:
    """Flat float32 parameters (lagot.h layout: W[in][out] row-major, then the bias, per
    layer) of the damped-Jacobi network described above."""
    W1 = np.zeros((64, 128)); b1 = np.zeros(128)
    W1[50, 0] = a
    b1[0] = c
    W2 = np.zeros((128, 128)); b2 = np.zeros(128)
    W2[0, 0] = 1.0
    W3 = np.zeros((128, 128)); b3 = np.zeros(128)
    W3[0, 0] = 1.0
    W4 = np.zeros((128, 1)); b4 = np.zeros(1)
    W4[0, 0] = k / a
    b4[0] = -k * c / a
    return np.concatenate([v.ravel() for v in (W1, b1, W2, b2, W3, b3, W4, b4)]).astype(np.float32)


def _set(ctx, params):
    import torch
    ctx.mlp_set_params(torch.tensor(params, dtype=torch.float32, device="cuda"))


def _oracle_err(oracle_mod, sc, psi):
    c = oracle_mod.cells(sc.x, sc.y, sc.z, psi)
    return float(np.max(np.abs(c.V - sc.nu) / sc.nu))


def test_learned_guess_kept(oracle_mod):
    _say("case: learned solve, damped-Jacobi network, slab_uniform 1k seed 0 (guess must be kept)")
    import paper_2601_05765_amd as L
    ctx = L.Context()
    _set(ctx, jacobi_params())
    sc = scenes.slab_uniform(1000, 0)
    x, y, z, nu, psi = _dev(sc)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, use_learned=1))
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.learned_accepted == 1
    err = _oracle_err(oracle_mod, sc, psi.cpu().numpy())
    _say(f"  oracle max rel err {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("k,kept", [(0.4, 2), (0.8, 3)])
def test_learned_guess_kept_after_halving(oracle_mod, k, kept):
    _say(f"case: learned solve, damped-Jacobi network k={k}, slab_uniform 1k (guess kept after {kept - 1} halvings)")
    import paper_2601_05765_amd as L
    ctx = L.Context()
    _set(ctx, jacobi_params(k=k))
    sc = scenes.slab_uniform(1000, 0)
    x, y, z, nu, psi = _dev(sc)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, use_learned=1))
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.learned_accepted == kept
    assert _oracle_err(oracle_mod, sc, psi.cpu().numpy()) <= 1e-5


@pytest.mark.parametrize("k", [1.6, -0.1])
def test_learned_guess_rejected_is_plain_solve(oracle_mod, k):
    _say(f"case: learned solve, damped-Jacobi network k={k} (guess must be rejected), bit-identical to the plain solve")
    import torch
    import paper_2601_05765_amd as L
    ctx = L.Context()
    _set(ctx, jacobi_params(k=k))
    sc = scenes.slab_uniform(1000, 0)
    x, y, z, nu, psi = _dev(sc)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, use_learned=1))
    _say(f"  {st.as_dict()}")
    assert st.status == 0 and st.learned_accepted == 0
    x, y, z, nu, psi2 = _dev(sc)
    st2 = ctx.solve(x, y, z, nu, psi2, opts=L.default_opts(tol=1e-5))
    assert st2.newton_iters == st.newton_iters
    assert torch.equal(psi, psi2)
    assert _oracle_err(oracle_mod, sc, psi.cpu().numpy()) <= 1e-5


def test_kept_guess_then_larger_calls(oracle_mod):
    """A kept guess swaps the context's two output sets; later calls with more sites than
    that call (but fewer than the context has held) must still have room in both. The
    context first holds 5,000 sites, then a learned solve at 1,000 keeps its guess, then
    solves at 3,000 and 5,000 and an evaluation at 4,000 run on the same context."""
    _say("case: kept learned guess at 1k on a context sized for 5k, then 3k/5k solves and a 4k evaluation")
    import paper_2601_05765_amd as L
    from parity import compare, assert_close
    ctx = L.Context()
    _set(ctx, jacobi_params())
    big = scenes.slab_uniform(5000, 21)
    x, y, z, nu, psi = _dev(big)
    ctx.cells(x, y, z, psi)
    sc = scenes.slab_uniform(1000, 0)
    x, y, z, nu, psi = _dev(sc)
    st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5, use_learned=1))
    assert st.status == 0 and st.learned_accepted == 1
    for n, seed in ((3000, 22), (5000, 23)):
        s2 = scenes.slab_uniform(n, seed)
        x, y, z, nu, psi = _dev(s2)
        st = ctx.solve(x, y, z, nu, psi, opts=L.default_opts(tol=1e-5))
        _say(f"  n={n}: {st.as_dict()}")
        assert st.status == 0
        assert _oracle_err(oracle_mod, s2, psi.cpu().numpy()) <= 1e-5
    s4 = scenes.slab_uniform(4000, 24)
    x, y, z, nu, psi = _dev(s4)
    out = ctx.cells(x, y, z, psi)
    idx = np.arange(0, 4000, 7)
    orc = oracle_mod.cells(s4.x, s4.y, s4.z, s4.psi0, idx=idx)
    assert_close(compare(out, orc, s4.psi0, idx))
