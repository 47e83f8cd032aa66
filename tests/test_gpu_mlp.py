"""GPU learned warm start (lagot_features, lagot_mlp_forward, lagot_mlp_train_step)
against the FP64 oracle (oracle/mlp.py), through the C-ABI.

Bars: neighbour lists bit-exact (ascending (distance, index)); inputs equal to the
oracle's after bf16 rounding; the network output within the bf16 bound of the
FP64 network evaluated on the same bf16-rounded inputs and weights; gradients of
the batch loss within 3% (norm) of the FP64 backward; the first Adam step equal to
-lr sign(g)."""
import sys

import numpy as np
import pytest

from oracle import mlp
from paper_2601_05765_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits_to_f64(b):
    return (np.asarray(b).astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def flat(params):
    return np.concatenate([p.ravel() for p in params]).astype(np.float32)


def unflat(v):
    out, o = [], 0
    for a, b in mlp.LAYERS:
        out.append(v[o:o + a * b].reshape(a, b).astype(np.float64))
        o += a * b
        out.append(v[o:o + b].astype(np.float64))
        o += b
    return out


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2601_05765_amd as L
    assert torch.cuda.is_available()
    return L.Context()


def _t(a, dt):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("name", ["slab_1k", "dam_break_20k_sample"])
def test_knn_and_inputs(ctx, oracle_mod, name):
    import torch
    _say(f"case: knn/inputs {name}")
    sc = scenes.slab_uniform(1000, 5) if name == "slab_1k" else scenes.dam_break(20_000, 3)
    psi_prev = sc.psi0 * np.random.default_rng(1).uniform(0.8, 1.2, size=sc.n)
    nbr, feats = ctx.features(_t(sc.x, torch.float32), _t(sc.y, torch.float32), _t(sc.z, torch.float32),
                              _t(psi_prev, torch.float64), _t(sc.nu, torch.float64))
    idx = np.arange(sc.n) if sc.n <= 1000 else np.sort(np.random.default_rng(2).choice(sc.n, 800, replace=False))
    P = sc.xyz64()
    ref = mlp.knn(P, 16, idx=idx)
    got = nbr.cpu().numpy()[idx]
    assert np.array_equal(got, ref)
    V = oracle_mod.cells(sc.x, sc.y, sc.z, psi_prev).V
    F = mlp.features(P, psi_prev, sc.nu, ref, V, idx=idx)
    G = bf16_bits_to_f64(feats.cpu().numpy()[idx])
    # the GPU forms offsets in float32 then rounds to bf16 (one bf16 ulp); the mismatch
    # inputs come from float32 cell volumes (within 1e-5 of nu, see the cell parity tests)
    tol = 2.0 ** -7 * np.abs(F) + 1e-30
    tol[:, 50:] += 2e-5
    assert np.all(np.abs(G - bf16_round(F)) <= tol)


def test_forward_within_bf16_bound(ctx):
    import torch
    _say("case: mlp forward")
    params = mlp.init_params(3)
    v = flat(params)
    ctx.mlp_set_params(_t(v, torch.float32))
    rng = np.random.default_rng(4)
    X = rng.normal(size=(3000, 64))
    X[:, 50:] = 0
    Xb = bf16_round(X)
    bits = (np.asarray(Xb, np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    out = ctx.mlp_forward(_t(bits, torch.int16)).cpu().numpy().astype(np.float64)
    pr = unflat(v)
    for li in (0, 2, 4):
        pr[li] = bf16_round(pr[li])
    ref, _ = mlp.forward(pr, Xb)
    scale = np.abs(ref).mean() + 1e-3
    err = np.abs(out - ref) / (np.abs(ref) + scale)
    _say(f"  max scaled err {err.max():.3e}")
    assert err.max() <= 3e-2


def test_gradients_and_first_adam_step(ctx):
    import torch
    _say("case: mlp backward + adam")
    params = mlp.init_params(5)
    v = flat(params)
    ctx.mlp_set_params(_t(v, torch.float32))
    rng = np.random.default_rng(6)
    m = 2048
    X = rng.normal(size=(m, 64))
    X[:, 50:] = 0
    Xb = bf16_round(X)
    y = rng.normal(size=m)
    bits = (np.asarray(Xb, np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    lr = 1e-4
    loss = ctx.mlp_train_step(_t(bits, torch.int16), _t(y, torch.float32), _t(np.arange(m), torch.int32), lr)
    g_gpu = ctx.mlp_last_grads().cpu().numpy().astype(np.float64)
    pr = unflat(v)
    for li in (0, 2, 4):
        pr[li] = bf16_round(pr[li])
    ref_loss, ref_grads = mlp.loss_and_grads(pr, Xb, y)
    g_ref = np.concatenate([g.ravel() for g in ref_grads])
    assert loss == pytest.approx(ref_loss, rel=2e-2)
    rel = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    cos = g_gpu @ g_ref / (np.linalg.norm(g_gpu) * np.linalg.norm(g_ref))
    _say(f"  grad rel err {rel:.3e} cos {cos:.6f}")
    assert rel <= 3e-2 and cos >= 0.999
    new = ctx.mlp_get_params().cpu().numpy().astype(np.float64)
    big = np.abs(g_gpu) > 1e-5
    step = new - v.astype(np.float64)
    # float32 parameters: the step is resolved to a few ulp of |p| (<= 2e-7 here)
    assert np.allclose(step[big], -lr * np.sign(g_gpu[big]), rtol=1e-3, atol=1e-6)


def test_training_reduces_loss(ctx):
    import torch
    _say("case: mlp training on a smooth target")
    ctx.mlp_set_params(_t(flat(mlp.init_params(7)), torch.float32))
    rng = np.random.default_rng(8)
    m = 16384
    X = rng.normal(size=(m, 64)) * 0.5
    X[:, 50:] = 0
    y = np.tanh(X[:, 0] - 0.5 * X[:, 3]) + 0.3 * X[:, 48]
    Xb = bf16_round(X)
    bits = _t((np.asarray(Xb, np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16), torch.int16)
    yt = _t(y, torch.float32)
    first = None
    for it in range(300):
        idx = _t(rng.choice(m, 1024, replace=False).astype(np.int32), torch.int32)
        loss = ctx.mlp_train_step(bits, yt, idx, 2e-3)
        first = loss if first is None else first
    _say(f"  loss {first:.4f} -> {loss:.4f}")
    assert loss < 0.1 * first


def test_adam_three_steps_against_oracle(ctx):
    """Three GPU training steps on one batch: after each step the GPU's parameters equal the
    oracle's Adam (bias corrections at t = 1, 2, 3) applied to the GPU's own gradients."""
    import torch
    _say("case: three Adam steps against the oracle optimiser")
    params = mlp.init_params(9)
    v = flat(params)
    ctx.mlp_set_params(_t(v, torch.float32))
    rng = np.random.default_rng(10)
    m = 1024
    X = rng.normal(size=(m, 64))
    X[:, 50:] = 0
    bits = (np.asarray(bf16_round(X), np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    y = rng.normal(size=m)
    lr = 3e-4
    ref = [v.astype(np.float64)]
    opt = mlp.Adam(ref, lr=lr)
    big = np.ones(v.shape[0], bool)
    for t in range(3):
        ctx.mlp_train_step(_t(bits, torch.int16), _t(y, torch.float32), _t(np.arange(m), torch.int32), lr)
        g = ctx.mlp_last_grads().cpu().numpy().astype(np.float64)
        big &= np.abs(g) > 1e-5
        opt.step(ref, [g])
        gpu = ctx.mlp_get_params().cpu().numpy().astype(np.float64)
        # float32 master weights: |p| * 2^-23 per rounding, a few roundings per step
        tolp = 4e-7 * np.abs(ref[0]) + 1e-3 * lr
        bad = np.abs(gpu - ref[0])[big] > tolp[big]
        _say(f"  step {t + 1}: max |gpu - oracle| {np.abs(gpu - ref[0])[big].max():.3e} over {big.sum()} params")
        assert not bad.any(), t
