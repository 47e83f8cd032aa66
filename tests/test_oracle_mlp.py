"""Pins of the FP64 warm-start oracle (oracle/mlp.py): neighbour search on a
lattice with known shells, GELU against math.erf, the backward pass against
central finite differences and against torch autograd (CPU, float64), and one
Adam step in closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_knn_on_lattice():
    """Cubic lattice, interior site: 6 face neighbours at h, then 12 edge neighbours at
    h sqrt(2); the first 16 are the 6 face ones and the 10 lowest-index edge ones."""
    m, h = 5, 1.0  # integer coordinates: equal distances are exactly equal, ties go by index
    g = np.arange(m) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    i = (2 * m + 2) * m + 2
    nb = mlp.knn(P, 16, idx=[i])[0]
    d = np.linalg.norm(P[nb] - P[i], axis=1)
    assert np.allclose(d[:6], h) and np.allclose(d[6:], h * math.sqrt(2))
    face = sorted(int(j) for j in range(len(P)) if abs(np.linalg.norm(P[j] - P[i]) - h) < 1e-12)
    edge = sorted(int(j) for j in range(len(P)) if abs(np.linalg.norm(P[j] - P[i]) - h * math.sqrt(2)) < 1e-12)
    assert sorted(nb[:6].tolist()) == face
    assert nb[6:].tolist() == edge[:10]


def test_features_layout():
    rng = np.random.default_rng(0)
    P = rng.uniform(size=(40, 3))
    nu = rng.uniform(1e-4, 2e-4, size=40)
    psi = rng.uniform(1e-3, 2e-3, size=40)
    V = rng.uniform(0.5e-4, 2.5e-4, size=40)
    nb = mlp.knn(P)
    F = mlp.features(P, psi, nu, nb, V)
    s = np.cbrt(nu)
    i = 7
    assert np.allclose(F[i, :3], (P[nb[i, 0]] - P[i]) / s[i])
    assert np.allclose(F[i, 45:48], (P[nb[i, 15]] - P[i]) / s[i])
    assert F[i, 48] == pytest.approx(psi[i] / s[i] ** 2)
    assert F[i, 49] == pytest.approx(nu[i] / nu.mean())
    assert F[i, 50] == pytest.approx((nu[i] - V[i]) / nu[i])
    j = nb[i, 12]
    assert F[i, 63] == pytest.approx((nu[j] - V[j]) / nu[j])


def test_gelu_closed_form():
    xs = np.linspace(-6, 6, 101)
    ref = np.array([0.5 * x * (1 + math.erf(x / math.sqrt(2))) for x in xs])
    assert np.allclose(mlp.gelu(xs), ref, rtol=1e-14, atol=1e-300)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (mlp.gelu(xs + h) - mlp.gelu(xs - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(xs), fd, atol=1e-8)


def _data(seed, m=64):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(m, mlp.D_IN))
    X[:, 50:] = 0
    y = rng.normal(size=m)
    return X, y


def test_backward_finite_differences():
    params = mlp.init_params(1)
    X, y = _data(2)
    loss, grads = mlp.loss_and_grads(params, X, y)
    rng = np.random.default_rng(3)
    for li in range(8):
        p = params[li]
        for _ in range(4):
            k = tuple(rng.integers(0, s) for s in p.shape)
            old = p[k]
            h = 1e-6
            p[k] = old + h
            lp, _ = mlp.loss_and_grads(params, X, y)
            p[k] = old - h
            lm, _ = mlp.loss_and_grads(params, X, y)
            p[k] = old
            fd = (lp - lm) / (2 * h)
            assert grads[li][k] == pytest.approx(fd, rel=1e-5, abs=1e-9), (li, k)


def test_backward_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    params = mlp.init_params(4)
    X, y = _data(5, m=128)
    loss, grads = mlp.loss_and_grads(params, X, y)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    h = torch.tensor(X)
    for li in range(4):
        h = h @ tp[2 * li] + tp[2 * li + 1]
        if li < 3:
            h = torch.nn.functional.gelu(h)
    tl = torch.mean((h[:, 0] - torch.tensor(y)) ** 2)
    tl.backward()
    assert float(tl) == pytest.approx(loss, rel=1e-12)
    for g, t in zip(grads, tp):
        assert np.allclose(g, t.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_first_step_closed_form():
    """First step: m = (1-b1) g, v = (1-b2) g^2, bias-corrected update = lr g / (|g| + eps)."""
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -0.01, 0.0])]
    opt = mlp.Adam(p, lr=0.1)
    opt.step(p, g)
    expect = np.array([1.0, -2.0, 0.5]) - 0.1 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.allclose(p[0], expect, rtol=1e-12)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias corrections make every step exactly
    lr g / (|g| + eps): m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2 (pins t > 1)."""
    p = [np.array([0.25, -1.5, 3.0])]
    g = np.array([0.02, -0.7, 1e-4])
    opt = mlp.Adam(p, lr=0.05)
    for t in range(1, 8):
        opt.step(p, [g.copy()])
        expect = np.array([0.25, -1.5, 3.0]) - t * 0.05 * g / (np.abs(g) + 1e-8)
        assert np.allclose(p[0], expect, rtol=1e-12, atol=1e-14), t


def test_adam_alternating_gradient_hand_values():
    """Gradients g, -g, g: the bias-corrected first moments are g, -0.01 g / 0.19 and
    0.091 g / 0.271 (worked by hand), and sqrt of the corrected second moment is |g|."""
    g0 = np.array([0.5, -0.2])
    p = [np.zeros(2)]
    opt = mlp.Adam(p, lr=1.0, eps=0.0)
    mhat = [1.0, -0.01 / 0.19, 0.091 / 0.271]
    total = np.zeros(2)
    for t, s in enumerate([1.0, -1.0, 1.0]):
        opt.step(p, [s * g0])
        total -= mhat[t] * g0 / np.abs(g0)
        assert np.allclose(p[0], total, rtol=1e-12), t
