"""FP64 reference of the learned warm start (TEST INFRASTRUCTURE ONLY).

The warm start predicts each site's weight increment for the next solve from its
local neighbourhood. Inputs per site i (64 values):
  * the offsets (p_j - p_i) / s_i of its 16 nearest sites j (ascending
    (distance, index)), s_i = nu_i^(1/3)                                 -> 48
  * psi_prev_i / s_i^2                                                    -> 1
  * nu_i / mean(nu)                                                       -> 1
  * (nu - V) / nu under the previous weights, of site i and of its 13
    nearest sites (V: the cells at the current positions, weights psi_prev) -> 14
Network: 64 -> 128 -> 128 -> 128 -> 1, GELU (erf form) after each hidden layer,
linear output = (psi_new_i - psi_prev_i) / s_i^2.
Training: mean squared error, Adam (beta1 0.9, beta2 0.999, eps 1e-8).
Parity pins live in tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import math

import numpy as np

D_IN, D_HID, N_NEI = 64, 128, 16
LAYERS = [(D_IN, D_HID), (D_HID, D_HID), (D_HID, D_HID), (D_HID, 1)]


def knn(P: np.ndarray, k: int = N_NEI, idx=None) -> np.ndarray:
    """k nearest other sites of each site (brute force), ordered by (squared distance, index)."""
    n = P.shape[0]
    idx = np.arange(n) if idx is None else np.asarray(idx)
    out = np.empty((len(idx), k), np.int64)
    for c, i in enumerate(idx):
        d2 = ((P - P[i]) ** 2).sum(1)
        d2[i] = np.inf
        order = np.lexsort((np.arange(n), d2))
        out[c] = order[:k]
    return out


def features(P: np.ndarray, psi_prev: np.ndarray, nu: np.ndarray, nbr: np.ndarray, V: np.ndarray,
             idx=None) -> np.ndarray:
    """The 64 inputs of each site (rows follow idx, default all sites); V = volumes of all
    cells at the current positions under psi_prev."""
    n = P.shape[0]
    idx = np.arange(n) if idx is None else np.asarray(idx)
    s = np.cbrt(nu[idx])
    X = np.zeros((len(idx), D_IN))
    off = (P[nbr] - P[idx][:, None, :]) / s[:, None, None]
    X[:, :3 * N_NEI] = off.reshape(len(idx), 3 * N_NEI)
    X[:, 3 * N_NEI] = psi_prev[idx] / s ** 2
    X[:, 3 * N_NEI + 1] = nu[idx] / nu.mean()
    res = (nu - V) / nu
    X[:, 50] = res[idx]
    X[:, 51:64] = res[nbr[:, :13]]
    return X


def gelu(x):
    """GELU, erf form: x * Phi(x)."""
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def init_params(seed: int = 0):
    """He-style normal init for the hidden layers, small output layer; float64."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in LAYERS:
        W = rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b))
        if b == 1:
            W *= 0.1
        params += [W, np.zeros(b)]
    return params


def forward(params, X):
    """Returns the output [m] and the cache of pre-activations for the backward pass."""
    h = X
    cache = []
    for li in range(4):
        W, b = params[2 * li], params[2 * li + 1]
        z = h @ W + b
        cache.append((h, z))
        h = gelu(z) if li < 3 else z
    return h[:, 0], cache


def loss_and_grads(params, X, y):
    """Mean squared error and its gradient with respect to every parameter."""
    out, cache = forward(params, X)
    m = X.shape[0]
    err = out - y
    loss = float(np.mean(err ** 2))
    grads = [None] * 8
    dz = (2.0 / m) * err[:, None]
    for li in range(3, -1, -1):
        h, z = cache[li]
        W = params[2 * li]
        grads[2 * li] = h.T @ dz
        grads[2 * li + 1] = dz.sum(0)
        if li > 0:
            dh = dz @ W.T
            dz = dh * gelu_grad(cache[li - 1][1])
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)
