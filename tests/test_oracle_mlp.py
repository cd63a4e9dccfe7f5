"""The FP64 cost-model oracle pinned by a hand-computed toy network, central
finite differences and the closed form of Adam's first steps."""
import numpy as np

from oracle import mlp as M


def test_sizes():
    assert M.n_params() == 7832


def test_toy_network_hand_computed(golden):
    g = golden("mlp_toy.json")
    sizes = tuple(g["sizes"])
    flat = M.flatten([g["W1"], g["b1"], g["W2"], g["b2"], g["W3"], g["b3"]])
    L, gr = M.grad(flat, np.array(g["x"], float), np.array(g["k"]), np.array(g["t"]), sizes)
    assert L == g["loss"]
    want = M.flatten([g["gW1"], g["gb1"], g["gW2"], g["gb2"], g["gW3"], g["gb3"]])
    assert np.array_equal(gr, want)


def test_gradient_matches_central_differences():
    r = np.random.default_rng(3)
    flat = M.he_uniform(7)
    X = r.normal(size=(6, 32))
    k = r.integers(0, 24, size=6)
    t = r.normal(size=6)
    _, g = M.grad(flat, X, k, t)
    h = 1e-6
    idx = np.concatenate([r.choice(M.n_params(), size=600, replace=False),
                          np.arange(M.n_params() - 24, M.n_params())])
    num = np.empty(idx.size)
    for j, p in enumerate(idx):
        e = np.zeros_like(flat)
        e[p] = h
        num[j] = (M.loss(flat + e, X, k, t) - M.loss(flat - e, X, k, t)) / (2 * h)
    err = np.linalg.norm(num - g[idx]) / np.linalg.norm(g[idx])
    assert err < 1e-6


def test_adam_first_steps_closed_form():
    g1 = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    m = np.zeros(4)
    v = np.zeros(4)
    p1, m, v = M.adam(p0, g1, m, v, 1, lr=0.1)
    # bias-corrected first step: m^ = g, v^ = g^2 -> step = lr g / (|g| + eps)
    assert np.allclose(p1, p0 - 0.1 * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-15)
    p2, m, v = M.adam(p1, g1, m, v, 2, lr=0.1)
    assert np.allclose(p2, p1 - 0.1 * g1 / (np.abs(g1) + 1e-8), rtol=0, atol=1e-12)


def test_training_reduces_loss():
    r = np.random.default_rng(0)
    X = r.normal(size=(512, 32))
    true = r.normal(size=(32, 24)) * 0.3
    k = r.integers(0, 24, size=512)
    t = (X @ true)[np.arange(512), k]
    flat = M.he_uniform(1)
    m = np.zeros_like(flat)
    v = np.zeros_like(flat)
    L0 = M.loss(flat, X, k, t)
    for s in range(1, 301):
        _, g = M.grad(flat, X, k, t)
        flat, m, v = M.adam(flat, g, m, v, s, lr=3e-3)
    assert M.loss(flat, X, k, t) < 0.2 * L0
