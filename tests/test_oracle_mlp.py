"""Pins of the MLP oracle: BF16 rounding rule, finite-difference gradients of
the float64 network, and Adam against its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_round_ties_to_even_and_exact_values():
    # exactly representable values are unchanged
    for v in [1.0, -2.0, 0.5, 3.0, 1.0 + 2 ** -7, 0.0]:
        assert mlp.bf16_round(np.array([v]))[0] == v
    # halfway cases: 1 + 2^-8 lies between 1 and 1 + 2^-7 -> ties to even (1.0)
    assert mlp.bf16_round(np.array([1.0 + 2 ** -8]))[0] == 1.0
    # 1 + 3*2^-8 lies between 1 + 2^-7 (odd mantissa) and 1 + 2^-6 -> rounds up
    assert mlp.bf16_round(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    x = np.random.default_rng(0).normal(size=1000)
    q = mlp.bf16_round(x)
    assert np.all(np.abs(q - x) <= 2 ** -8 * np.abs(x) + 1e-300)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(64, 32, 32, 64, seed=2)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.1 * rng.normal(size=p[k].shape)
    X = rng.normal(size=(5, 64))
    T = rng.normal(size=(5, 64))
    Y, cache = mlp.forward(p, X, emulate=False)
    g = mlp.backward(p, cache, Y, T, emulate=False)
    eps = 1e-6
    for k in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=6, replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss(mlp.forward(p, X, emulate=False)[0], T)
            flat[idx] = old - eps
            lm = mlp.loss(mlp.forward(p, X, emulate=False)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert g[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-10)


def test_emulated_gradients_close_to_float64():
    rng = np.random.default_rng(3)
    p = mlp.init_params(64, 32, 32, 64, seed=4)
    X = rng.normal(size=(8, 64))
    T = rng.normal(size=(8, 64))
    Y, c = mlp.forward(p, X, emulate=False)
    g = mlp.backward(p, c, Y, T, emulate=False)
    Yq, cq = mlp.forward(p, X, emulate=True)
    gq = mlp.backward(p, cq, Yq, T, emulate=True)
    for k in g:
        assert np.linalg.norm(gq[k] - g[k]) <= 2e-2 * np.linalg.norm(g[k])


@pytest.mark.parametrize("shape,B", [((300, 96, 80, 200), 33), ((2600, 64, 64, 1950), 64)])
def test_emulated_gradients_close_to_float64_with_shared_relu_decisions(shape, B):
    """Deep products (K = 2,600) and hidden layers where a few pre-activations
    sit within the BF16 rounding error of zero: with the ReLU decisions of the
    BF16 pass, the float64 gradients differ only by operand rounding
    (normwise <= 2e-2, about 1e-3 per rounding stage)."""
    rng = np.random.default_rng(12)
    p = mlp.init_params(*shape, seed=11)
    for k in ["b1", "b2", "b3"]:
        p[k] = 0.05 * rng.normal(size=p[k].shape)
    X = rng.normal(size=(B, shape[0]))
    T = rng.normal(size=(B, shape[3]))
    Yq, cq = mlp.forward(p, X, emulate=True)
    gq = mlp.backward(p, cq, Yq, T, emulate=True)
    Y, c = mlp.forward(p, X, emulate=False, masks=(cq[1], cq[3]))
    g = mlp.backward(p, c, Y, T, emulate=False)
    for k in g:
        assert np.linalg.norm(gq[k] - g[k]) <= 2e-2 * np.linalg.norm(g[k]), k
    # with its own decisions the float64 pass is the plain network
    Y0, c0 = mlp.forward(p, X, emulate=False)
    assert np.array_equal(c0[1], (X @ p["W1"].T + p["b1"]) > 0)


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step moves every coordinate by
    lr * g / (|g| + eps) ~ lr * sign(g)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    st = {}
    mlp.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01 * 1e-3 / (1e-3 + 1e-8)])


def test_training_reduces_loss_on_a_linear_map():
    rng = np.random.default_rng(5)
    M = rng.normal(size=(16, 16)) * 0.3
    p = mlp.init_params(16, 32, 32, 16, seed=6)
    st = {}
    X = rng.normal(size=(64, 16))
    T = X @ M.T
    l0 = mlp.loss(mlp.forward(p, X)[0], T)
    for _ in range(200):
        Y, c = mlp.forward(p, X)
        mlp.adam_step(p, mlp.backward(p, c, Y, T), st, lr=3e-3)
    assert mlp.loss(mlp.forward(p, X)[0], T) < 0.2 * l0
