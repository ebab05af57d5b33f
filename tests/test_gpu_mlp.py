"""GPU warm-start network against the NumPy oracle with the same BF16
rounding points: forward outputs, gradients (P17) and Adam steps."""
import numpy as np
import pytest

from oracle import mlp as omlp
from pd_inputs.mlp_init import mlp_init_params, pack, unpack
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("shape,B", [((64, 32, 32, 64), 8), ((300, 96, 80, 200), 33),
                                     ((2600, 64, 64, 1950), 64)])
def test_mlp_forward_and_gradients_match_oracle(shape, B):
    import torch
    from paper_2008_01541_amd import MLP
    n_in, n_h1, n_h2, n_out = shape
    p = mlp_init_params(n_in, n_h1, n_h2, n_out, seed=11)
    rng = np.random.default_rng(12)
    for k in ["b1", "b2", "b3"]:
        p[k] = 0.05 * rng.normal(size=p[k].shape)
    flat = pack(p)
    p32 = unpack(flat, *shape)                  # the exact FP32 values the GPU holds
    X = rng.normal(size=(B, n_in)).astype(np.float32)
    T = rng.normal(size=(B, n_out)).astype(np.float32)
    net = MLP(n_in, n_h1, n_h2, n_out, max_batch=64, params_flat=flat)
    y = torch.empty(B * n_out, dtype=torch.float32, device="cuda")
    net.forward(dev(X), y)
    Y_or, cache = omlp.forward(p32, X.astype(np.float64), emulate=True)
    assert _rel(host(y, (B, n_out)), Y_or) <= 1e-4
    g, loss = net.gradients(dev(X), dev(T))
    g_or = omlp.backward(p32, cache, Y_or, T.astype(np.float64), emulate=True)
    gd = unpack(g, *shape)
    for k in g_or:
        assert _rel(gd[k], g_or[k]) <= 1e-4, k
    assert loss == pytest.approx(omlp.loss(Y_or, T), rel=1e-4)
    # P17 against pure float64: the float64 network takes the ReLU decisions
    # of the BF16 pass (a decision made by floating point is taken in the same
    # precision on both sides); what remains is BF16 operand rounding, a few
    # unit roundoffs (2^-8) normwise.
    Y64, c64 = omlp.forward(p32, X.astype(np.float64), emulate=False, masks=(cache[1], cache[3]))
    g64 = omlp.backward(p32, c64, Y64, T.astype(np.float64), emulate=False)
    for k in g64:
        assert _rel(gd[k], g64[k]) <= 2e-2, k


def test_mlp_adam_steps_match_oracle():
    import torch
    from paper_2008_01541_amd import MLP
    shape = (120, 48, 40, 90)
    p = mlp_init_params(*shape, seed=21)
    flat = pack(p)
    p_or = unpack(flat, *shape)
    rng = np.random.default_rng(22)
    net = MLP(*shape, max_batch=16, params_flat=flat)
    st = {}
    for it in range(3):
        X = rng.normal(size=(16, shape[0])).astype(np.float32)
        T = rng.normal(size=(16, shape[3])).astype(np.float32)
        loss = net.train_step(dev(X), dev(T), lr=1e-3)
        Y, c = omlp.forward(p_or, X.astype(np.float64))
        assert loss == pytest.approx(omlp.loss(Y, T), rel=1e-3)
        omlp.adam_step(p_or, omlp.backward(p_or, c, Y, T.astype(np.float64)), st, lr=1e-3)
    got = unpack(net.params(), *shape)
    for k in p_or:
        # Adam normalises steps, so compare the accumulated update, not raw values
        upd_g = got[k] - unpack(flat, *shape)[k]
        upd_o = p_or[k] - unpack(flat, *shape)[k]
        assert _rel(upd_g, upd_o) <= 5e-2, k
