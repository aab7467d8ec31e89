"""GPU training kernels of the surrogate MLP (BF16 MFMA, FP32 accumulate)
against the FP64 reference with the same BF16-rounded parameters/inputs."""
import numpy as np
import pytest

import oracle.mlp_ref as M

pytestmark = pytest.mark.gpu


def trainer(p):
    from paper_2603_13190_amd.ldpm import Mlp
    return Mlp(p)


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 9)).astype(np.float32)
    y = np.stack([np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2], np.tanh(x[:, 3] - x[:, 4]),
                  0.3 * x[:, 5] ** 2 - 0.2 * x[:, 6] * x[:, 7] + 0.1 * x[:, 8]], 1).astype(np.float32)
    return x, y


def test_forward_matches_reference():
    rng = np.random.default_rng(3)
    p = M.init_params(rng).astype(np.float32)
    x, _ = _data(1000, 4)
    g = trainer(p).forward(x)
    ref = M.forward(M.bf16_round(p), M.bf16_round(x))
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    assert err < 2e-2, err


def test_gradient_matches_reference():
    rng = np.random.default_rng(5)
    p = M.init_params(rng).astype(np.float32)
    x, y = _data(256, 6)
    tr = trainer(p)
    tr.set_data(x, y)
    loss, g = tr.grad(256, 0)
    lref, gref = M.loss_and_grad(M.bf16_round(p), M.bf16_round(x), y.astype(np.float64))
    assert abs(loss - lref) < 2e-2 * lref
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    assert err < 3e-2, err
    # every layer, not only the largest one
    k = 0
    for o, i in M.SIZES:
        for n in (o * i, o):
            seg = slice(k, k + n)
            e = np.linalg.norm(g[seg] - gref[seg]) / max(np.linalg.norm(gref[seg]), 1e-12)
            assert e < 6e-2, (o, i, n, e)
            k += n
    # bitwise reproducible (fixed-order reduction over blocks)
    loss2, g2 = tr.grad(256, 0)
    assert np.array_equal(g, g2) and loss == loss2


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    p = M.init_params(rng).astype(np.float32)
    x, y = _data(32768, 8)
    tr = trainer(p)
    tr.set_data(x, y)
    l0, _ = tr.grad(4096, 0)
    tr.train(400, batch=4096, lr=3e-3)
    l1, _ = tr.grad(4096, 0)
    assert l1 < 0.1 * l0, (l0, l1)
    # trained parameters evaluated by the reference agree with the GPU forward
    pt = tr.params()
    yg = tr.forward(x[:2000])
    yr = M.forward(M.bf16_round(pt), M.bf16_round(x[:2000]))
    assert np.linalg.norm(yg - yr) / np.linalg.norm(yr) < 2e-2
