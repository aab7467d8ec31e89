"""Pins of the FP64 reference MLP used to check the GPU training kernels."""
import numpy as np
import torch

import oracle.mlp_ref as M


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(rng)
    x = rng.normal(size=(7, 9))
    t = rng.normal(size=(7, 3))
    _, g = M.loss_and_grad(p, x, t)
    idx = rng.choice(p.size, 300, replace=False)
    h = 1e-6
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (M.loss_and_grad(pp, x, t)[0] - M.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_loss_is_mean_squared_error_of_forward():
    rng = np.random.default_rng(1)
    p = M.init_params(rng)
    x = rng.normal(size=(11, 9))
    t = rng.normal(size=(11, 3))
    loss, _ = M.loss_and_grad(p, x, t)
    y = M.forward(p, x)
    assert abs(loss - np.mean(np.sum((y - t) ** 2, 1))) < 1e-12


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-6, 6, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875]])
    ours = M.bf16_round(a)
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)
