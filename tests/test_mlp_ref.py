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


class _RoundedTanh:
    """tanh whose output is rounded to BF16 and whose incoming gradient is
    rounded to BF16 after the tanh derivative (taken at the rounded value)."""

    @staticmethod
    def make():
        class F(torch.autograd.Function):
            @staticmethod
            def forward(ctx, z):
                h = torch.from_numpy(M.bf16_round(torch.tanh(z).numpy()))
                ctx.save_for_backward(h)
                return h

            @staticmethod
            def backward(ctx, g):
                (h,) = ctx.saved_tensors
                return torch.from_numpy(M.bf16_round((g * (1 - h * h)).numpy()))
        return F.apply


def _rounded_grad(g):
    class F(torch.autograd.Function):
        @staticmethod
        def forward(ctx, y):
            return y.clone()

        @staticmethod
        def backward(ctx, gy):
            return torch.from_numpy(M.bf16_round(gy.numpy()))
    return F.apply(g)


def test_bf16_backprop_equals_autograd_with_rounded_operands():
    """The BF16 rounding points of the reference (inputs, weights,
    activations, dL/dy, dz) against torch autograd in FP64 over a network
    whose tanh layers and output round in the same places (custom functions;
    weights rounded with a straight-through gradient)."""
    rng = np.random.default_rng(4)
    p = M.init_params(rng).astype(np.float32).astype(np.float64)
    x = rng.normal(size=(96, 9))
    t = rng.normal(size=(96, 3))
    norm = 128.0
    loss, g = M.loss_and_grad(p, x, t, rnd=M.bf16_points, norm=norm)
    act = _RoundedTanh.make()
    layers = M.unpack(p)
    params = []
    for W, b in layers:
        params += [torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)]
    h = torch.from_numpy(M.bf16_round(x))
    for k in range(3):
        Wr = params[2 * k] + (torch.from_numpy(M.bf16_round(params[2 * k].detach().numpy())) - params[2 * k]).detach()
        h = act(h @ Wr.T + params[2 * k + 1])
    W4r = params[6] + (torch.from_numpy(M.bf16_round(params[6].detach().numpy())) - params[6]).detach()
    y = _rounded_grad(h @ W4r.T + params[7])
    lt = ((y - torch.from_numpy(t)) ** 2).sum() / norm
    lt.backward()
    ga = np.concatenate([q.grad.numpy().ravel() for q in params])
    assert abs(float(lt.detach()) - loss) <= 1e-12 * loss
    assert np.abs(ga - g).max() <= 1e-12 * np.abs(g).max()
    # the rounding does act: the BF16 gradient differs from the plain one
    _, g0 = M.loss_and_grad(p, x, t, norm=norm)
    assert np.abs(g0 - g).max() > 1e-4 * np.abs(g).max()


def test_gradient_magnitudes_bound_the_gradient():
    """The per-entry term magnitudes are sums of |terms|: they bound |grad|
    and equal it where every term has one sign (an all-positive chain: zero
    weights, positive biases and targets below the outputs)."""
    rng = np.random.default_rng(5)
    p = M.init_params(rng)
    x = rng.normal(size=(40, 9))
    t = rng.normal(size=(40, 3))
    _, g, mg = M.loss_and_grad(p, x, t, rnd=M.bf16_points, magnitude=True)
    assert np.all(mg >= np.abs(g))
    assert np.all(mg > 0)
    y, my = M.forward(p, x, rnd=M.bf16_points, magnitude=True)
    assert np.all(my >= np.abs(y) - 1e-12 * np.abs(y).max())
    layers = [(np.zeros_like(W), np.abs(b) + 0.1) for W, b in M.unpack(p)]
    q = M.pack(layers)
    xp = np.abs(x)
    _, g, mg = M.loss_and_grad(q, xp, np.full((40, 3), -5.0), magnitude=True)
    wsel = np.concatenate([np.concatenate([np.ones(o * i), np.ones(o)]) for o, i in M.SIZES]) > 0
    assert np.allclose(np.abs(g[wsel]), mg[wsel], rtol=1e-12, atol=0)
