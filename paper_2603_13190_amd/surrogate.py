"""Facet-law surrogate pipeline: capture (input, exact-law target) samples
from FP64 runs of the solver, normalise, train the MLP on the GPU with the
library's BF16 MFMA kernels, and install it into a mixed-precision system.

The exact law stays both the fallback (facets leaving the envelope are
handed back for good) and the reference for the surrogate's error.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import ldpm

N_PARAMS = 9155
SIZES = [(64, 9), (64, 64), (64, 64), (3, 64)]


def init_params(seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in SIZES:
        s = 1.0 / np.sqrt(i)
        parts.append(rng.uniform(-s, s, o * i))
        parts.append(rng.uniform(-s, s, o))
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class Model:
    params: np.ndarray
    x_mean: np.ndarray
    x_scale: np.ndarray
    y_scale: np.ndarray
    box_lo: np.ndarray
    box_hi: np.ndarray
    y_dead: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    y_tau: float = 0.0
    train_loss: float = float("nan")
    holdout_rmse: np.ndarray = None
    n_train: int = 0

    def install(self, system, kappa_t=1.1, kappa_c=0.9, damage_max=0.05):
        system.set_surrogate(self.params, self.x_mean, self.x_scale, self.y_scale,
                             self.box_lo, self.box_hi, kappa_t, kappa_c, damage_max, self.y_dead,
                             self.y_tau)


def capture(sysd, steps, facet_stride=7, step_stride=50, capacity=2_000_000, seed_offset=0,
            kappa_t=1.1, kappa_c=0.9, damage_max=0.05):
    """Run the FP64 solver for `steps` and record in-envelope samples."""
    g = ldpm.System(sysd, precision="fp64")
    g.capture_begin(capacity, facet_stride, seed_offset % facet_stride, step_stride,
                    kappa_t, kappa_c, damage_max)
    g.step(steps)
    rows = g.capture_end()
    g.close()
    if rows["offered"] > capacity:
        raise ValueError(f"capture offered {rows['offered']} rows for a capacity of {capacity}: "
                         "the kept subset would depend on arrival order")
    return rows


def fit(samples, seed=0, steps=3000, batch=8192, lr=2e-3, holdout=0.1, tau=1e-2,
        zero_rel=1e-9, dead_quantile=0.999):
    """Normalise, split, train on the GPU; returns a Model.

    The target is the residual relative to s = |t_old + E de| + tau (MPa),
    so the network's error scales with each facet's own traction; the output
    dead zone is the `dead_quantile` quantile of |prediction| over held-out
    rows whose exact residual vanishes (|r| <= zero_rel s)."""
    x = np.concatenate([s["x"] for s in samples]).astype(np.float64)
    y = np.concatenate([s["y"] for s in samples]).astype(np.float64)
    sc = np.concatenate([s["s"] for s in samples]).astype(np.float64) + tau
    rng = np.random.default_rng(seed)
    perm = rng.permutation(x.shape[0])
    x, y, sc = x[perm], y[perm], sc[perm]
    yr = y / sc[:, None]
    nh = int(holdout * x.shape[0])
    xh, yh, sh, xt, yt = x[:nh], yr[:nh], sc[:nh], x[nh:], yr[nh:]
    mean = xt.mean(0)
    std = xt.std(0)
    scale = 1.0 / np.where(std > 0, std, 1.0)
    ysd = yt.std(0)
    ysc = np.where(ysd > 0, ysd, 1.0)
    norm = lambda a: ((a - mean) * scale).astype(np.float32)
    tr = ldpm.Mlp(init_params(seed))
    tr.set_data(norm(xt), (yt / ysc).astype(np.float32))
    loss = tr.train(steps, batch=batch, lr=lr)
    pred = tr.forward(norm(xh)).astype(np.float64) * ysc if nh > 0 else np.zeros((0, 3))
    # held-out error in MPa
    rmse = np.sqrt(np.mean(((pred - yh) * sh[:, None]) ** 2, axis=0)) if nh > 0 else np.zeros(3)
    dead = np.zeros(3)
    for c in range(3):
        z = np.abs(yh[:, c]) <= zero_rel
        if z.sum() >= 100:
            dead[c] = np.quantile(np.abs(pred[z, c]), dead_quantile)
    params = tr.params()
    tr.close()
    return Model(params=params, x_mean=mean, x_scale=scale, y_scale=ysc, box_lo=x.min(0),
                 box_hi=x.max(0), y_dead=dead, y_tau=tau, train_loss=loss, holdout_rmse=rmse,
                 n_train=xt.shape[0])
