"""Plain FP64 reference of the facet-law surrogate MLP (9 -> 64 -> 64 -> 64
-> 3, tanh) and its backpropagation.  TEST INFRASTRUCTURE: used to check the
GPU training kernels' forward pass and gradients.

Parameters: one flat vector, weights stored [out][in]:
W1[64][9] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3].
Loss: sum over samples of sum_j (y_j - target_j)^2, divided by `norm`
(the number of samples unless given).

Rounding points.  The surrogate runs its matrix products on BF16 operands
with wider accumulation, so a value is rounded to BF16 wherever it becomes a
matrix operand: the inputs x, the weights W (not the biases), the hidden
activations h after tanh, the output gradient dL/dy and the pre-activation
gradients dz.  `rnd` is the rounding applied at those points; with
rnd=None every value stays FP64, which is the plain backpropagation the
finite-difference pin checks.  bf16_points() gives the BF16 rounding.
"""
import numpy as np

SIZES = [(64, 9), (64, 64), (64, 64), (3, 64)]
N_PARAMS = sum(o * i + o for o, i in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, k = [], 0
    for o, i in SIZES:
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)


def bf16_points(a):
    """The rounding of matrix operands: FP64 -> FP32 -> BF16 (the GPU forms
    each such value in FP32 before rounding it)."""
    return bf16_round(a)


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def init_params(rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    layers = []
    for o, i in SIZES:
        s = 1.0 / np.sqrt(i)
        layers.append((rng.uniform(-s, s, (o, i)), rng.uniform(-s, s, o)))
    return pack(layers)


def _layers(p, rnd):
    return [(rnd(W), np.asarray(b, dtype=np.float64)) for W, b in unpack(p)]


def _forward_all(L, x, rnd):
    hs = [rnd(x)]
    for W, b in L[:-1]:
        hs.append(rnd(np.tanh(hs[-1] @ W.T + b)))
    W4, b4 = L[-1]
    return hs, hs[-1] @ W4.T + b4


def forward(p, x, rnd=None, magnitude=False):
    """Network output y (n, 3); with magnitude=True also |h3| |W4|^T + |b4|,
    the scale an output's rounding differences are measured against."""
    rnd = rnd or _ident
    L = _layers(p, rnd)
    hs, y = _forward_all(L, np.asarray(x, dtype=np.float64), rnd)
    if not magnitude:
        return y
    W4, b4 = L[-1]
    return y, np.abs(hs[-1]) @ np.abs(W4).T + np.abs(b4)


def loss_and_grad(p, x, t, rnd=None, norm=None, magnitude=False):
    """Squared-error loss / norm and its gradient by backpropagation.

    With magnitude=True a third value is returned: for every parameter the
    sum of the absolute values of the terms its gradient adds up
    (|dz|^T |h| for a weight, sum |dz| for a bias), the scale an entry's
    rounding differences are measured against."""
    rnd = rnd or _ident
    L = _layers(p, rnd)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    norm = float(B if norm is None else norm)
    hs, y = _forward_all(L, x, rnd)
    r = y - t
    loss = np.sum(r * r) / norm
    dz = rnd(2.0 * r / norm)                       # dL/dy
    grads, mags = [None] * 4, [None] * 4
    for li in (3, 2, 1, 0):
        W, _ = L[li]
        grads[li] = (dz.T @ hs[li], dz.sum(0))
        mags[li] = (np.abs(dz).T @ np.abs(hs[li]), np.abs(dz).sum(0))
        if li > 0:
            dz = rnd((dz @ W) * (1.0 - hs[li] ** 2))
    if magnitude:
        return loss, pack(grads), pack(mags)
    return loss, pack(grads)
