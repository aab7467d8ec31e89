"""Plain FP64 reference of the facet-law surrogate MLP (9 -> 64 -> 64 -> 64
-> 3, tanh) and its backpropagation.  TEST INFRASTRUCTURE: used to check the
GPU training kernels' forward pass and gradients.

Parameters: one flat vector, weights stored [out][in]:
W1[64][9] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3].
Loss: mean over samples of sum_j (y_j - target_j)^2.
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


def init_params(rng):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    layers = []
    for o, i in SIZES:
        s = 1.0 / np.sqrt(i)
        layers.append((rng.uniform(-s, s, (o, i)), rng.uniform(-s, s, o)))
    return pack(layers)


def forward(p, x):
    L = unpack(p)
    h = np.asarray(x, dtype=np.float64)
    for W, b in L[:-1]:
        h = np.tanh(h @ W.T + b)
    W, b = L[-1]
    return h @ W.T + b


def loss_and_grad(p, x, t):
    """Mean squared-error loss and its gradient by backpropagation."""
    L = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    hs = [x]
    for W, b in L[:-1]:
        hs.append(np.tanh(hs[-1] @ W.T + b))
    W4, b4 = L[-1]
    y = hs[-1] @ W4.T + b4
    r = y - t
    loss = np.sum(r * r) / B
    dy = 2.0 * r / B
    grads = [None] * 4
    grads[3] = (dy.T @ hs[3], dy.sum(0))
    dh = dy @ W4
    for li in (2, 1, 0):
        W, b = L[li]
        dz = dh * (1.0 - hs[li + 1] ** 2)
        grads[li] = (dz.T @ hs[li], dz.sum(0))
        dh = dz @ W
    return loss, pack(grads)
