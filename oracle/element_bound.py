"""Element bound of the stable explicit step, plain NumPy, FP64.

TEST INFRASTRUCTURE ONLY: the reference for the GPU element bound.

The paper sets the explicit step from an eigenvalue analysis of each
tetrahedron (section on free vibrations in the linear elastic regime): the
largest eigenvalue of K_e v = lambda M_e v over the elements bounds the
assembled system's largest eigenvalue, and dt = fraction * 2 / sqrt(lambda).
Here K_e is the elastic stiffness of tetrahedron e, the sum over its 12
facets of (A / l) B^T D B with the jump [[u]] = B q = u_J - [c^J]x th_J -
u_I + [c^I]x th_I (eq. strain1), c^J = c^I - l n and D = E0 (alpha 1 +
(1 - alpha) n n^T); M_e is the tetrahedron's share of the lumped masses of
its four nodes (its part of each node's cell: rho V three times, then the
diagonal of rho (tr S 1 - S)).  DoFs per node (u_x, u_y, u_z, th_x, th_y,
th_z), nodes in the tetrahedron's own order.
"""
from __future__ import annotations

import numpy as np

from .implicit import _skew


def element_stiffness(tets, facet_I, facet_J, cI, n, A, L, E0, alpha):
    """K_e (T, 24, 24) from tet-major facet arrays (facet 12 t + k belongs to
    tetrahedron t)."""
    tets = np.asarray(tets, dtype=np.int64)
    T = tets.shape[0]
    I = np.asarray(facet_I, dtype=np.int64).reshape(T, 12)
    J = np.asarray(facet_J, dtype=np.int64).reshape(T, 12)
    cI = np.asarray(cI, dtype=np.float64).reshape(T, 12, 3)
    n = np.asarray(n, dtype=np.float64).reshape(T, 12, 3)
    A = np.asarray(A, dtype=np.float64).reshape(T, 12)
    L = np.asarray(L, dtype=np.float64).reshape(T, 12)
    K = np.zeros((T, 24, 24))
    rows = np.arange(T)
    eye = np.broadcast_to(np.eye(3), (T, 3, 3))
    for k in range(12):
        a = np.argmax(tets == I[:, k:k + 1], axis=1)      # position of I within the tetrahedron
        b = np.argmax(tets == J[:, k:k + 1], axis=1)
        cJ = cI[:, k] - L[:, k, None] * n[:, k]
        BI = np.concatenate([-eye, _skew(cI[:, k])], 2)     # (T, 3, 6)
        BJ = np.concatenate([eye, -_skew(cJ)], 2)
        nk = n[:, k]
        D = E0 * (alpha * np.eye(3)[None] + (1.0 - alpha) * nk[:, :, None] * nk[:, None, :])
        w = (A[:, k] / L[:, k])[:, None, None]
        B = (BI, BJ)
        pos = (a, b)
        for s in range(2):
            for r in range(2):
                Kb = w * np.einsum("tki,tkl,tlj->tij", B[s], D, B[r])
                for i in range(6):
                    for j in range(6):
                        K[rows, 6 * pos[s] + i, 6 * pos[r] + j] += Kb[:, i, j]
    return K


def element_lambda_max(K, share):
    """Largest eigenvalue of W K_e W, W = diag(share)^(-1/2), per element
    (numpy.linalg.eigvalsh); share (T, 4, 6)."""
    m = np.asarray(share, dtype=np.float64).reshape(-1, 24)
    w = 1.0 / np.sqrt(m)
    Kh = K * w[:, :, None] * w[:, None, :]
    return np.linalg.eigvalsh(Kh)[:, -1]
