"""Plain tessellation of a tetrahedralised particle set into LDPM facets and
polyhedral cells, FP64.

TEST INFRASTRUCTURE ONLY: the reference for the GPU tessellation.

The paper's preprocessor (its cited mesh generator) is not available; its
LDPM geometry is built here with the construction the input generator
documents:
- on every tetrahedron edge (a, b) a point at mid-gap between the two
  particle surfaces, s = (|x_b - x_a| + r_a - r_b) / 2 from x_a, kept within
  [0.05, 0.95] of the edge;
- on every face the centroid of its three edge points; in the tetrahedron
  the centroid of its four face points;
- two facets per edge (a, b), one per face (a, b, c) through it: the
  triangle (edge point, point of that face, tetrahedron point), 12 per
  tetrahedron, ordered by edge (0,1), (0,2), (0,3), (1,2), (1,3), (2,3) and
  within an edge by the third node c in increasing order;
- facet k joins I = min and J = max of the edge's particle ids; n = (x_J -
  x_I) / l, l the edge length; the triangle's vector area is taken along n,
  A0 its magnitude and A = A0 n.n0 its projection (eq. balance); c^I runs
  from x_I to the triangle's centroid; m = normalise(n x e_k) with e_k the
  axis of the smallest |n_k| (the lowest such k);
- each cell is the union, over its facets, of the cones from the particle
  centre to the facet triangles; volume, first and second moments are the
  exact cone integrals, signed by whether the triangle faces away from the
  centre (outward normal of the I cell is +n, of the J cell -n).
Returns per facet (tet-major) I, J, cI, n, m, A, A0, l, per particle
mass, the diagonal and full inertia tensors about the centre, volume and
centroid offset, and per tetrahedron its share of its four nodes' lumped
masses (T, 4, 6: rho V three times, then the diagonal of rho (tr S - S) of
its cones).
"""
from __future__ import annotations

import numpy as np

EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _facet_list():
    out = []
    for a, b in EDGES:
        for c in range(4):
            if c != a and c != b:
                out.append((a, b, c))
    return out


def tessellate(x, diam, tets, rho):
    x = np.asarray(x, dtype=np.float64)
    r = 0.5 * np.asarray(diam, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    T = tets.shape[0]
    N = x.shape[0]
    # edge points
    ep = {}
    for a, b in EDGES:
        xa, xb = x[tets[:, a]], x[tets[:, b]]
        L = np.sqrt(((xb - xa) ** 2).sum(1))
        s = 0.5 * (L + r[tets[:, a]] - r[tets[:, b]])
        s = np.minimum(np.maximum(s, 0.05 * L), 0.95 * L)
        p = xa + (xb - xa) * (s / L)[:, None]
        ep[(a, b)] = p
        ep[(b, a)] = p
    # face points (face = the three nodes other than `miss`)
    fp = {}
    for miss in range(4):
        u, v, w = [c for c in range(4) if c != miss]
        fp[miss] = (ep[(u, v)] + ep[(u, w)] + ep[(v, w)]) / 3.0
    tp = (fp[0] + fp[1] + fp[2] + fp[3]) / 4.0
    F = 12 * T
    out = {k: None for k in ("I", "J", "cI", "n", "m", "A", "A0", "len")}
    I = np.zeros((T, 12), np.int64)
    J = np.zeros((T, 12), np.int64)
    cI = np.zeros((T, 12, 3))
    nn = np.zeros((T, 12, 3))
    A = np.zeros((T, 12))
    A0 = np.zeros((T, 12))
    Ln = np.zeros((T, 12))
    vol = np.zeros(N)
    mom1 = np.zeros((N, 3))
    mom2 = np.zeros((N, 3, 3))
    share = np.zeros((T, 4, 6))   # each tetrahedron's part of its nodes' lumped masses
    rows = np.arange(T)
    for k, (a, b, c) in enumerate(_facet_list()):
        d = 6 - a - b - c                     # the node missing from face (a, b, c)
        P0, P1, P2 = ep[(a, b)], fp[d], tp
        ga, gb = tets[:, a], tets[:, b]
        Ii, Jj = np.minimum(ga, gb), np.maximum(ga, gb)
        xi, xj = x[Ii], x[Jj]
        L = np.sqrt(((xj - xi) ** 2).sum(1))
        n = (xj - xi) / L[:, None]
        av = 0.5 * np.cross(P1 - P0, P2 - P0)
        sg = np.sign((av * n).sum(1))
        sg[sg == 0.0] = 1.0
        av = av * sg[:, None]
        I[:, k], J[:, k], nn[:, k], Ln[:, k] = Ii, Jj, n, L
        A[:, k] = (av * n).sum(1)
        A0[:, k] = np.sqrt((av * av).sum(1))
        cI[:, k] = (P0 + P1 + P2) / 3.0 - xi
        # cone (centre, triangle) integrals for the two cells; the triangle
        # P0, P1, P2 winds about +n when orient = +1
        orient = np.sign((np.cross(P1 - P0, P2 - P0) * av).sum(1))
        for side, node, loc in ((1.0, Ii, np.where(ga < gb, a, b)), (-1.0, Jj, np.where(ga < gb, b, a))):
            o = x[node]
            q1, q2, q3 = P0 - o, P1 - o, P2 - o
            V = side * orient * (np.cross(q1, q2) * q3).sum(1) / 6.0
            ssum = q1 + q2 + q3
            S = (q1[:, :, None] * q1[:, None, :] + q2[:, :, None] * q2[:, None, :]
                 + q3[:, :, None] * q3[:, None, :] + ssum[:, :, None] * ssum[:, None, :]) * (V / 20.0)[:, None, None]
            np.add.at(vol, node, V)
            np.add.at(mom1, node, V[:, None] * ssum / 4.0)
            np.add.at(mom2, node, S)
            dS = np.einsum("tii->ti", S)
            share[rows, loc, 0:3] += (rho * V)[:, None]
            share[rows, loc, 3:6] += rho * (dS.sum(1)[:, None] - dS)
    n_f = nn.reshape(F, 3)
    ax = np.argmin(np.abs(n_f), axis=1)
    e = np.zeros_like(n_f)
    e[np.arange(F), ax] = 1.0
    m = np.cross(n_f, e)
    m /= np.sqrt((m * m).sum(1))[:, None]
    tr = np.trace(mom2, axis1=1, axis2=2)
    Jfull = rho * (tr[:, None, None] * np.eye(3)[None] - mom2)
    return dict(facet_I=I.reshape(F), facet_J=J.reshape(F), facet_cI=cI.reshape(F, 3), facet_n=n_f,
                facet_m=m, facet_area=A.reshape(F), facet_area0=A0.reshape(F), facet_len=Ln.reshape(F),
                mass=rho * vol, inertia=np.ascontiguousarray(np.einsum("nii->ni", Jfull)), cell_inertia=Jfull,
                cell_vol=vol, cell_r=mom1 / np.maximum(vol, 1e-300)[:, None], tet_node_share=share)
