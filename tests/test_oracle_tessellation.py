"""Pins of the oracle's tessellation (oracle/tessellation.py): exact
geometric identities of the construction and of the cells it builds.

- sum_k A_k l_k = 3 V_tet for the 12 facets of every tetrahedron (the
  facets split the tetrahedron into four node regions with planar facets;
  divergence theorem);
- the cells tile the specimen: their volumes sum to its volume, and their
  mass blocks give the exact kinetic energy of a rigid motion of a cube;
- frames are orthonormal with n along I -> J, I < J, A <= A0, and facet
  centroids lie inside their tetrahedron;
- the input generator builds the same geometry (cross-check of two
  independent codes).
"""
import numpy as np

from oracle.tessellation import tessellate
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached

L = 30.0


def _case():
    def make():
        s = S.tension_cube(edge=L, d0=4.0, da=8.0, seed=7)
        return s, tessellate(s["x0"], s["diam"], s["tet_nodes"], S.RHO)
    return cached("oracle_tess", make)


def _tet_volumes(x, tets):
    p = x[tets]
    return np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6.0


def test_area_times_length_is_three_tet_volumes():
    s, o = _case()
    V = _tet_volumes(s["x0"], s["tet_nodes"])
    Al = (o["facet_area"] * o["facet_len"]).reshape(-1, 12).sum(1)
    assert np.all(V > 0)
    assert np.abs(Al - 3 * V).max() < 1e-11 * V.max()


def test_cells_tile_the_cube_and_give_the_rigid_kinetic_energy():
    s, o = _case()
    assert abs(o["cell_vol"].sum() - L ** 3) < 1e-9 * L ** 3
    rho = S.RHO
    V, W = np.array([0.3, -0.2, 0.5]), np.array([2.0, -1.0, 3.0])
    x = s["x0"]
    u = V + np.cross(W, x)
    c = o["mass"][:, None] * o["cell_r"]
    KE = 0.5 * (o["mass"] * (u * u).sum(1)).sum() + (u * np.cross(W, c)).sum() \
        + 0.5 * np.einsum("i,nij,j->", W, o["cell_inertia"], W)
    M = rho * L ** 3
    JO = rho * (np.eye(3) * (2 * L ** 5 / 3) - (np.ones((3, 3)) - np.eye(3)) * (L ** 5 / 4))
    exact = 0.5 * M * V @ V + M * V @ np.cross(W, np.full(3, L / 2)) + 0.5 * W @ JO @ W
    assert abs(KE - exact) < 1e-11 * exact


def test_frames_orientation_and_centroids():
    s, o = _case()
    x = s["x0"]
    n, m = o["facet_n"], o["facet_m"]
    d = x[o["facet_J"]] - x[o["facet_I"]]
    assert np.all(o["facet_I"] < o["facet_J"])
    assert np.allclose(d / o["facet_len"][:, None], n, atol=1e-14)
    assert np.allclose((n * m).sum(1), 0.0, atol=1e-14) and np.allclose(np.linalg.norm(m, axis=1), 1.0)
    assert np.all(o["facet_area"] > 0) and np.all(o["facet_area"] <= o["facet_area0"] * (1 + 1e-12))
    T = s["tet_nodes"].shape[0]
    xk = (x[o["facet_I"]] + o["facet_cI"]).reshape(T, 12, 3)
    p = x[s["tet_nodes"]]
    Jm = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], -1)
    lam = np.linalg.solve(Jm[:, None], (xk - p[:, None, 0])[..., None])[..., 0]
    assert (1 - lam.sum(-1)).min() > -1e-9 and lam.min() > -1e-9


def test_the_input_generator_builds_the_same_geometry():
    s, o = _case()
    for k in ("facet_I", "facet_J", "facet_cI", "facet_n", "facet_m", "facet_area", "facet_area0", "facet_len",
              "mass", "inertia", "cell_inertia", "cell_vol", "cell_r"):
        a, b = np.asarray(o[k], float), np.asarray(s[k], float)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max(), k
