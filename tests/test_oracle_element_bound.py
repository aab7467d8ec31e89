"""Pins of the oracle's element bound of the stable step
(oracle/element_bound.py) and of the per-tetrahedron mass shares of the
oracle tessellation:

- the shares of each node sum to its cell mass and diagonal inertia;
- a single tetrahedron: the element eigenvalue is the largest eigenvalue of
  the assembled generalised problem K0 v = lambda M v (K0 from the oracle's
  global assembly, which its own pins tie to the matrix-free forces);
- several tetrahedra: the largest element eigenvalue bounds the assembled
  one from above (the element-by-element bound), and not loosely;
- every element matrix has exactly the six rigid-body zero modes;
- the input generator's element bound (an independent vectorised code)
  agrees.
"""
import numpy as np
import scipy.linalg as la

from oracle.element_bound import element_lambda_max, element_stiffness
from oracle.implicit import elastic_stiffness
from oracle.tessellation import tessellate
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached


def _elements(s):
    t = tessellate(s["x0"], s["diam"], s["tet_nodes"], S.RHO)
    mat = s["material"]
    K = element_stiffness(s["tet_nodes"], t["facet_I"], t["facet_J"], t["facet_cI"], t["facet_n"],
                          t["facet_area"], t["facet_len"], float(mat["E0"]), float(mat["alpha"]))
    return t, K


def _cube():
    return cached("eb_cube", lambda: S.tension_cube(edge=30.0, d0=4.0, da=8.0, seed=7))


def test_shares_sum_to_the_cell_masses():
    s = _cube()
    t, _ = _elements(s)
    sh = t["tet_node_share"]
    N = s["x0"].shape[0]
    acc = np.zeros((N, 6))
    np.add.at(acc, np.asarray(s["tet_nodes"]).ravel(), sh.reshape(-1, 6))
    assert np.abs(acc[:, 0] - t["mass"]).max() <= 1e-13 * t["mass"].max()
    assert np.abs(acc[:, 3:] - t["inertia"]).max() <= 1e-13 * t["inertia"].max()
    assert np.array_equal(acc[:, 0], acc[:, 1]) and np.array_equal(acc[:, 0], acc[:, 2])


def _assembled_lambda(s, t):
    K0 = elastic_stiffness(dict(s, facet_I=t["facet_I"], facet_J=t["facet_J"], facet_cI=t["facet_cI"],
                                facet_n=t["facet_n"], facet_area=t["facet_area"],
                                facet_len=t["facet_len"])).toarray()
    M = np.concatenate([np.repeat(t["mass"][:, None], 3, 1), t["inertia"]], 1).ravel()
    return la.eigh(K0, np.diag(M), eigvals_only=True)[-1]


def test_single_tetrahedron_is_the_assembled_problem():
    s = S.single_tet()
    t, K = _elements(s)
    lam_e = element_lambda_max(K, t["tet_node_share"])
    lam = _assembled_lambda(s, t)
    assert abs(lam_e[0] - lam) <= 1e-11 * lam


def test_element_bound_holds_and_is_tight():
    s = S.few_particle(12, seed=3)
    t, K = _elements(s)
    lam_e = element_lambda_max(K, t["tet_node_share"])
    lam = _assembled_lambda(s, t)
    assert lam_e.max() >= lam * (1 - 1e-12)
    assert lam_e.max() <= 4.0 * lam


def test_six_rigid_modes_per_element():
    s = _cube()
    t, K = _elements(s)
    m = t["tet_node_share"].reshape(-1, 24)
    w = 1.0 / np.sqrt(m)
    ev = np.linalg.eigvalsh(K * w[:, :, None] * w[:, None, :])
    assert np.all(np.abs(ev[:, :6]) <= 1e-10 * ev[:, -1:])
    assert np.all(ev[:, 6] > 1e-6 * ev[:, -1])


def test_the_generator_computes_the_same_bound():
    s = _cube()
    t, K = _elements(s)
    lam_o = element_lambda_max(K, t["tet_node_share"])
    mat = s["material"]
    tets = np.asarray(s["tet_nodes"], dtype=np.int64)
    _, tri = S.tessellate(s["x0"], s["diam"], tets)
    em = S.element_mass_share(s["x0"], tets, tri, S.RHO)
    lam_g = S.element_lambda_max(dict(s, _elem_mass=em), mat["E0"], mat["alpha"])
    assert np.abs(lam_o - lam_g).max() <= 1e-12 * lam_o.max()
