"""Invariants of the seeded input generator (geometry the solver consumes)."""
import numpy as np

from paper_2603_13190_amd import specimen as S
from tests.conftest import cached


def cube():
    return cached("gen_cube30", lambda: S.tension_cube(edge=30.0, d0=4.0, da=8.0, seed=7))


def _tet_volumes(s):
    p = s["x0"][s["tet_nodes"]]
    return np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0]) / 6


def test_sum_area_times_length_is_three_volumes():
    """The 12 facets split each tetrahedron into four node regions with
    planar facets, so sum_k A_k l_k = 3 V_tet (divergence theorem)."""
    s = cube()
    V = _tet_volumes(s)
    T = V.size
    Al = (s["facet_area"] * s["facet_len"]).reshape(T, 12).sum(1)
    assert np.all(V > 0)
    assert np.abs(Al - 3 * V).max() < 1e-11 * V.max()


def test_cells_fill_the_specimen_and_mass_is_rho_V():
    s = cube()
    assert abs(s["cell_vol"].sum() - 30.0 ** 3) < 1e-9 * 30.0 ** 3
    assert abs(s["mass"].sum() - S.RHO * 30.0 ** 3) < 1e-9 * S.RHO * 30.0 ** 3
    assert np.all(s["mass"] > 0) and np.all(s["inertia"] > 0)


def test_facet_frames():
    s = cube()
    n, m = s["facet_n"], s["facet_m"]
    d = s["x0"][s["facet_J"]] - s["x0"][s["facet_I"]]
    assert np.allclose(np.linalg.norm(d, axis=1), s["facet_len"], rtol=1e-14)
    assert np.allclose(d / s["facet_len"][:, None], n, atol=1e-14)
    assert np.allclose(np.einsum("ij,ij->i", n, m), 0, atol=1e-14)
    assert np.allclose(np.linalg.norm(m, axis=1), 1, atol=1e-14)
    assert np.all(s["facet_I"] < s["facet_J"])
    assert np.all(s["facet_area"] > 0)
    assert np.all(s["facet_area"] <= s["facet_area0"] * (1 + 1e-12))
    assert np.array_equal(s["facet_tet"], np.arange(s["facet_tet"].size) // 12)


def test_facet_centroids_inside_their_tetrahedron():
    s = cube()
    T = s["tet_nodes"].shape[0]
    xk = (s["x0"][s["facet_I"]] + s["facet_cI"]).reshape(T, 12, 3)
    p = s["x0"][s["tet_nodes"]]
    Jm = np.stack([p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]], -1)
    lam = np.linalg.solve(Jm[:, None], (xk - p[:, None, 0])[..., None])[..., 0]
    bary = np.concatenate([1 - lam.sum(-1, keepdims=True), lam], -1)
    assert bary.min() > -1e-9


def test_fuller_diameters_volume_distribution():
    """Volume fraction passing d follows the truncated Fuller curve."""
    rng = np.random.default_rng(0)
    d0, da, nF = 4.0, 10.0, 0.4
    d = S.fuller_diameters(rng, 2e7, d0, da, nF)
    assert d.min() >= d0 and d.max() <= da
    w = d ** 3
    for x in (5.0, 6.5, 8.0, 9.5):
        emp = w[d <= x].sum() / w.sum()
        th = ((x / da) ** nF - (d0 / da) ** nF) / (1 - (d0 / da) ** nF)
        assert abs(emp - th) < 0.01


def test_placement_respects_gap_and_surface():
    rng = np.random.default_rng(1)
    shape = S.Shape("box", (40.0, 40.0, 40.0))
    x, d = S.place_particles(shape, 4.0, 8.0, rng, gap=0.1)
    from scipy.spatial.distance import pdist, squareform
    D = squareform(pdist(x))
    np.fill_diagonal(D, np.inf)
    lim = (d[:, None] + d[None, :]) / 2 * 1.1
    assert np.all(D >= lim * (1 - 1e-12))
    r = d / 2
    assert np.all(x - r[:, None] > 0) and np.all(x + r[:, None] < 40.0)


def test_batched_concatenation_offsets():
    a = S.tension_cube(edge=20.0, seed=1)
    b = S.tension_cube(edge=25.0, seed=2)
    c = S.concat_specimens([a, b])
    assert c["particle_off"].tolist() == [0, a["meta"]["N"], a["meta"]["N"] + b["meta"]["N"]]
    assert c["facet_I"][a["meta"]["F"]:].min() >= a["meta"]["N"]
    assert np.array_equal(c["facet_tet"], np.arange(c["facet_tet"].size) // 12)
    assert c["prog_off"].size - 1 == (a["prog_off"].size - 1) + (b["prog_off"].size - 1)


def test_cylinder_has_no_boundary_slivers():
    """Points on a curved surface: boundary slivers spanning the hull are
    peeled, the mesh fills the cylinder (up to the inscribed-polygon deficit
    of ~22 surface nodes per ring, about 1.4 %) and no edge is long."""
    g = S.build_geometry(S.Shape("cylinder", (40.0, 60.0)), 4.0, 8.0, seed=2)
    vol = np.pi * 20.0 ** 2 * 60.0
    assert abs(g["cell_vol"].sum() - vol) < 0.03 * vol
    assert g["facet_len"].max() < 4 * 8.0
    assert np.all(g["mass"] > 0)
