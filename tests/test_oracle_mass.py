"""Pins of the mass representations (eq. balance: the cell's inertia tensors;
the implementations' mass matrices) in the generator and the oracle.

- the full rigid-cell block gives the exact kinetic energy of a rigid motion
  of the whole specimen (the cells tile it), closed form for a cube; the
  lumped diagonal does not;
- central difference with the block: modal dispersion of the generalised
  eigenproblem K phi = w^2 M phi (scipy), stability limit, energy balance
  with prescribed DoFs and reactions;
- a block that is diagonal reproduces the lumped path;
- the sphere variant: equal split of tetrahedron masses, m d^2 / 10;
- the rescaled time step keeps the stability margin (dense eigenvalues).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached

MB = S.MATERIAL_MB
L_CUBE = 20.0


def _free_cube():
    """20 mm cube, every DoF free, no loads, elastic."""
    def make():
        s = dict(S.tension_cube(edge=L_CUBE, d0=4.0, da=8.0, seed=5, rate=2.0, ramp=2e-4))
        N = s["x0"].shape[0]
        s["dof_mode"] = np.zeros((N, 6), np.uint8)
        s["dof_prog"] = -np.ones((N, 6), np.int32)
        s["dof_scale"] = np.zeros((N, 6))
        s["material"] = dict(MB, law=0)
        return s
    return cached("mass_free_cube", make)


def _block(s):
    return cached(("mass_block", id(s)), lambda: S.mass_variant(s, "cell_block"))


def _dense_block(s):
    N = s["x0"].shape[0]
    iu = np.triu_indices(6)
    M = np.zeros((6 * N, 6 * N))
    for i in range(N):
        B = np.zeros((6, 6))
        B[iu] = s["mass_block"][i]
        B = B + B.T - np.diag(np.diag(B))
        M[6 * i:6 * i + 6, 6 * i:6 * i + 6] = B
    return M


def _stiffness(o):
    K = np.zeros((6 * o.N, 6 * o.N))
    for i in range(6 * o.N):
        q = np.zeros((o.N, 6))
        q.flat[i] = 1.0
        K[:, i] = o.elastic_internal_force(q).ravel()
    return 0.5 * (K + K.T)


def _rigid_velocity(x, V, W):
    v = np.zeros((x.shape[0], 6))
    v[:, :3] = V + np.cross(W, x)
    v[:, 3:] = W
    return v


def _cube_kinetic_energy(rho, L, V, W):
    """1/2 int rho |V + W x x|^2 over [0, L]^3."""
    M = rho * L ** 3
    xc = np.full(3, L / 2)
    JO = rho * (np.eye(3) * (2 * L ** 5 / 3) - (np.ones((3, 3)) - np.eye(3)) * (L ** 5 / 4))
    return 0.5 * M * V @ V + M * V @ np.cross(W, xc) + 0.5 * W @ JO @ W


def test_cell_block_gives_the_exact_rigid_body_kinetic_energy():
    """The cells tile the cube and move rigidly with their particles, so the
    per-cell blocks sum to the continuum kinetic energy of any rigid motion;
    a rigid motion has no strain, so it also persists unchanged."""
    s = dict(_block(_free_cube()))
    V, W = np.array([0.3, -0.2, 0.5]), np.array([2.0, -1.0, 3.0])
    s["v0"] = _rigid_velocity(s["x0"], V, W)
    rho = s["mass"].sum() / L_CUBE ** 3
    exact = _cube_kinetic_energy(rho, L_CUBE, V, W)
    o = O.Oracle(s).step(1)
    assert abs(o.energies()["W_kin0"] - exact) < 1e-12 * exact
    o.step(20)
    assert np.abs(o.v - s["v0"]).max() < 1e-9 * np.abs(s["v0"]).max()
    assert abs(o.energies()["W_kin"] - exact) < 1e-9 * exact
    lumped = dict(_free_cube(), v0=s["v0"])
    ol = O.Oracle(lumped).step(1)
    assert abs(ol.energies()["W_kin0"] - exact) > 1e-2 * exact


@pytest.mark.parametrize("which", [6, 20, -1])
def test_central_difference_modal_dispersion_with_the_cell_block(which):
    """From rest in a mode of K phi = w^2 M phi (M the assembled blocks):
    q^n = cos(n w~ dt) phi with sin(w~ dt / 2) = w dt / 2."""
    base = dict(S.few_particle(12, seed=3))
    base["material"] = dict(MB, law=0)
    s = S.mass_variant(base, "cell_block")
    o = O.Oracle(s)
    K = _stiffness(o)
    w2, phi = sl.eigh(K, _dense_block(s))
    w = math.sqrt(max(w2[which], 0.0))
    s = dict(s, dt=0.9 * 2.0 / math.sqrt(w2[-1]))
    o = O.Oracle(s)
    amp = 1e-3 / np.abs(phi[:, which]).max()
    o.q[...] = (amp * phi[:, which]).reshape(o.N, 6)
    wt = 2.0 * math.asin(w * s["dt"] / 2.0) / s["dt"]
    prev = 0
    for n_steps in (1, 7, 50, 333):
        o.step(n_steps - prev)
        prev = n_steps
        expect = amp * phi[:, which] * math.cos(o.step_index * wt * s["dt"])
        assert np.abs(o.q.ravel() - expect).max() < 1e-8 * amp * np.abs(phi[:, which]).max()


def test_stability_limit_with_the_cell_block():
    base = dict(S.few_particle(12, seed=3))
    base["material"] = dict(MB, law=0)
    s = S.mass_variant(base, "cell_block")
    K = _stiffness(O.Oracle(s))
    wmax = math.sqrt(sl.eigh(K, _dense_block(s), eigvals_only=True)[-1])
    rng = np.random.default_rng(0)
    q0 = rng.normal(size=(s["x0"].shape[0], 6)) * 1e-6
    for f, grows in ((0.98, False), (1.02, True)):
        o = O.Oracle(dict(s, dt=f * 2.0 / wmax))
        o.q[...] = q0
        try:
            o.step(3000)
            grew = np.abs(o.q).max() > 1e3 * np.abs(q0).max()
        except FloatingPointError:
            grew = True
        assert grew == grows, f


def test_energy_balance_with_the_cell_block_and_reactions():
    """Prescribed velocities on coupled DoFs: with the reactions
    R_P = (M a)_P - f_P counted in W_ext, the balance closes (a wrong
    partition of the solve or of the reactions breaks it)."""
    s = dict(S.tension_cube(edge=20.0, d0=4.0, da=8.0, seed=5, rate=2.0, ramp=2e-4))
    s["material"] = dict(MB, law=0)
    s = S.mass_variant(s, "cell_block")
    errs = []
    for k in (1, 2):
        o = O.Oracle(dict(s, dt=s["dt"] / k))
        o.step(1500 * k)
        en = o.energies()
        assert en["W_ext"] > 0
        errs.append(en["err"])
    assert max(errs) < 1e-8


def test_diagonal_block_reproduces_the_lumped_path():
    s = dict(S.tension_cube(edge=20.0, d0=4.0, da=8.0, seed=5, rate=2.0, ramp=2e-4))
    N = s["x0"].shape[0]
    M = np.zeros((N, 6, 6))
    for i in range(3):
        M[:, i, i] = s["mass"]
        M[:, 3 + i, 3 + i] = s["inertia"][:, i]
    iu = np.triu_indices(6)
    d = dict(s, mass_block=np.ascontiguousarray(M[:, iu[0], iu[1]]))
    a = O.Oracle(s).step(600)
    b = O.Oracle(d).step(600)
    for f in ("q", "v", "t", "fext"):
        x, y = getattr(a, f), getattr(b, f)
        assert np.abs(x - y).max() <= 1e-13 * np.abs(x).max(), f
    assert abs(a.energies()["W_kin"] - b.energies()["W_kin"]) <= 1e-13 * a.energies()["W_kin"]


def test_sphere_variant():
    s = _free_cube()
    v = S.mass_variant(s, "sphere")
    rho = s["mass"].sum() / L_CUBE ** 3
    assert abs(v["mass"].sum() - rho * L_CUBE ** 3) < 1e-12 * rho * L_CUBE ** 3
    assert np.allclose(v["inertia"], (v["mass"] * s["diam"] ** 2 / 10.0)[:, None], rtol=1e-15)


@pytest.mark.parametrize("kind", ["cell_block", "sphere"])
def test_rescaled_step_keeps_the_stability_margin(kind):
    """dt of a variant: dt_variant * w_max(variant) = min(1, ...) of
    dt * w_max(lumped), from dense generalised eigenvalues."""
    base = dict(_free_cube())
    v = S.mass_variant(base, kind)
    K = _stiffness(O.Oracle(base))
    D = np.diag(np.concatenate([np.repeat(base["mass"][:, None], 3, 1), base["inertia"]], 1).ravel())
    Mv = _dense_block(v) if kind == "cell_block" else \
        np.diag(np.concatenate([np.repeat(v["mass"][:, None], 3, 1), v["inertia"]], 1).ravel())
    wl = math.sqrt(sl.eigh(K, D, eigvals_only=True)[-1])
    wv = math.sqrt(sl.eigh(K, Mv, eigvals_only=True)[-1])
    margin = base["dt"] * wl
    assert v["dt"] * wv <= margin * (1 + 1e-6)
    assert v["dt"] == base["dt"] or abs(v["dt"] * wv - margin) < 1e-6 * margin
