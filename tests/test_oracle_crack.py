"""Pins of the oracle's crack-opening field, field comparison and random
perturbation against what the paper and the mathematics fix.

- crack opening (numerical-examples section, comparison of crack patterns):
  closed forms along strain paths whose tractions have closed forms
  (pure-tension softening, elastic unloading, frictional sliding, pore
  collapse), and zero for elastic states;
- Pearson's correlation and NRMSE (same section): library routines
  (numpy.corrcoef, scipy.stats.pearsonr) and closed forms;
- random perturbation (section on the numerical study of time step,
  convergence criteria and stability): masking of prescribed DoFs, rigid
  jumps, the strain-energy change of an elastic jump, consistency of the
  history with the perturbed positions, and the energy balance.
"""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached

MB = S.MATERIAL_MB


def _w(e_last, t_last, L, p=MB):
    return O.crack_opening(np.atleast_2d(e_last), np.atleast_2d(t_last), np.array([L]),
                           p["E0"], p["alpha"])[0]


# ------------------------------------------------------------ crack opening
def test_crack_opening_of_pure_tension_softening_closed_form():
    """Pure tension past the peak: t = sigma_t exp(-H_t (e - e0) / sigma_t),
    so w_N = l (e - t / E0) in closed form, and w = 0 before the peak."""
    p = dict(MB)
    L = 6.0
    es = np.linspace(0, 2e-3, 2001)[1:]
    path = np.zeros((es.size, 3)); path[:, 0] = es
    T, _ = O.drive_facet(p, L, path)
    W = O.crack_opening(path, T, np.full(es.size, L), p["E0"], p["alpha"])
    Ht = 2 * p["E0"] / (p["l_t"] / L - 1)
    e0 = p["sigma_t"] / p["E0"]
    t_cf = np.where(es <= e0, p["E0"] * es, p["sigma_t"] * np.exp(-Ht * (es - e0) / p["sigma_t"]))
    w_cf = np.where(es <= e0, 0.0, L * (es - t_cf / p["E0"]))
    assert np.abs(W[:, 0] - w_cf).max() < 1e-12 * L * es.max()
    assert np.abs(W[:, 1:3]).max() == 0.0
    assert np.array_equal(W[:, 3], np.abs(W[:, 0]))
    assert W[-1, 0] > 0.99 * L * es[-1]  # a fully opened crack carries no traction


def test_crack_opening_is_frozen_during_elastic_unloading():
    """Unloading from the softening branch is elastic with slope E0 (k_t = 0),
    so the inelastic strain, hence w_N, keeps its value at the start of the
    unloading until the traction reaches zero; after that w_N = l e."""
    p = dict(MB)
    L = 6.0
    up = np.linspace(0, 3e-4, 301)[1:]
    down = np.linspace(3e-4, 0.5e-4, 301)[1:]
    es = np.concatenate([up, down])
    path = np.zeros((es.size, 3)); path[:, 0] = es
    T, _ = O.drive_facet(p, L, path)
    W = O.crack_opening(path, T, np.full(es.size, L), p["E0"], p["alpha"])
    wpk = W[up.size - 1, 0]
    tpk = T[up.size - 1, 0]
    still = down >= 3e-4 - tpk / p["E0"]
    assert np.abs(W[up.size:, 0][still] - wpk).max() < 1e-9 * wpk
    assert np.abs(W[up.size:, 0][~still] - L * down[~still]).max() < 1e-9 * wpk


@pytest.mark.parametrize("pN", [10.0, 100.0])
def test_crack_opening_of_frictional_slip_closed_form(pN):
    """Compression with an elastic normal strain and shear driven past the
    friction plateau sigma_bs(-p): the normal part contributes nothing, and
    the shear opening (slip) is l (e_T - sigma_bs / (alpha E0)) along the
    driven direction."""
    p = dict(MB, mu_inf=0.1)
    E0, al = p["E0"], p["alpha"]
    L = 6.0
    eN = -pN / E0
    es = np.linspace(0, 1e-2, 4001)[1:]
    path = np.zeros((es.size, 3)); path[:, 0] = eN; path[:, 1] = 0.6 * es; path[:, 2] = 0.8 * es
    T, _ = O.drive_facet(p, L, path, eV_path=np.full(es.size, eN))
    sbs = p["r_st"] * p["sigma_t"] + (p["mu0"] - p["mu_inf"]) * p["sigma_N0"] * (1 - math.exp(-pN / p["sigma_N0"])) \
        + p["mu_inf"] * pN
    w = _w(path[-1], T[-1], L, p)
    slip = L * (es[-1] - sbs / (al * E0))
    assert w[0] == 0.0
    assert abs(w[1] - 0.6 * slip) < 1e-9 * slip
    assert abs(w[2] - 0.8 * slip) < 1e-9 * slip
    assert abs(w[3] - slip) < 1e-9 * slip


def test_closing_inelastic_normal_strain_is_not_a_crack():
    """Hydrostatic compression beyond pore collapse (closed form of the
    compressive boundary): the inelastic normal strain is negative, and only
    a positive one opens a crack, so w = 0 while l (e_N - t_N / E0) < 0."""
    p = dict(MB)
    E0 = p["E0"]
    ec1 = p["kc0"] * p["sigma_c0"] / E0
    es = np.linspace(0, 1.3 * ec1, 4001)[1:]
    path = np.zeros((es.size, 3)); path[:, 0] = -es
    T, _ = O.drive_facet(p, 6.0, path, eV_path=-es)
    W = O.crack_opening(path, T, np.full(es.size, 6.0), E0, p["alpha"])
    raw = 6.0 * (path[:, 0] - T[:, 0] / E0)
    collapsed = es > 1.01 * p["sigma_c0"] / E0
    assert raw[collapsed].max() < 0 and raw.min() < -1e-3 * 6.0 * ec1
    assert np.all(W[collapsed] == 0.0)
    # elastic part: t = E0 e up to the rounding of the incremental update
    assert np.abs(W).max() < 1e-13 * 6.0 * ec1


def _small_cube():
    return cached("cube20", lambda: S.elastic_vibration_cube(edge=20.0, d0=4.0, da=8.0, seed=5))


def test_elastic_trajectory_has_no_crack_opening():
    """With t = E e there is no inelastic strain: w vanishes up to rounding."""
    s = _small_cube()
    o = O.Oracle(s).step(200)
    W = o.crack_opening()
    scale = np.abs(o.e).max() * s["facet_len"].max()
    assert scale > 0
    assert np.abs(W).max() < 1e-13 * scale


# --------------------------------------------------------- field comparison
def test_pearson_and_nrmse_against_library_routines():
    rng = np.random.default_rng(3)
    x = np.abs(rng.standard_cauchy(5001)) * 1e-2
    r = x + rng.normal(scale=1e-3, size=x.size)
    st = O.field_stats(x, r)
    assert abs(st["pearson"] - np.corrcoef(x, r)[0, 1]) < 1e-13
    assert abs(st["pearson"] - scipy.stats.pearsonr(x, r)[0]) < 1e-13
    rmse = math.sqrt(float(np.mean((x - r) ** 2)))
    assert abs(st["nrmse"] - 100.0 * rmse / r.max()) < 1e-12 * st["nrmse"]


def test_pearson_and_nrmse_closed_forms():
    rng = np.random.default_rng(4)
    r = rng.uniform(0.0, 2.0, 777)
    assert abs(O.field_stats(2.5 * r + 3.0, r)["pearson"] - 1.0) < 1e-14
    assert abs(O.field_stats(-r, r)["pearson"] + 1.0) < 1e-14
    same = O.field_stats(r, r)
    assert same["nrmse"] == 0.0 and abs(same["pearson"] - 1.0) < 1e-14
    c = 0.125
    st = O.field_stats(r + c, r)          # a uniform offset: NRMSE = 100 c / max
    assert abs(st["nrmse"] - 100.0 * c / r.max()) < 1e-13 * st["nrmse"]


def test_cap_limits_both_fields_first():
    """The unconfined-compression tables compare openings limited to 4 mm."""
    rng = np.random.default_rng(5)
    x = rng.exponential(1.0, 4000)
    r = rng.exponential(1.0, 4000)
    a = O.field_stats(x, r, cap=4.0)
    xc, rc = np.minimum(x, 4.0), np.minimum(r, 4.0)
    assert x.max() > 4.0 and r.max() > 4.0
    assert abs(a["pearson"] - scipy.stats.pearsonr(xc, rc)[0]) < 1e-13
    assert a["ref_max"] == 4.0
    assert abs(a["nrmse"] - 100.0 * math.sqrt(np.mean((xc - rc) ** 2)) / 4.0) < 1e-12 * a["nrmse"]


def test_degenerate_fields():
    one = O.field_stats([1.0], [2.0])
    assert math.isnan(one["pearson"]) and one["nrmse"] == 50.0
    z = O.field_stats([0.0, 1.0], [0.0, 0.0])
    assert math.isnan(z["pearson"]) and math.isinf(z["nrmse"])
    with pytest.raises(ValueError):
        O.field_stats([], [])


# ------------------------------------------------------ random perturbation
def _elastic_tension(edge=20.0, seed=5, rate=2.0, law=0):
    s = dict(S.tension_cube(edge=edge, d0=4.0, da=8.0, seed=seed, rate=rate, ramp=2e-4))
    s["material"] = dict(MB, law=law)
    return s


def _tension_state(law, steps=400):
    s = cached(("crack_tension", law), lambda: _elastic_tension(law=law, rate=20.0))
    o = O.Oracle(s).step(steps)
    return s, o


def _strain_energy(s, e):
    E = MB["E0"] * np.array([1.0, MB["alpha"], MB["alpha"]])
    return 0.5 * np.sum(s["facet_area"] * s["facet_len"] * np.einsum("ij,j,ij->i", e, E, e))


def test_zero_perturbation_changes_nothing():
    """A zero jump re-evaluates the law with a zero increment: positions,
    velocities and strains stay bitwise, tractions up to rounding, no work."""
    s, o = _tension_state(1, 100)
    before = [a.copy() for a in (o.q, o.v, o.e, o.emax, o.t)]
    W0 = o.energies()
    assert o.perturb(np.zeros((o.N, 6))) == 0.0
    for a, b in zip(before[:4], (o.q, o.v, o.e, o.emax)):
        assert np.array_equal(a, b)
    assert np.abs(o.t - before[4]).max() <= 1e-13 * np.abs(before[4]).max()
    assert o.energies()["W_int"] == W0["W_int"] and o.energies()["W_pert"] == 0.0


def test_perturbation_moves_free_dofs_only():
    s, o = _tension_state(1, 100)
    q0 = o.q.copy()
    d = S.perturbation(o.N, 1e-4, seed=1, index=0)
    o.perturb(d)
    free = s["dof_mode"] == 0
    assert np.array_equal(o.q[~free], q0[~free])
    assert np.array_equal(o.q[free], q0[free] + d[free])
    assert np.all(np.abs(d) <= 0.5e-4) and np.abs(d).max() > 0.45e-4


def test_history_matches_the_perturbed_positions():
    """After the jump the stored strain is the strain of the last evaluated
    configuration plus the jump, i.e. of q^n - dt v^{n-1/2} after the jump."""
    for law in (0, 1):
        s, o = _tension_state(law, 300)
        o.perturb(S.perturbation(o.N, 2e-4, seed=2, index=0))
        e_pos = o.strains(o.last_configuration())
        assert np.abs(o.e - e_pos).max() < 1e-12 * np.abs(o.e).max()


def test_rigid_jump_leaves_the_state_and_does_no_work():
    """A small rigid motion of every particle (all DoFs free) adds no strain:
    tractions and history stay, and the jump does no work."""
    s = dict(S.few_particle(12, seed=3))
    s["v0"] = np.zeros((s["x0"].shape[0], 6))
    s["v0"][:, :3] = 50.0 * (s["x0"] - s["x0"].mean(0))    # expanding: facets in tension
    o = O.Oracle(s).step(40)
    t0 = o.t.copy()
    rng = np.random.default_rng(7)
    a, w = rng.normal(size=3) * 1e-3, rng.normal(size=3) * 1e-4
    d = np.zeros((o.N, 6))
    d[:, :3] = a + np.cross(w, s["x0"])
    d[:, 3:] = w
    W = o.perturb(d)
    assert np.abs(t0).max() > 0
    assert np.abs(o.t - t0).max() < 1e-9 * np.abs(t0).max()
    U = float(np.sum(s["facet_area"] * s["facet_len"] * np.abs(o.e * o.t).sum(1)))
    assert abs(W) < 1e-9 * U


def test_elastic_jump_work_is_the_strain_energy_change():
    """With t = E e the trapezoid work of the jump equals the change of the
    strain energy 1/2 sum A l e.E e, and is counted in W_int and W_pert."""
    s, o = _tension_state(0, 300)
    U0 = _strain_energy(s, o.e)
    Wi0 = o.energies()["W_int"]
    W = o.perturb(S.perturbation(o.N, 2e-4, seed=3, index=0))
    U1 = _strain_energy(s, o.e)
    assert abs(W - (U1 - U0)) < 1e-10 * U1
    en = o.energies()
    assert en["W_pert"] == W and abs(en["W_int"] - (Wi0 + W)) < 1e-14 * abs(en["W_int"])
    # and the reverse jump restores the strain and returns the work
    W2 = o.perturb(-S.perturbation(o.N, 2e-4, seed=3, index=0))
    assert abs(W + W2) < 1e-10 * abs(W)
    assert abs(_strain_energy(s, o.e) - U0) < 1e-10 * U0


def test_energy_balance_counts_the_perturbation_work():
    """Energy-balance measure with periodic perturbations: W_pert closes the
    balance up to the measure's own dispersion error for the high-frequency
    content a random jump excites (a few % of W_pert at 0.8 of the stable
    step, against 1e-13 without perturbations); leaving W_pert out leaves
    all of it open."""
    s, o = _tension_state(0, 0)
    for k in range(6):
        o.step(250)
        o.perturb(S.perturbation(o.N, 1e-4, seed=4, index=k))
    o.step(250)
    en = o.energies()
    src = abs(en["W_ext"] + en["W_pert"])
    assert en["W_pert"] > 0.0
    assert en["err"] * src < 0.05 * en["W_pert"]
    open_ = O.energy_error(en["W_ext"], en["W_int"], en["W_kin"], en["W_kin0"]) * abs(en["W_ext"])
    assert abs(open_ - en["W_pert"]) < 0.05 * en["W_pert"]


def test_perturbation_before_the_first_step_is_an_initial_displacement():
    s, o = _tension_state(1, 0)
    d = S.perturbation(o.N, 1e-4, seed=5, index=0)
    assert o.perturb(d) == 0.0
    free = s["dof_mode"] == 0
    assert np.array_equal(o.q[free], d[free]) and np.all(o.t == 0.0)


def test_volumetric_strain_field_is_at_the_last_evaluated_configuration():
    """u = eps x: every tetrahedron has e_V = tr(eps)/3 (linearised volume
    change over 3 V); the field is taken at q^n - dt v^{n-1/2}."""
    s = _small_cube()
    o = O.Oracle(s).step(3)
    eps = np.array([[1e-4, 2e-5, 0.0], [2e-5, -3e-5, 1e-5], [0.0, 1e-5, 5e-5]])
    q = np.zeros((o.N, 6))
    q[:, :3] = s["x0"] @ eps.T
    v = np.random.default_rng(8).normal(size=(o.N, 6))
    o.set_state(q + float(s["dt"]) * v, v, o.t, o.e, o.emax, o.fext, step=3)
    ev = o.volumetric_strain_field()
    assert np.abs(ev - np.trace(eps) / 3.0).max() < 1e-9 * abs(np.trace(eps))
