"""Implicit HHT-alpha integration on the GPU (modified Newton on the initial
elastic stiffness, matrix-free CG solves) against the oracle's HHT-alpha
driver (sparse LU solves), FP64.

Both sides converge every step to a tight Newton tolerance, so the accepted
states agree to the FP64 trajectory bar (1e-9) whatever the inner solver.
"""
import numpy as np
import pytest

import oracle as O
from oracle.implicit import HHT
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached
from tests.gpu_util import rel, tension_full

pytestmark = pytest.mark.gpu

MB = S.MATERIAL_MB
OPTS = dict(tol=1e-8, max_iter=60, cg_tol=1e-13, cg_max_iter=20000)


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    return System(sysd, **kw)


def compare(g, o, tol, what, fields=("q", "v", "t", "emax", "fext")):
    st = g.read_state()
    for f in fields:
        e = rel(st[f], getattr(o, f))
        assert e <= tol, (what, f, e)


def el_tension():
    return cached("im_el_tension", lambda: dict(S.tension_cube(edge=20.0, d0=4.0, da=8.0, seed=5, rate=2.0,
                                                               ramp=2e-4), material=dict(MB, law=0)))


def el_vibration():
    return cached("im_el_vib", lambda: S.elastic_vibration_cube(edge=20.0, d0=4.0, da=8.0, seed=5))


def inel_tension():
    return cached("im_tension", lambda: S.tension_cube(edge=30.0, d0=4.0, da=8.0, seed=2, rate=2.0, ramp=2e-4))


@pytest.mark.parametrize("alpha", [0.0, -0.1])
def test_elastic_tension_with_reactions(alpha):
    s = el_tension()
    dt = 10 * s["dt"]
    o = O.Oracle(s)
    HHT(o, s, dt=dt, alpha=alpha, tol=OPTS["tol"], max_iter=OPTS["max_iter"]).step(100)
    g = gpu(s)
    st = g.implicit_step(100, dt, alpha=alpha, **OPTS)
    assert st["not_converged"] == 0
    compare(g, o, 1e-9, f"elastic tension alpha={alpha}")
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_ext", "W_kin"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * abs(eo[k]), (k, eg[k], eo[k])
    if alpha == 0.0:
        assert eg["err"] < 1e-12                    # the trapezoidal rule's energy identity
    assert abs(eg["time"] - 100 * dt) < 1e-15


def test_free_vibration_large_steps():
    s = el_vibration()
    dt = 20 * s["dt"]
    o = O.Oracle(s)
    HHT(o, s, dt=dt, alpha=0.0, tol=OPTS["tol"], max_iter=OPTS["max_iter"]).step(60)
    g = gpu(s)
    g.implicit_step(60, dt, alpha=0.0, **OPTS)
    compare(g, o, 1e-9, "free vibration", fields=("q", "v", "t"))
    assert g.energy()["err"] < 1e-12


def test_inelastic_tension_before_the_peak():
    s = inel_tension()
    dt = 10 * s["dt"]
    o = O.Oracle(s)
    h = HHT(o, s, dt=dt, alpha=-0.1, tol=OPTS["tol"], max_iter=OPTS["max_iter"])
    h.step(19)
    g = gpu(s)
    st = g.implicit_step(19, dt, alpha=-0.1, **OPTS)
    ko = sum(k for k, _ in h.iters)
    print("newton iterations: oracle", ko, "gpu", st["newton_iters"], "cg", st["cg_iters"])
    assert abs(st["newton_iters"] - ko) <= 19
    assert o.emax.max() > 0.5 * s["material"]["sigma_t"] / s["material"]["E0"]
    compare(g, o, 1e-9, "inelastic implicit")
    wg, wo = g.crack_opening().cpu().numpy().T, o.crack_opening()
    assert np.abs(wg - wo).max() <= 1e-9 * max(np.abs(wo).max(), np.abs(o.e).max() * s["facet_len"].max())
    ev = g.volumetric_strain().cpu().numpy()
    evo = o.volstrains(o.q)
    assert np.abs(ev - evo).max() <= 1e-9 * np.abs(evo).max()
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_ext", "W_kin"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * abs(eo[k]), (k, eg[k], eo[k])


@pytest.mark.parametrize("rho_inf", [0.8, 0.3, 0.0])
def test_generalised_alpha(rho_inf):
    """Generalised-alpha (a_m = (2 rho - 1)/(rho + 1), a_f = rho/(rho + 1)):
    elastic tension and inelastic tension up to the peak.  At rho_inf = 0
    the elastic case's last steps stop at the iteration cap on both sides
    (their residual stays just above the relative tolerance), which the
    comparison covers as well."""
    from oracle.implicit import gen_alpha_params
    am, af = gen_alpha_params(rho_inf)
    for s, n in ((el_tension(), 60), (inel_tension(), 19)):
        dt = 10 * s["dt"]
        o = O.Oracle(s)
        HHT(o, s, dt=dt, tol=OPTS["tol"], max_iter=OPTS["max_iter"], alpha_m=am, alpha_f=af).step(n)
        g = gpu(s)
        g.implicit_step(n, dt, rho_inf=rho_inf, **OPTS)
        compare(g, o, 1e-9, f"generalised-alpha rho={rho_inf}")


def test_implicit_is_deterministic_and_resumes_in_chunks():
    s = inel_tension()
    dt = 10 * s["dt"]
    a = gpu(s)
    a.implicit_step(12, dt, alpha=-0.1, **OPTS)
    b = gpu(s)
    b.implicit_step(5, dt, alpha=-0.1, **OPTS)
    b.implicit_step(7, dt, alpha=-0.1, **OPTS)
    sa, sb = a.read_state(), b.read_state()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(sa[k], sb[k]), k


def test_full_size_tension_cube():
    """The 100 mm cube (218,604 facets, 23k DoFs): 15 steps at 20 explicit
    steps each."""
    s = tension_full()
    dt = 20 * s["dt"]
    o = O.Oracle(s)
    HHT(o, s, dt=dt, alpha=-0.1, tol=OPTS["tol"], max_iter=OPTS["max_iter"]).step(15)
    g = gpu(s)
    g.set_launch(tets_per_block=16, particle_threads=256, xcd_remap=1)
    g.implicit_step(15, dt, alpha=-0.1, **OPTS)
    compare(g, o, 1e-9, "full-size implicit")


def test_implicit_error_paths():
    from paper_2603_13190_amd.ldpm import LdpmError
    s = el_tension()
    dt = 10 * s["dt"]
    with pytest.raises(LdpmError, match="FP64"):
        gpu(s, precision="mixed").implicit_step(1, dt)
    with pytest.raises(LdpmError, match="explicit steps"):
        gpu(s).step(3).implicit_step(1, dt)
    g = gpu(s)
    g.implicit_step(2, dt, **OPTS)
    with pytest.raises(LdpmError, match="implicitly"):
        g.step(1)
    with pytest.raises(LdpmError, match="explicit runs"):
        g.perturb(np.zeros((g.N, 6)))
    with pytest.raises(LdpmError, match="fixed"):
        g.implicit_step(1, 2 * dt, **OPTS)
    with pytest.raises(LdpmError, match="alpha"):
        gpu(s).implicit_step(1, dt, alpha=-0.6)
    with pytest.raises(LdpmError, match="lumped"):
        gpu(S.mass_variant(s, "cell_block")).implicit_step(1, dt)
