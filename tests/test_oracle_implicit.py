"""Pins of the implicit HHT-alpha oracle (oracle/implicit.py) against what
the mathematics fixes:

- alpha = 0 is the trapezoidal (average-acceleration) rule: for a linear
  system it conserves 1/2 v^T M v + U exactly, so the energy balance closes
  to rounding at any step size, with or without prescribed DoFs; started
  from rest in a mode it gives q_n = cos(n theta) phi with
  cos(theta) = (1 - W^2/4) / (1 + W^2/4), W = w dt, unconditionally;
- alpha = -1/3 damps the highest frequencies by rho_inf = (1 + alpha) /
  (1 - alpha) = 1/2 per step (asymptotically);
- second-order accuracy in dt;
- small steps reproduce the explicit solution of an inelastic run, and the
  modified Newton iteration on the initial stiffness converges before the
  peak.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from oracle.implicit import HHT, elastic_stiffness, gen_alpha_params
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached

MB = S.MATERIAL_MB


def _few_elastic():
    def make():
        s = dict(S.few_particle(12, seed=3))
        s["material"] = dict(MB, law=0)
        return s
    return cached("implicit_few", make)


def _modes(s):
    o = O.Oracle(s)
    K = np.zeros((6 * o.N, 6 * o.N))
    for i in range(6 * o.N):
        q = np.zeros((o.N, 6))
        q.flat[i] = 1.0
        K[:, i] = o.elastic_internal_force(q).ravel()
    K = 0.5 * (K + K.T)
    Mv = np.concatenate([np.repeat(s["mass"][:, None], 3, 1), s["inertia"]], 1).ravel()
    w2, phi = sl.eigh(K, np.diag(Mv))
    return w2, phi, K


def test_elastic_stiffness_is_the_oracle_internal_force():
    s = _few_elastic()
    _, _, K = _modes(s)
    K0 = elastic_stiffness(s).toarray()
    assert np.abs(K0 - K).max() < 1e-12 * np.abs(K).max()


@pytest.mark.parametrize("factor", [1.0, 10.0, 40.0])
def test_trapezoidal_rule_conserves_energy_with_reactions(factor):
    """Elastic tension with prescribed top and bottom faces: W_ext (applied
    forces and reactions, trapezoid) equals W_int + W_kin to rounding."""
    s = cached("implicit_el_tension", lambda: dict(
        S.tension_cube(edge=20.0, d0=4.0, da=8.0, seed=5, rate=2.0, ramp=2e-4), material=dict(MB, law=0)))
    o = O.Oracle(s)
    h = HHT(o, s, dt=factor * s["dt"], alpha=0.0, tol=1e-10, max_iter=20)
    h.step(int(1500 / factor))
    en = o.energies()
    assert en["W_ext"] > 0
    assert en["err"] < 1e-13


def test_trapezoidal_rule_conserves_energy_in_free_vibration():
    s = cached("implicit_el_vib", lambda: S.elastic_vibration_cube(edge=20.0, d0=4.0, da=8.0, seed=5))
    o = O.Oracle(s)
    h = HHT(o, s, dt=20 * s["dt"], alpha=0.0, tol=1e-10, max_iter=20)
    h.step(200)
    en = o.energies()
    assert en["W_kin0"] > 0
    assert en["err"] < 1e-12


@pytest.mark.parametrize("which,W", [(6, 0.5), (20, 3.0), (-1, 30.0)])
def test_trapezoidal_modal_phase(which, W):
    s = dict(_few_elastic())
    w2, phi, _ = _modes(s)
    w = math.sqrt(w2[which])
    dt = W / w
    amp = 1e-3 / np.abs(phi[:, which]).max()
    s["q0"] = (amp * phi[:, which]).reshape(-1, 6)
    o = O.Oracle(s)
    h = HHT(o, s, dt=dt, alpha=0.0, tol=1e-12, max_iter=5)
    th = math.acos((1 - W * W / 4) / (1 + W * W / 4))
    for n in (1, 5, 40):
        h.step(n - o.step_index)
        expect = amp * phi[:, which] * math.cos(n * th)
        assert np.abs(o.q.ravel() - expect).max() < 1e-8 * amp * np.abs(phi[:, which]).max(), (n, W)


def _mode_run(which, W, alpha, n, rho_inf=None):
    s = dict(_few_elastic())
    w2, phi, _ = _modes(s)
    w = math.sqrt(w2[which])
    amp = 1e-3 / np.abs(phi[:, which]).max()
    s["q0"] = (amp * phi[:, which]).reshape(-1, 6)
    o = O.Oracle(s)
    if rho_inf is None:
        h = HHT(o, s, dt=W / w, alpha=alpha, tol=1e-12, max_iter=5)
    else:
        am, af = gen_alpha_params(rho_inf)
        h = HHT(o, s, dt=W / w, tol=1e-12, max_iter=5, alpha_m=am, alpha_f=af)
    peak = 0.0
    for _ in range(n):
        h.step(1)
        peak = max(peak, np.abs(o.q).max())
    return np.abs(o.q).max() / 1e-3, peak / 1e-3


def test_hht_damps_high_frequencies_and_keeps_low_ones():
    """alpha = -1/3 (rho_inf = 1/2) removes the highest mode at W = 1e4
    within 30 steps (the limit amplification decays like n rho_inf^n), while
    the trapezoidal rule keeps its amplitude; at W = 0.05 the dissipation of
    alpha = -1/3 over 100 steps is below 1e-3."""
    end, _ = _mode_run(-1, 1e4, -1.0 / 3.0, 30)
    assert end < 1e-5
    _, peak = _mode_run(-1, 1e4, 0.0, 30)
    assert abs(peak - 1.0) < 1e-6
    _, peak = _mode_run(6, 0.05, -1.0 / 3.0, 100)
    end, _ = _mode_run(6, 0.05, -1.0 / 3.0, 126)   # about one period
    assert peak > 0.999 and end > 0.99


def test_generalised_alpha_spectral_radius_controls_high_frequencies():
    """Generalised-alpha with rho_inf = 0 annihilates the highest mode at
    W = 1e4 (below 1e-6 in 10 steps); rho_inf = 1 keeps it; a low mode keeps
    its amplitude for rho_inf = 0.8."""
    end, _ = _mode_run(-1, 1e4, None, 10, rho_inf=0.0)
    assert end < 1e-6
    end, peak = _mode_run(-1, 1e4, None, 40, rho_inf=1.0)
    assert end > 0.999 and abs(peak - 1.0) < 1e-6
    _, peak = _mode_run(6, 0.05, None, 126, rho_inf=0.8)
    assert peak > 0.999


@pytest.mark.parametrize("rho_inf", [None, 0.8])
def test_hht_is_second_order(rho_inf):
    s = dict(_few_elastic())
    w2, phi, _ = _modes(s)
    w = math.sqrt(w2[6])
    amp = 1e-3 / np.abs(phi[:, 6]).max()
    s["q0"] = (amp * phi[:, 6]).reshape(-1, 6)
    T = 2.75 * (2 * math.pi / w)        # cos(w T) = 0: the error is the phase error
    errs = []
    am, af = gen_alpha_params(rho_inf) if rho_inf is not None else (0.0, 0.1)
    for k in (1, 2):
        n = 40 * k
        o = O.Oracle(s)
        HHT(o, s, dt=T / n, tol=1e-12, max_iter=5, alpha_m=am, alpha_f=af).step(n)
        errs.append(np.abs(o.q.ravel() - amp * phi[:, 6] * math.cos(w * T)).max())
    assert 3.5 < errs[0] / errs[1] < 4.5


def _tension():
    return cached("implicit_tension", lambda: S.tension_cube(edge=30.0, d0=4.0, da=8.0, seed=2, rate=2.0,
                                                            ramp=2e-4))


def test_small_steps_reproduce_the_explicit_run():
    """Inelastic tension before the peak: HHT (alpha = 0) at the explicit
    step follows the explicit trajectory (both second order)."""
    s = _tension()
    prog, area = s["meta"]["load_prog"], s["meta"]["area"]
    oe = O.Oracle(s)
    oi = O.Oracle(s)
    h = HHT(oi, s, dt=s["dt"], alpha=0.0, tol=1e-10, max_iter=50)
    se, si = [], []
    for _ in range(6):
        oe.step(50)
        h.step(50)
        se.append(oe.reaction_sum(prog) / area)
        si.append(oi.reaction_sum(prog) / area)
    se, si = np.array(se), np.array(si)
    assert np.abs(se - si).max() < 2e-2 * np.abs(se).max()
    # the explicit energies after n steps belong to t_{n-1}
    oi2 = O.Oracle(s)
    HHT(oi2, s, dt=s["dt"], alpha=0.0, tol=1e-10, max_iter=50).step(299)
    assert abs(oi2.energies()["W_int"] - oe.energies()["W_int"]) < 2e-3 * oe.energies()["W_int"]


def test_modified_newton_converges_before_the_peak():
    s = _tension()
    o = O.Oracle(s)
    h = HHT(o, s, dt=10 * s["dt"], alpha=-0.1, tol=1e-8, max_iter=100)
    h.step(20)
    ks = [k for k, _ in h.iters]
    assert max(ks) < 100 and all(r <= 1e-8 for _, r in h.iters)
    assert o.emax.max() > s["material"]["sigma_t"] / s["material"]["E0"]   # the run reaches the peak
