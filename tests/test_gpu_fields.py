"""Crack-opening field, volumetric-strain field, field comparison and random
perturbation: the HIP library (through the C-ABI) against the FP64 oracle.

FP64: fields and perturbed trajectories within 1e-9 relative (the bar of
the FP64 path), one-jump maps within 1e-12, comparison statistics within
1e-12; masking, batching and determinism exact.
"""
import numpy as np
import pytest

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.gpu_util import oracle_state, rel, tension_full, tension_small, confined_full

pytestmark = pytest.mark.gpu


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    return System(sysd, **kw)


def host(t):
    return t.cpu().numpy()


def _crack_gpu(g):
    return host(g.crack_opening()).T        # (F, 4)


def _field_close(a, b, tol, what, floor=0.0):
    scale = max(np.abs(b).max(), floor)
    assert scale > 0, what
    err = np.abs(a - b).max() / scale
    assert err <= tol, f"{what}: {err}"


# ------------------------------------------------------------ crack opening
@pytest.mark.parametrize("n_steps", [0, 1, 300, 1100])
def test_crack_opening_along_the_tension_trajectory(n_steps):
    """Before the peak, around it and well past it (open cracks), within the
    trajectory bar."""
    s = tension_small()
    o = O.Oracle(s).step(n_steps)
    g = gpu(s).step(n_steps)
    wg, wo = _crack_gpu(g), o.crack_opening()
    assert np.all(wg[:, 0] >= 0.0)
    if n_steps == 0:
        assert np.all(wg == 0.0)
        return
    floor = np.abs(o.strains(o.q)).max() * s["facet_len"].max()
    scale = max(np.abs(wo).max(), floor)
    tol = 1e-9
    err = np.abs(wg - wo).max() / scale
    print(f"crack opening after {n_steps} steps: max |w| {np.abs(wo).max():.3e}, rel. difference {err:.2e}")
    assert err <= tol, n_steps
    if n_steps == 1100:
        assert wo[:, 3].max() > 1e-4          # cracks are open


def test_crack_opening_one_step_after_an_oracle_state():
    """From the oracle's post-peak state, one step on each side: the fields
    agree to the one-step bar."""
    s = tension_small()
    o = O.Oracle(s).step(1000)
    g = gpu(s, init_state=oracle_state(o))
    o.step(1)
    g.step(1)
    _field_close(_crack_gpu(g), o.crack_opening(), 1e-12, "crack one step")


def test_crack_opening_mixed_precision_close_to_fp64():
    s = tension_small()
    a = gpu(s, precision="fp64").step(1100)
    b = gpu(s, precision="mixed").step(1100)
    from paper_2603_13190_amd.ldpm import compare_fields
    st = compare_fields(b.crack_opening()[3].contiguous(), a.crack_opening()[3].contiguous())
    print("mixed vs FP64 crack pattern", st)
    assert st["pearson"] > 0.95 and st["nrmse"] < 5.0, st


def test_crack_opening_full_size_from_a_seeded_state():
    """The 100 mm cube (218k facets) from a seeded loaded state (strains,
    velocities and history drawn by the input generator)."""
    s = tension_full()
    st = S.synthetic_state(s, seed=11, strain=np.diag([-5e-5, -5e-5, 3e-4]))
    o = O.Oracle(s)
    o.set_state(st["q"], st["v"], st["t"], o.strains(st["q"] - s["dt"] * st["v"]), st["emax"], st["fext"],
                st["step"])
    g = gpu(s, init_state=st)
    g.set_launch(tets_per_block=16, particle_threads=256, xcd_remap=1)
    wo = o.crack_opening()
    assert (wo[:, 0] > 0).sum() > 1000 and (wo[:, 0] == 0).sum() > 1000
    _field_close(_crack_gpu(g), wo, 1e-12, "full-size crack")


# ------------------------------------------------------- volumetric strains
@pytest.mark.parametrize("n_steps", [0, 1, 700])
def test_volumetric_strain_field(n_steps):
    s = tension_small()
    o = O.Oracle(s).step(n_steps)
    g = gpu(s).step(n_steps)
    ev = host(g.volumetric_strain())
    if n_steps == 0:
        assert np.all(ev == 0.0)
        return
    # after one step the field is that of q^0 = 0: compare on the scale of
    # the current configuration's strains
    floor = np.abs(o.volstrains(o.q)).max()
    _field_close(ev, o.volumetric_strain_field(), 1e-9, f"e_V after {n_steps}", floor=floor)


def test_volumetric_strain_full_size_confined_from_a_seeded_state():
    s = confined_full()
    st = S.synthetic_state(s, seed=12, strain=np.diag([-2e-3, -2e-3, -6e-3]))
    o = O.Oracle(s)
    o.set_state(st["q"], st["v"], st["t"], o.strains(st["q"] - s["dt"] * st["v"]), st["emax"], st["fext"],
                st["step"])
    g = gpu(s, init_state=st)
    _field_close(host(g.volumetric_strain()), o.volumetric_strain_field(), 1e-12, "confined e_V")


# ---------------------------------------------------------- field comparison
def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 4097, 1_000_003])
def test_compare_fields_matches_oracle(n):
    from paper_2603_13190_amd.ldpm import compare_fields
    rng = np.random.default_rng(n)
    x = np.abs(rng.standard_cauchy(n)) * 0.1
    r = np.abs(x + rng.normal(scale=0.05, size=n))
    for cap in (None, 4.0):
        so = O.field_stats(x, r, cap=cap)
        sg = compare_fields(_dev(x), _dev(r), cap=cap)
        assert sg["n"] == n
        assert sg["ref_max"] == so["ref_max"]
        for k in ("mean_x", "mean_ref", "rmse", "nrmse"):
            assert abs(sg[k] - so[k]) <= 1e-12 * abs(so[k]), (n, cap, k, sg[k], so[k])
        if n == 1:
            assert np.isnan(sg["pearson"]) and np.isnan(so["pearson"])
        else:
            assert abs(sg["pearson"] - so["pearson"]) <= 1e-12, (n, cap, sg["pearson"], so["pearson"])


def test_compare_fields_is_deterministic_and_exact_on_identities():
    from paper_2603_13190_amd.ldpm import compare_fields
    rng = np.random.default_rng(1)
    r = rng.exponential(1.0, 12_660_001)
    dr = _dev(r)
    a = compare_fields(dr, dr)
    b = compare_fields(dr, dr)
    assert a == b
    assert a["nrmse"] == 0.0 and abs(a["pearson"] - 1.0) < 1e-14
    c = compare_fields(_dev(r + 0.25), dr)
    assert abs(c["nrmse"] - 25.0 / r.max()) < 1e-12 * c["nrmse"]
    z = compare_fields(_dev(np.ones(5)), _dev(np.zeros(5)))
    assert np.isnan(z["pearson"]) and np.isinf(z["nrmse"])


def test_compare_fields_rejects_host_memory():
    from paper_2603_13190_amd import ldpm
    import ctypes as C
    x = np.ones(8)
    o = ldpm.FieldStats()
    rc = ldpm.lib().ldpm_compare_fields(x.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p), 8, 0.0,
                                        None, C.byref(o))
    assert rc == ldpm.LDPM_ERR_ARG and "device memory" in ldpm.lib().ldpm_last_error().decode()


# ------------------------------------------------------ random perturbation
def _compare_states(g, o, tol, what):
    st = g.read_state()
    for f in ("q", "v", "t", "emax", "fext"):
        e = rel(st[f], getattr(o, f))
        assert e <= tol, (what, f, e)


def test_perturbed_trajectory_matches_oracle():
    """Perturbations every 100 steps before the peak, then every 200 steps
    through the softening, within the trajectory bar."""
    s = tension_small()
    o = O.Oracle(s)
    g = gpu(s)
    eta = 2e-5
    tol = 1e-9
    for k, n in enumerate([100] * 3 + [200] * 4):
        o.step(n)
        g.step(n)
        d = S.perturbation(o.N, eta, seed=21, index=k)
        wo = o.perturb(d)
        wg = g.perturb(d)
        assert abs(wg - wo) <= tol * abs(wo), (k, wg, wo)
        _compare_states(g, o, tol, f"after jump {k}")
        if k == 2:
            eo, eg = o.energies(), g.energy()
            for key in ("W_int", "W_ext", "W_kin", "W_pert"):
                assert abs(eg[key] - eo[key]) <= 1e-9 * abs(eo[key]), (key, eg[key], eo[key])
    eo, eg = o.energies(), g.energy()
    for key in ("W_int", "W_ext", "W_kin", "W_pert"):
        assert abs(eg[key] - eo[key]) <= 1e-9 * abs(eo[key]), (key, eg[key], eo[key])
    wg, wo = _crack_gpu(g), o.crack_opening()
    assert np.abs(wg - wo).max() <= 1e-9 * np.abs(wo).max()


def test_one_jump_map_from_an_oracle_state():
    s = tension_small()
    o = O.Oracle(s).step(900)
    g = gpu(s, init_state=oracle_state(o))
    d = S.perturbation(o.N, 5e-5, seed=22, index=0)
    wo, wg = o.perturb(d), g.perturb(d)
    assert abs(wg - wo) <= 1e-12 * abs(wo)
    _compare_states(g, o, 1e-12, "one jump")


def test_jump_masks_prescribed_dofs_bitwise():
    s = tension_small()
    g = gpu(s).step(50)
    q0 = g.read_state()["q"]
    d = S.perturbation(q0.shape[0], 1e-4, seed=23, index=0)
    g.perturb(d)
    q1 = g.read_state()["q"]
    free = s["dof_mode"] == 0
    assert np.array_equal(q1[~free], q0[~free])
    assert np.array_equal(q1[free], q0[free] + d[free])


def test_jump_before_the_first_step():
    s = tension_small()
    o = O.Oracle(s)
    g = gpu(s)
    d = S.perturbation(o.N, 1e-4, seed=24, index=0)
    assert g.perturb(d) == 0.0 and o.perturb(d) == 0.0
    o.step(30)
    g.step(30)
    _compare_states(g, o, 1e-12, "jump at step 0")


def test_jump_full_size_from_a_seeded_state():
    s = tension_full()
    st = S.synthetic_state(s, seed=13, strain=np.diag([-5e-5, -5e-5, 2e-4]))
    o = O.Oracle(s)
    o.set_state(st["q"], st["v"], st["t"], o.strains(st["q"] - s["dt"] * st["v"]), st["emax"], st["fext"],
                st["step"])
    g = gpu(s, init_state=st)
    d = S.perturbation(o.N, 2e-5, seed=25, index=0)
    wo, wg = o.perturb(d), g.perturb(d)
    assert abs(wg - wo) <= 1e-12 * abs(wo)
    _compare_states(g, o, 1e-12, "full-size jump")


def test_batched_jump_equals_alone_bitwise():
    specs = [S.tension_cube(edge=e, d0=4.0, da=8.0, seed=i, rate=2.0, ramp=2e-4)
             for i, e in enumerate((20.0, 26.0))]
    dt = min(x["dt"] for x in specs)
    batch = S.concat_specimens(specs, dt=dt)
    po, to = batch["particle_off"], batch["tet_off"]
    ds = [S.perturbation(sp["x0"].shape[0], 1e-4, seed=26, index=i) for i, sp in enumerate(specs)]
    gb = gpu(batch).step(200)
    gb.perturb(np.concatenate(ds))
    sb = gb.step(50).read_state()
    for i, sp in enumerate(specs):
        sp = dict(sp)
        sp["dt"] = dt
        ga = gpu(sp).step(200)
        ga.perturb(ds[i])
        sa = ga.step(50).read_state()
        assert np.array_equal(sb["q"][po[i]:po[i + 1]], sa["q"])
        assert np.array_equal(sb["t"][12 * to[i]:12 * to[i + 1]], sa["t"])
        ea, eb = ga.energy(), gb.energy(i)
        for k in ("W_int", "W_ext", "W_kin", "W_pert"):
            assert ea[k] == eb[k], (i, k)


def test_jump_in_mixed_precision_and_resume_keeps_w_pert():
    s = tension_small()
    a = gpu(s, precision="fp64").step(300)
    b = gpu(s, precision="mixed").step(300)
    d = S.perturbation(a.N, 5e-5, seed=27, index=0)
    wa, wb = a.perturb(d), b.perturb(d)
    assert abs(wb - wa) <= 1e-3 * abs(wa)
    st = a.read_state()
    assert st["w_pert"][0] == wa
    c = gpu(s, precision="fp64", init_state=st)
    assert c.energy()["W_pert"] == wa
