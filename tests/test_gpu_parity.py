"""GPU (HIP library, through the C-ABI) against the FP64 CPU oracle.

FP64 path: one-step maps from identical states agree to 1e-12 relative per
field, trajectories to 1e-9 relative (the bar stated for the FP64 path);
integer/bitwise properties (determinism, batching, launch shapes, resume) are
exact.
"""
import numpy as np
import pytest

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached
from tests.gpu_util import (confined_small, elastic_small, oracle_state, rel, tension_full,
                            tension_small)

pytestmark = pytest.mark.gpu

TOL_STEP = 1e-12
TOL_TRAJ = 1e-9


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    return System(sysd, **kw)


def compare(g, o, fields=("q", "v", "t", "emax", "fext"), tol=TOL_TRAJ, what=""):
    st = g.read_state()
    errs = {}
    for f in fields:
        ref = getattr(o, f)
        errs[f] = rel(st[f], ref)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: relative errors above {tol}: {errs}"
    return errs


def test_library_is_the_hip_extension():
    from paper_2603_13190_amd import ldpm
    L = ldpm.lib()
    assert L._name.endswith("libldpm.so")


@pytest.mark.parametrize("tb", [8, 16, 32, 64])
def test_one_step_maps_elastic(tb):
    s = elastic_small()
    o = O.Oracle(s).step(37)
    g = gpu(s, init_state=oracle_state(o))
    g.set_launch(tets_per_block=tb)
    o.step(1)
    g.step(1)
    compare(g, o, tol=TOL_STEP, what=f"elastic TB={tb}")


def test_first_step_from_rest_and_initial_velocity():
    s = elastic_small()
    o = O.Oracle(s).step(1)
    g = gpu(s).step(1)
    compare(g, o, tol=TOL_STEP, what="first step")


@pytest.mark.parametrize("n_before", [50, 400, 900])
def test_one_step_maps_tension(n_before):
    """One step from oracle states before the peak, around it and after it."""
    s = tension_small()
    o = O.Oracle(s).step(n_before)
    g = gpu(s, init_state=oracle_state(o))
    o.step(1)
    g.step(1)
    compare(g, o, tol=TOL_STEP, what=f"tension after {n_before}")


def test_one_step_map_tension_with_reload_rule():
    """k_t = 0.5 (reload from e_tr = k_t (e_max - sigma_bt/E0) after unloading):
    one step from a post-peak oracle state."""
    s = dict(tension_small())
    s["material"] = dict(s["material"], k_t=0.5)
    o = O.Oracle(s).step(900)
    assert (o.emax > s["material"]["sigma_t"] / s["material"]["E0"]).any()
    g = gpu(s, init_state=oracle_state(o))
    o.step(1)
    g.step(1)
    compare(g, o, tol=TOL_STEP, what="tension k_t = 0.5 after 900")


@pytest.mark.parametrize("n_before", [300, 900, 1400])
def test_one_step_maps_confined_compression(n_before):
    s = confined_small()
    o = O.Oracle(s).step(n_before)
    assert (o.t[:, 0] < 0).any()
    g = gpu(s, init_state=oracle_state(o))
    o.step(1)
    g.step(1)
    compare(g, o, tol=TOL_STEP, what=f"confined after {n_before}")


def test_trajectory_elastic_vibration():
    s = elastic_small()
    o = O.Oracle(s)
    g = gpu(s)
    for chunk in (1, 99, 400, 1500):
        o.step(chunk)
        g.step(chunk)
        compare(g, o, fields=("q", "v", "t", "fext"), what=f"elastic step {o.step_index}")
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_ext", "W_kin", "W_kin0"):
        assert abs(eg[k] - eo[k]) <= TOL_TRAJ * max(abs(eo[k]), eo["W_kin0"]), (k, eg[k], eo[k])


def test_trajectory_tension_prepeak():
    s = tension_small()
    o = O.Oracle(s)
    g = gpu(s)
    for chunk in (10, 90, 200):
        o.step(chunk)
        g.step(chunk)
        compare(g, o, what=f"tension step {o.step_index}")
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_ext", "W_kin"):
        assert abs(eg[k] - eo[k]) <= TOL_TRAJ * abs(eo[k]), (k, eg[k], eo[k])


def test_trajectory_tension_postpeak_reported():
    """Past the peak the response is history- and branch-sensitive: compare
    the nominal stress history and energies (divergence is reported)."""
    s = tension_small()
    o = O.Oracle(s)
    g = gpu(s)
    prog = s["meta"]["load_prog"]
    so, sg = [], []
    for _ in range(12):
        o.step(100)
        g.step(100)
        so.append(o.reaction_sum(prog))
        sg.append(g.reaction(prog))
    so, sg = np.array(so), np.array(sg)
    assert np.abs(o.emax).max() > 10 * 4.0 / 43700.0      # well past the peak strain
    assert abs(sg.max() - so.max()) <= 1e-6 * abs(so).max()
    st = g.read_state()
    print("post-peak relative q difference", rel(st["q"], o.q))
    assert rel(st["q"], o.q) < 1e-6


def test_full_size_tension_sampled():
    """The full 100 mm workload at the benchmark's launch shape: a few
    hundred steps against the oracle, all fields."""
    s = tension_full()
    o = O.Oracle(s).step(150)
    g = gpu(s)
    g.set_launch(tets_per_block=16, particle_threads=256, xcd_remap=1)
    g.step(150)
    compare(g, o, what="full-size tension")


def test_determinism_bitwise():
    s = tension_small()
    a = gpu(s).step(700).read_state()
    b = gpu(s).step(700).read_state()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(a[k], b[k]), k


def test_launch_shape_does_not_change_results():
    s = tension_small()
    ref = None
    for tb, pt, rm, sf in ((16, 256, 1, 0), (32, 128, 0, 1), (64, 512, 1, 0), (16, 64, 0, 1), (8, 256, 1, 1),
                           (16, 256, 1, 1)):
        g = gpu(s)
        g.set_launch(tets_per_block=tb, particle_threads=pt, xcd_remap=rm, stream_facets=sf)
        assert g.get_launch()["stream_facets"] == sf
        st = g.step(300).read_state()
        if ref is None:
            ref = st
        else:
            for k in ("q", "v", "t", "emax", "w_int"):
                assert np.array_equal(st[k], ref[k]), (tb, pt, rm, sf, k)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_facet_stream_policy_default_and_results(precision):
    """stream_facets defaults by the facet kernel's bytes per launch (off
    for the small cube) and either setting gives the same state bitwise."""
    s = tension_small()
    g = gpu(s, precision=precision)
    assert g.get_launch()["stream_facets"] == 0
    a = g.step(200).read_state()
    h = gpu(s, precision=precision)
    h.set_launch(tets_per_block=16, stream_facets=1)
    b = h.step(200).read_state()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(a[k], b[k]), k


def test_resume_is_bitwise():
    s = tension_small()
    full = gpu(s).step(500).read_state()
    g1 = gpu(s).step(230)
    mid = g1.read_state()
    g2 = gpu(s, init_state=mid).step(270)
    st = g2.read_state()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(st[k], full[k]), k
    assert st["step"] == 500


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_equals_alone_bitwise(precision):
    specs = [S.tension_cube(edge=e, d0=4.0, da=8.0, seed=i, rate=2.0, ramp=2e-4)
             for i, e in enumerate((20.0, 26.0, 23.0))]
    dt = min(x["dt"] for x in specs)
    batch = S.concat_specimens(specs, dt=dt)
    gb = gpu(batch, precision=precision).step(300)
    sb = gb.read_state()
    po, to = batch["particle_off"], batch["tet_off"]
    for i, sp in enumerate(specs):
        sp = dict(sp)
        sp["dt"] = dt
        st = gpu(sp, precision=precision).step(300).read_state()
        assert np.array_equal(sb["q"][po[i]:po[i + 1]], st["q"])
        assert np.array_equal(sb["t"][12 * to[i]:12 * to[i + 1]], st["t"])
        eb = gb.energy(i)
        ea = gpu(sp, precision=precision).step(300).energy()
        for k in ("W_int", "W_ext", "W_kin", "W_kin0"):
            assert eb[k] == ea[k], (i, k)


def test_single_tet_and_ragged_blocks():
    """One tetrahedron (a block with 15 empty tet slots) and a system whose
    tet count is not a multiple of any block size."""
    for s in (S.single_tet(), S.few_particle(17, seed=9)):
        s = dict(s)
        rng = np.random.default_rng(0)
        s["v0"] = rng.normal(size=s["v0"].shape) * 1e-1
        o = O.Oracle(s).step(60)
        for tb in (16, 64):
            g = gpu(s)
            g.set_launch(tets_per_block=tb)
            g.step(60)
            compare(g, o, fields=("q", "v", "t", "emax"), what=f"{s['name']} TB={tb}")


def test_body_force():
    s = dict(S.few_particle(12, seed=3))
    s["body_force"] = np.array([1e-4, -2e-4, 3e-4])
    o = O.Oracle(s).step(80)
    g = gpu(s).step(80)
    compare(g, o, fields=("q", "v", "fext"), what="body force")


def test_unstable_step_is_reported():
    """dt far above the stability limit: non-finite velocities raise the
    sticky flag and the next synchronising call reports it."""
    from paper_2603_13190_amd.ldpm import LDPM_ERR_UNSTABLE, LdpmError
    s = dict(S.few_particle(12, seed=3))
    s["dt"] = s["dt"] * 50
    s["v0"] = np.ones_like(s["v0"])
    s["material"] = dict(s["material"], law=0)
    g = gpu(s).step(3000)
    with pytest.raises(LdpmError) as ei:
        g.sync()
    assert ei.value.status == LDPM_ERR_UNSTABLE


def test_mixed_precision_accuracy_tension():
    """FP32 facets / FP64 state against the FP64 oracle: peak nominal stress
    within 1 % and energy-balance error within 1e-3."""
    s = tension_small()
    o = O.Oracle(s)
    g = gpu(s, precision="mixed")
    prog = s["meta"]["load_prog"]
    so, sg = [], []
    for _ in range(12):
        o.step(100)
        g.step(100)
        so.append(o.reaction_sum(prog))
        sg.append(g.reaction(prog))
    so, sg = np.array(so), np.array(sg)
    peak_err = abs(sg.max() - so.max()) / abs(so.max())
    eg = g.energy()
    eo = o.energies()
    print("mixed: peak stress error", peak_err, "energy err", eg["err"], "oracle", eo["err"])
    assert peak_err <= 1e-2
    assert eg["err"] <= 1e-3
    assert abs(eg["W_int"] - eo["W_int"]) <= 1e-2 * abs(eo["W_int"])


@pytest.mark.parametrize("tb", [8, 16, 32])
def test_persistent_launch_is_bitwise_equal(tb):
    """n steps in persistent cooperative launches (with a chunk boundary at
    1024 steps) give the same bits as two kernels per step."""
    s = tension_small()
    ref = gpu(s).step(1100).read_state()
    g = gpu(s)
    g.set_launch(tets_per_block=tb, persistent=1)
    st = g.step(1100).read_state()
    g.sync()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(st[k], ref[k]), k


def _uneven3():
    specs = [S.sliding_compression_cube(e, d0=4.0, da=8.0, seed=20 + i, rate=1.0, ramp=2e-4)
             for i, e in enumerate((20.0, 31.0, 25.0))]
    return S.concat_specimens(specs, dt=min(x["dt"] for x in specs))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tb", [8, 16, 32, 64])
def test_persistent_launch_uneven_batch_is_bitwise_equal(precision, tb):
    """Three specimens of uneven size batched into one system: persistent
    cooperative launches (a chunk boundary at 1024 steps) give the same bits
    as two kernels per step, in FP64 and in mixed precision."""
    batch = cached("uneven3_seed20", _uneven3)
    r = gpu(batch, precision=precision)
    r.set_launch(tets_per_block=16, persistent=0)
    ref = r.step(1100).read_state()
    g = gpu(batch, precision=precision)
    g.set_launch(tets_per_block=tb, persistent=1)
    st = g.step(1100).read_state()
    g.sync()
    assert np.abs(st["t"]).max() > 0
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(st[k], ref[k]), k
    for i in range(3):
        assert g.energy(i) == r.energy(i), i


def test_autotune_is_refused_with_a_surrogate_or_a_capture():
    """Trial steps would leave their traces in the surrogate's hand-back
    flags and in a capture's rows: tuning is refused while either is active,
    and the trajectory is untouched."""
    from paper_2603_13190_amd import surrogate as SG
    from paper_2603_13190_amd.ldpm import LDPM_ERR_STATE, LdpmError
    s = tension_small()
    g = gpu(s, precision="mixed")
    g.set_surrogate(SG.init_params(0), np.zeros(9), np.ones(9), np.ones(3), np.full(9, -1.0),
                    np.full(9, 1.0), 0.8, 0.9, 0.05)
    g.step(10)
    with pytest.raises(LdpmError) as ei:
        g.autotune(steps_per_trial=5)
    assert ei.value.status == LDPM_ERR_STATE
    assert g.read_state()["step"] == 10
    c = gpu(s, precision="fp64")
    c.capture_begin(1000, facet_stride=50, facet_offset=0, step_stride=5, kappa_t=1.1, kappa_c=0.9,
                    damage_max=0.05)
    c.step(10)
    with pytest.raises(LdpmError) as ei:
        c.autotune(steps_per_trial=5)
    assert ei.value.status == LDPM_ERR_STATE
    rows = c.capture_end()
    assert set(np.unique(rows["step"])) <= {0, 5}


def test_autotune_keeps_the_trajectory():
    """The autotuner runs trials on the live system and restores its state:
    the continued trajectory is bitwise the one without tuning."""
    s = tension_small()
    ref = gpu(s).step(300).read_state()
    g = gpu(s).step(100)
    best, us, trials = g.autotune(steps_per_trial=20)
    assert len(trials) == 37 and us > 0
    assert best in [t[0] for t in trials]
    # 36 shapes at the handle's facet-stream policy, then the best one with the other
    assert {t[0]["stream_facets"] for t in trials[:36]} == {0}
    assert trials[36][0] == dict(min(trials[:36], key=lambda t: t[1])[0], stream_facets=1)
    st = g.step(200).read_state()
    for k in ("q", "v", "t", "emax", "fext", "w_int", "w_ext", "w_kin"):
        assert np.array_equal(st[k], ref[k]), k
    assert g.get_launch() == best


def test_autotune_choice_is_cached_per_shape():
    """A second system of the same shape (and precision) reuses the tuned
    launch shape without new trials."""
    s = tension_small()
    g1 = gpu(s)
    best1, _, trials1 = g1.autotune(steps_per_trial=10)
    g2 = gpu(s)
    best2, _, trials2 = g2.autotune(steps_per_trial=10)
    assert len(trials2) == 0
    assert best2 == best1 == g2.get_launch()


def test_batched_uneven_specimens_against_oracle():
    """Three specimens of uneven size in one batched system: per-specimen
    energies and reactions from the GPU against the oracle run of each."""
    specs = [S.sliding_compression_cube(e, d0=4.0, da=8.0, seed=10 + i, rate=1.0, ramp=2e-4)
             for i, e in enumerate((20.0, 31.0, 25.0))]
    dt = min(x["dt"] for x in specs)
    batch = S.concat_specimens(specs, dt=dt)
    g = gpu(batch)
    g.set_launch(tets_per_block=32)
    g.step(400)
    for i, sp in enumerate(specs):
        sp = dict(sp)
        sp["dt"] = dt
        o = O.Oracle(sp).step(400)
        eo, eg = o.energies(), g.energy(i)
        for k in ("W_int", "W_ext", "W_kin"):
            assert abs(eg[k] - eo[k]) <= TOL_TRAJ * abs(eo[k]), (i, k, eg[k], eo[k])
        ro = o.reaction_sum(sp["meta"]["load_prog"])
        rg = g.reaction(i)          # specimen i's single program is batched id i
        assert abs(rg - ro) <= TOL_TRAJ * abs(ro), (i, rg, ro)
