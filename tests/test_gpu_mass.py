"""Full cell mass blocks (eq. balance) on the GPU against the FP64 oracle,
and the sphere-inertia variant (a diagonal input, same kernels as the
lumped path).

FP64 bar: one-step maps 1e-12, trajectories 1e-9; launch shapes and
batching bitwise.
"""
import numpy as np
import pytest

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.conftest import cached
from tests.gpu_util import elastic_full, oracle_state, rel, tension_small

pytestmark = pytest.mark.gpu


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    return System(sysd, **kw)


def compare(g, o, tol, what, fields=("q", "v", "t", "emax", "fext")):
    st = g.read_state()
    for f in fields:
        e = rel(st[f], getattr(o, f))
        assert e <= tol, (what, f, e)


def block(s):
    return S.mass_variant(s, "cell_block")


def tension_block():
    return cached("tension_block", lambda: block(tension_small()))


@pytest.mark.parametrize("n_before", [0, 50, 900])
def test_one_step_maps_with_the_cell_block(n_before):
    s = tension_block()
    o = O.Oracle(s).step(n_before)
    g = gpu(s, init_state=oracle_state(o)) if n_before else gpu(s)
    o.step(1)
    g.step(1)
    compare(g, o, 1e-12, f"block, one step after {n_before}")


def test_trajectory_with_the_cell_block():
    s = tension_block()
    o = O.Oracle(s)
    g = gpu(s)
    for chunk in (10, 90, 200):
        o.step(chunk)
        g.step(chunk)
        compare(g, o, 1e-9, f"block trajectory step {o.step_index}")
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_ext", "W_kin", "W_kin0"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * abs(eo[k]), (k, eg[k], eo[k])


def test_elastic_cube50_with_the_cell_block():
    """The 50 mm elastic vibration cube (full size) with the cell blocks:
    2000 steps against the oracle, energies included."""
    s = cached("elastic_block", lambda: block(elastic_full()))
    o = O.Oracle(s).step(2000)
    g = gpu(s)
    g.set_launch(tets_per_block=16, particle_threads=256, xcd_remap=1)
    g.step(2000)
    compare(g, o, 1e-9, "elastic cube 50 block", fields=("q", "v", "t"))
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_kin", "W_kin0"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * eo["W_kin0"], k


def test_rigid_motion_kinetic_energy_on_the_gpu():
    s = dict(tension_block())
    N = s["x0"].shape[0]
    s["dof_mode"] = np.zeros((N, 6), np.uint8)
    s["dof_prog"] = -np.ones((N, 6), np.int32)
    s["dof_scale"] = np.zeros((N, 6))
    s["material"] = dict(s["material"], law=0)
    s = block(s)
    V, W = np.array([0.3, -0.2, 0.5]), np.array([2.0, -1.0, 3.0])
    v0 = np.zeros((N, 6))
    v0[:, :3] = V + np.cross(W, s["x0"])
    v0[:, 3:] = W
    s["v0"] = v0
    o = O.Oracle(s).step(30)
    g = gpu(s).step(30)
    eg = g.energy()
    assert abs(eg["W_kin0"] - o.energies()["W_kin0"]) <= 1e-13 * eg["W_kin0"]
    assert abs(eg["W_kin"] - eg["W_kin0"]) <= 1e-9 * eg["W_kin0"]
    assert rel(g.read_state()["v"], v0) <= 1e-9


def test_cell_block_launch_shapes_and_batching_are_bitwise():
    s = tension_block()
    ref = None
    for tb, pt, rm in ((16, 256, 1), (32, 64, 0), (8, 1024, 1)):
        g = gpu(s)
        g.set_launch(tets_per_block=tb, particle_threads=pt, xcd_remap=rm)
        st = g.step(300).read_state()
        if ref is None:
            ref = st
        else:
            for k in ("q", "v", "t", "w_int", "w_kin"):
                assert np.array_equal(st[k], ref[k]), (tb, pt, rm, k)
    specs = [block(S.tension_cube(edge=e, d0=4.0, da=8.0, seed=i, rate=2.0, ramp=2e-4))
             for i, e in enumerate((20.0, 24.0))]
    dt = min(x["dt"] for x in specs)
    batch = S.concat_specimens(specs, dt=dt)
    assert "mass_block" in batch
    sb = gpu(batch).step(200).read_state()
    po = batch["particle_off"]
    for i, sp in enumerate(specs):
        sa = gpu(dict(sp, dt=dt)).step(200).read_state()
        assert np.array_equal(sb["q"][po[i]:po[i + 1]], sa["q"])


def test_cell_block_rejects_the_persistent_launch_and_tunes_without_it():
    from paper_2603_13190_amd.ldpm import LdpmError
    s = tension_block()
    g = gpu(s)
    with pytest.raises(LdpmError, match="persistent"):
        g.set_launch(tets_per_block=16, persistent=1)
    best, us, trials = g.autotune(steps_per_trial=5)
    assert len(trials) == 33 and best["persistent"] == 0


def test_sphere_variant_against_the_oracle():
    s = cached("tension_sphere", lambda: S.mass_variant(tension_small(), "sphere"))
    o = O.Oracle(s).step(300)
    g = gpu(s).step(300)
    compare(g, o, 1e-9, "sphere inertia")


def test_mixed_precision_with_the_cell_block():
    s = tension_block()
    a = gpu(s, precision="fp64").step(400)
    b = gpu(s, precision="mixed").step(400)
    assert rel(b.read_state()["q"], a.read_state()["q"]) < 1e-4
