"""Full-size workloads in the benchmark's launch shape against the oracle,
on outputs the oracle can compute in seconds."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import (batch_full, confined_full, cylinder_full, elastic_full, rel)

pytestmark = pytest.mark.gpu

BENCH_LAUNCH = dict(tets_per_block=16, particle_threads=256, xcd_remap=1)


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    g = System(sysd, **kw)
    g.set_launch(**BENCH_LAUNCH)
    return g


def test_elastic_cube50_whole_trajectory():
    """50 mm elastic cube, initial sinusoidal velocity, 10k steps: state and
    energies along the whole trajectory within 1e-9."""
    s = elastic_full()
    o = O.Oracle(s)
    g = gpu(s)
    for _ in range(4):
        o.step(2500)
        g.step(2500)
        st = g.read_state()
        for f in ("q", "v", "t"):
            assert rel(st[f], getattr(o, f)) <= 1e-9, f
    eo, eg = o.energies(), g.energy()
    for k in ("W_int", "W_kin", "W_kin0"):
        assert abs(eg[k] - eo[k]) <= 1e-9 * eo["W_kin0"], k
    assert eg["err"] < 1e-3


def test_confined_cube150_one_step_from_a_seeded_loaded_state():
    """150 mm confined compression (648k facets): one step from a seeded
    loaded state (compressive strain field with noise, velocities, facet
    history, drawn by the input generator), on both sides."""
    from paper_2603_13190_amd import specimen as S
    s = confined_full()
    st = S.synthetic_state(s, seed=5, strain=np.diag([-2e-3, -2e-3, -6e-3]), t_normal=(-150.0, 0.0),
                           t_shear=20.0, step=60000)
    o = O.Oracle(s)
    e_old = o.strains(st["q"] - s["dt"] * st["v"])     # q^{n-1} = q^n - dt v^{n-1/2}
    o.set_state(st["q"], st["v"], st["t"], e_old, st["emax"], st["fext"], st["step"])
    g = gpu(s, init_state=st)
    o.step(1)
    g.step(1)
    assert (o.t[:, 0] < -1.0).sum() > 100000            # compressive facets
    assert (o.e[:, 0] < -s["material"]["sigma_c0"] / s["material"]["E0"]).sum() > 1000   # beyond pore collapse
    st2 = g.read_state()
    for f in ("q", "v", "t", "emax", "fext"):
        assert rel(st2[f], getattr(o, f)) <= 1e-10, f


def test_batch64_sampled_specimens():
    """The 64-specimen batch (6.9M facets): 300 steps, four specimens checked
    against oracle runs of each alone (same dt)."""
    from paper_2603_13190_amd import specimen as S
    b = batch_full()
    g = gpu(b).step(300)
    st = g.read_state()
    po, to = b["particle_off"], b["tet_off"]
    rng = np.random.default_rng(0)
    for i in sorted(rng.choice(64, 4, replace=False)):
        sp = S.sliding_compression_cube(b["meta"]["edges"][i], d0=4.0, da=8.0, seed=int(i), rate=2.5e-2)
        sp["dt"] = b["dt"]
        assert sp["meta"]["F"] == b["meta"]["specimen_F"][i]
        o = O.Oracle(sp).step(300)
        assert rel(st["q"][po[i]:po[i + 1]], o.q) <= 1e-9, i
        assert rel(st["t"][12 * to[i]:12 * to[i + 1]], o.t) <= 1e-9, i
        eo, eg = o.energies(), g.energy(int(i))
        assert abs(eg["W_int"] - eo["W_int"]) <= 1e-9 * abs(eo["W_int"]), i


def test_cylinder_sampled():
    """100 x 200 mm cylinder (2.3M facets): 200 steps against the oracle."""
    s = cylinder_full()
    o = O.Oracle(s).step(200)
    g = gpu(s).step(200)
    st = g.read_state()
    for f in ("q", "v", "t"):
        assert rel(st[f], getattr(o, f)) <= 1e-9, f
