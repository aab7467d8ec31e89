"""Helpers shared by the GPU parity tests (no arithmetic of the method)."""
import numpy as np

from paper_2603_13190_amd import specimen as S
from tests.conftest import cached


def rel(a, b):
    """||a - b||_inf / ||b||_inf (0 if both vanish)."""
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    den = np.abs(b).max() if b.size else 0.0
    num = np.abs(a - b).max() if b.size else 0.0
    if den == 0.0:
        return float(num)
    return float(num / den)


def oracle_state(o):
    """Oracle state as an init_state dict for the GPU (accumulators zero)."""
    return dict(q=o.q.copy(), v=o.v.copy(), t=o.t.copy(), emax=o.emax.copy(),
                fext=o.fext.copy(), step=o.step_index)


def tension_small(edge=30.0, seed=2, rate=2.0):
    return cached(("tension", edge, seed, rate),
                  lambda: S.tension_cube(edge=edge, d0=4.0, da=8.0, seed=seed, rate=rate, ramp=2e-4))


def elastic_small(edge=30.0, seed=4):
    return cached(("elastic", edge, seed),
                  lambda: S.elastic_vibration_cube(edge=edge, d0=4.0, da=8.0, seed=seed))


def confined_small(edge=30.0, seed=3, n_steps=1500):
    return cached(("confined", edge, seed, n_steps),
                  lambda: S.confined_compression_cube(edge=edge, d0=4.0, da=8.0, seed=seed,
                                                      pressure=60.0, final_strain=3e-2,
                                                      n_steps=n_steps))


def tension_full():
    return cached("tension_full", lambda: S.tension_cube(edge=100.0, d0=4.0, da=10.0, seed=1))


def elastic_full():
    return cached("elastic_full", lambda: S.elastic_vibration_cube(edge=50.0, d0=4.0, da=8.0, seed=1))


def confined_full():
    return cached("confined_full", lambda: S.confined_compression_cube(edge=150.0, d0=4.0, da=12.0, seed=1))


def batch_full():
    return cached("batch_full", lambda: S.batch_sliding_compression(64, seed=0))


def cylinder_full():
    return cached("cylinder_full", lambda: S.cylinder_cycle(d0=2.0, da=4.0, seed=1))


def cylinder_bench():
    """The benchmark's cylinder: 100 x 200 mm, d 1.1-2.2 mm (12.66M facets)."""
    return cached("cylinder_bench", lambda: S.cylinder_cycle(d0=1.1, da=2.2, seed=1))
