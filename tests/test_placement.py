"""The input generator's native placement loop (gen/placement.c) accepts
exactly the candidates its Python loop accepts: identical centres and
diameters, bit for bit, on boxes and cylinders of several sizes and seeds.
Input-generator code, no GPU."""
import numpy as np
import pytest

from paper_2603_13190_amd import gen
from paper_2603_13190_amd import specimen as S


def _place(shape, d0, da, seed, native):
    rng = np.random.default_rng(seed)
    return S.place_particles(shape, d0, da, rng, native=native)


@pytest.mark.parametrize("shape,d0,da,seed", [
    (S.Shape("box", (30.0, 30.0, 30.0)), 4.0, 8.0, 1),
    (S.Shape("box", (50.0, 40.0, 30.0)), 3.0, 6.0, 7),
    (S.Shape("cylinder", (40.0, 60.0)), 2.0, 4.0, 3),
    (S.Shape("cylinder", (30.0, 30.0)), 2.0, 5.0, 11),
])
def test_native_placement_is_the_python_placement(shape, d0, da, seed):
    assert gen.lib() is not None
    xp, dp = _place(shape, d0, da, seed, native=False)
    xn, dn = _place(shape, d0, da, seed, native=True)
    assert xp.shape[0] > 20
    assert np.array_equal(xn, xp) and np.array_equal(dn, dp)


def test_native_placement_keeps_the_gap():
    shape = S.Shape("box", (40.0, 40.0, 40.0))
    gap = 0.1
    x, d = _place(shape, 2.0, 5.0, 5, native=True)
    r = 0.5 * d
    dd = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    lim = (r[:, None] + r[None, :]) * (1.0 + gap)
    np.fill_diagonal(dd, np.inf)
    assert np.all(dd >= lim)

