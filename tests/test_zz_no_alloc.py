"""The allocation-free field comparison (ldpm_compare_fields_noalloc: block
partials and results in the library's static per-GPU device buffer) against
ldpm_compare_fields (its own buffer from hipMalloc), through the C-ABI: two
calls in a row, the second on a smaller input, each bitwise equal to the
allocating entry point on the same fields."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _fields(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    ref = np.abs(rng.normal(size=n)) * 0.5
    x = ref + 1e-3 * rng.normal(size=n)
    return (torch.tensor(x, dtype=torch.float64, device="cuda"),
            torch.tensor(ref, dtype=torch.float64, device="cuda"), x, ref)


def _same(a, b):
    for k in a:
        va, vb = a[k], b[k]
        if isinstance(va, float) and math.isnan(va):
            assert math.isnan(vb), k
        else:
            assert va == vb, (k, va, vb)


def test_noalloc_comparison_equals_the_allocating_one_on_two_calls():
    from paper_2603_13190_amd.ldpm import compare_fields
    # first call: more blocks than the grid cap (grid-stride partials), with a cap
    x, r, xh, rh = _fields(1_000_003, 1)
    a = compare_fields(x, r, cap=1.5, noalloc=True)
    b = compare_fields(x, r, cap=1.5)
    _same(a, b)
    xc, rc = np.minimum(xh, 1.5), np.minimum(rh, 1.5)
    assert a["n"] == xh.size
    assert abs(a["pearson"] - np.corrcoef(xc, rc)[0, 1]) <= 1e-12
    assert abs(a["nrmse"] - 100.0 / rc.max() * math.sqrt(np.mean((xc - rc) ** 2))) <= 1e-10 * a["nrmse"]
    # second call, smaller (fewer blocks than the first left partials for)
    x2, r2, xh2, rh2 = _fields(5_001, 2)
    a2 = compare_fields(x2, r2, noalloc=True)
    b2 = compare_fields(x2, r2)
    _same(a2, b2)
    assert a2["n"] == 5_001
    assert abs(a2["pearson"] - np.corrcoef(xh2, rh2)[0, 1]) <= 1e-12
    # and once more on the first fields: nothing of the second call is left over
    _same(compare_fields(x, r, cap=1.5, noalloc=True), b)


def test_noalloc_comparison_errors():
    """Host arguments and a non-positive n are refused with LDPM_ERR_ARG."""
    import ctypes as C
    import torch
    from paper_2603_13190_amd import ldpm
    L = ldpm.lib()
    fn = L.ldpm_compare_fields_noalloc
    o = ldpm.FieldStats()
    h = np.ones(8)
    assert fn(h.ctypes.data_as(C.c_void_p), h.ctypes.data_as(C.c_void_p), 8, 0.0, None,
              C.byref(o)) == ldpm.LDPM_ERR_ARG
    d = torch.ones(8, dtype=torch.float64, device="cuda")
    assert fn(C.c_void_p(d.data_ptr()), C.c_void_p(d.data_ptr()), 0, 0.0, None, C.byref(o)) == ldpm.LDPM_ERR_ARG
