"""The C-ABI library loads, exports every declared symbol, and rejects
invalid systems on the host (no GPU needed: validation precedes any device
call)."""
import os
import re

import numpy as np
import pytest

from paper_2603_13190_amd import ldpm
from paper_2603_13190_amd import specimen as S
from tests.conftest import ROOT, cached


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "ldpm.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpm_[a-z_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    L = ldpm.lib()
    names = declared_symbols()
    assert "ldpm_load_system" in names and "ldpm_step" in names
    assert "ldpm_read_state" in names and "ldpm_energy" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(ldpm.EXPORTS) == set(names)


def small():
    return cached("abi_small", lambda: S.few_particle(12, seed=3))


def _load(mod):
    s = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in small().items()}
    s["material"] = dict(s["material"])
    mod(s)
    d, keep = ldpm.make_desc(s)
    return ldpm.try_load(d)


def _set(key, idx, val):
    def f(s):
        s[key][idx] = val
    return f


@pytest.mark.parametrize("name,mod,msg", [
    ("dt", lambda s: s.__setitem__("dt", 0.0), "dt"),
    ("dt_nan", lambda s: s.__setitem__("dt", float("nan")), "dt"),
    ("mass", _set("mass", 3, 0.0), "mass"),
    ("inertia", _set("inertia", (2, 1), -1.0), "rot_inertia"),
    ("node_range", _set("tet_nodes", (0, 0), 10 ** 6), "out of range"),
    ("facet_not_in_tet", lambda s: s["facet_J"].__setitem__(5, (set(range(s["x0"].shape[0])) - set(s["tet_nodes"][0])).pop()), "distinct nodes"),
    ("len", _set("facet_len", 4, -1.0), "length"),
    ("l_t", lambda s: s["material"].__setitem__("l_t", 1.0), "l_t"),
    ("r_s", lambda s: s["material"].__setitem__("r_s", 0.1), "r_s"),
    ("law", lambda s: s["material"].__setitem__("law", 3), "law"),
    ("nan_geom", _set("facet_cI", (7, 1), float("nan")), "non-finite"),
    ("dof_mode", _set("dof_mode", (0, 0), 7), "dof_mode"),
    ("dof_prog", _set("dof_prog", (0, 0), 5), "dof_prog"),
    ("mass_block_not_pd", lambda s: s.__setitem__("mass_block", np.zeros((s["x0"].shape[0], 21))),
     "positive definite"),
    ("mass_block_nan", lambda s: s.__setitem__("mass_block", np.full((s["x0"].shape[0], 21), np.nan)),
     "non-finite mass_block"),
])
def test_invalid_systems_are_rejected(name, mod, msg):
    rc, err, h = _load(mod)
    assert rc == ldpm.LDPM_ERR_ARG, (name, rc, err)
    assert msg in err, (name, err)
    assert h is None


def test_facet_count_must_be_twelve_per_tet():
    s = dict(small())
    d, keep = ldpm.make_desc(s)
    d.n_facets = d.n_facets - 1
    rc, err, _ = ldpm.try_load(d)
    assert rc == ldpm.LDPM_ERR_ARG and "12" in err


def test_batched_offsets_validated():
    a = S.few_particle(10, seed=1)
    b = S.few_particle(12, seed=2)
    c = S.concat_specimens([a, b])
    c["tet_off"] = c["tet_off"].copy()
    c["tet_off"][1] += 1          # a tet of specimen 1 would reference specimen 0's nodes
    d, keep = ldpm.make_desc(c)
    rc, err, _ = ldpm.try_load(d)
    assert rc == ldpm.LDPM_ERR_ARG and "crosses specimens" in err


def test_program_times_must_increase():
    s = dict(S.tension_cube(edge=20.0, seed=1))
    s["prog_t"] = s["prog_t"].copy()
    s["prog_t"][1] = s["prog_t"][0]
    d, keep = ldpm.make_desc(s)
    rc, err, _ = ldpm.try_load(d)
    assert rc == ldpm.LDPM_ERR_ARG and "increase" in err


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        ldpm.System(small())
