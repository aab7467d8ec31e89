"""Facet-law surrogate inside the step (BF16 MFMA inference, sticky fallback
to the exact FP32 law) and capture of its training samples."""
import numpy as np
import pytest

import oracle as O
from paper_2603_13190_amd import specimen as S
from tests.gpu_util import confined_small, tension_small

pytestmark = pytest.mark.gpu

KT, KC, DMAX = 1.1, 0.9, 0.05


def gpu(sysd, **kw):
    from paper_2603_13190_amd.ldpm import System
    return System(sysd, **kw)


def _frame_features(p, e, eo, told):
    """Features in the frame of the trial shear traction (independent of the
    GPU code: written from the feature definition)."""
    de = e - eo
    al, E0 = p["alpha"], p["E0"]
    ts = told[:, 1:] + al * E0 * de[:, 1:]
    nrm = np.sqrt((ts.astype(np.float32) ** 2).sum(1))
    u = np.where(nrm[:, None] > 1e-15, ts / np.where(nrm > 0, nrm, 1)[:, None], [1.0, 0.0])

    def rot(a):
        return a[:, 0] * u[:, 0] + a[:, 1] * u[:, 1], -a[:, 0] * u[:, 1] + a[:, 1] * u[:, 0]
    x = np.zeros((e.shape[0], 9))
    x[:, 0] = de[:, 0]
    x[:, 1], x[:, 2] = rot(de[:, 1:])
    x[:, 3] = eo[:, 0]
    x[:, 4], x[:, 5] = rot(eo[:, 1:])
    x[:, 6] = told[:, 0]
    x[:, 7], x[:, 8] = rot(told[:, 1:])
    return x, rot


def test_capture_rows_match_oracle_law():
    """Captured features and exact residuals of sampled facets at one step
    equal those recomputed from the oracle's state and law."""
    s = tension_small()
    p = s["material"]
    g = gpu(s, precision="fp64")
    g.capture_begin(200000, facet_stride=3, facet_offset=1, step_stride=100, kappa_t=KT,
                    kappa_c=KC, damage_max=DMAX)
    g.step(301)
    rows = g.capture_end()
    assert rows["offered"] == rows["x"].shape[0] > 0
    assert np.all(rows["facet"] % 3 == 1) and set(np.unique(rows["step"])) <= {0, 100, 200, 300}
    n = 200
    o = O.Oracle(s).step(n)          # state before step n
    eo, told = o.e.copy(), o.t.copy()
    e = o.strains()
    ev = o.volstrains()[s["facet_tet"]]
    sel = rows["step"] == n
    fac = rows["facet"][sel].astype(np.int64)
    tnew = np.zeros((fac.size, 3))
    for i, f in enumerate(fac):
        tnew[i], _ = O.facet_law(p, s["facet_len"][f], e[f], eo[f], ev[f], told[f], o.emax[f])
    x, rot = _frame_features(p, e[fac], eo[fac], told[fac])
    r = tnew - (told[fac] + p["E0"] * np.array([1, p["alpha"], p["alpha"]]) * (e[fac] - eo[fac]))
    rp, rq = rot(r[:, 1:])
    # the perpendicular components cancel in FP32: tolerances per vector group
    err = np.abs(rows["x"][sel] - x)
    for g0 in (0, 3, 6):
        scale = np.abs(x[:, g0:g0 + 3]).max()
        print("feature group", g0, "max err / scale", err[:, g0:g0 + 3].max() / scale)
        assert err[:, g0:g0 + 3].max() <= 1e-5 * scale
    tsc = np.abs(told).max()
    # residual scale |t_old + E de| (float 14 of a row)
    ttr = told[fac] + p["E0"] * np.array([1, p["alpha"], p["alpha"]]) * (e[fac] - eo[fac])
    s_ref = np.linalg.norm(ttr, axis=1)
    assert np.abs(rows["s"][sel] - s_ref).max() <= 1e-6 * s_ref.max()
    assert np.abs(rows["y"][sel][:, 0] - r[:, 0]).max() <= 1e-6 * tsc
    assert np.abs(rows["y"][sel][:, 1] - rp).max() <= 1e-6 * tsc
    assert np.abs(rows["y"][sel][:, 2] - rq).max() <= 1e-6 * tsc


def test_surrogate_fallback_is_bitwise_the_fp32_law():
    """With an empty envelope every facet is handed back at once: the run is
    bitwise the plain mixed-precision run."""
    from paper_2603_13190_amd import surrogate as SG
    s = tension_small()
    ref = gpu(s, precision="mixed").step(400).read_state()
    g = gpu(s, precision="mixed")
    lo = np.full(9, 1.0)
    hi = np.full(9, -1.0)      # empty box
    g.set_surrogate(SG.init_params(0), np.zeros(9), np.ones(9), np.ones(3), lo, hi, KT, KC, DMAX)
    st = g.step(400).read_state()
    assert g.surrogate_count() == s["meta"]["F"]
    for k in ("q", "v", "t", "emax", "fext", "w_int"):
        assert np.array_equal(st[k], ref[k]), k


def test_surrogate_end_to_end_accuracy_and_sticky_gate():
    """Capture from FP64 runs (tension and confined compression), train on
    the GPU, install into a mixed run of the tension specimen: the nominal
    stress history stays close to the FP64 oracle, the energy balance holds,
    and handed-back facets never return to the surrogate."""
    from paper_2603_13190_amd import surrogate as SG
    ts = tension_small()
    samples = [SG.capture(ts, 1200, facet_stride=2, step_stride=20),
               SG.capture(confined_small(), 1500, facet_stride=2, step_stride=20)]
    assert min(x["x"].shape[0] for x in samples) > 1000
    model = SG.fit(samples, seed=0, steps=1500, batch=8192, lr=2e-3)
    g = gpu(ts, precision="mixed")
    model.install(g, KT, KC, DMAX)
    o = O.Oracle(ts)
    prog = ts["meta"]["load_prog"]
    so, sg, counts = [], [], []
    for _ in range(12):
        o.step(100)
        g.step(100)
        so.append(o.reaction_sum(prog))
        sg.append(g.reaction(prog))
        counts.append(g.surrogate_count())
    so, sg = np.array(so), np.array(sg)
    F = ts["meta"]["F"]
    hist_err = np.abs(sg - so).max() / abs(so.max())
    print("handed back:", counts, "of", F, "peak err", abs(sg.max() - so.max()) / abs(so.max()),
          "history err", hist_err, "energy err", g.energy()["err"], "holdout rmse", model.holdout_rmse)
    st = g.surrogate_stats()
    print("surrogate counts:", st)
    assert all(b >= a for a, b in zip(counts, counts[1:]))
    assert counts[0] < F                         # the surrogate does carry facets
    assert st["handed_back"] == counts[-1]
    assert st["handed_back_envelope"] + st["handed_back_box"] + st["handed_back_damage"] == st["handed_back"]
    # the network carries facets into softening (damage up to damage_max)
    assert st["damaged_network_updates"] > 0
    # the surrogate form's bar: peak stress within 1 %, energy balance within
    # 1e-3; every sample of the nominal stress history within 1 % of the peak
    assert abs(sg.max() - so.max()) <= 1e-2 * abs(so.max())
    assert hist_err <= 1e-2
    assert g.energy()["err"] <= 1e-3


def test_surrogate_arguments_are_validated():
    """Invalid surrogate descriptions are rejected with a status, not run."""
    from paper_2603_13190_amd import surrogate as SG
    from paper_2603_13190_amd.ldpm import LDPM_ERR_ARG, LDPM_ERR_STATE, LdpmError
    s = tension_small()
    p0 = SG.init_params(0)
    args = (np.zeros(9), np.ones(9), np.ones(3), np.full(9, -1.0), np.full(9, 1.0))
    g = gpu(s, precision="mixed")
    for kw in (dict(y_dead=(-1.0, 0.0, 0.0)), dict(y_tau=-0.01), dict(y_dead=(np.nan, 0.0, 0.0))):
        with pytest.raises(LdpmError) as ei:
            g.set_surrogate(p0, *args, KT, KC, DMAX, **kw)
        assert ei.value.status == LDPM_ERR_ARG, kw
    bad = p0.copy()
    bad[5] = np.inf
    with pytest.raises(LdpmError) as ei:
        g.set_surrogate(bad, *args, KT, KC, DMAX)
    assert ei.value.status == LDPM_ERR_ARG
    g64 = gpu(s, precision="fp64")
    with pytest.raises(LdpmError) as ei:
        g64.set_surrogate(p0, *args, KT, KC, DMAX)
    assert ei.value.status == LDPM_ERR_STATE


def test_capture_overflow_is_an_error():
    """A capture that offers more rows than its capacity raises instead of
    returning an arrival-order-dependent subset."""
    from paper_2603_13190_amd import surrogate as SG
    with pytest.raises(ValueError):
        SG.capture(tension_small(), 50, facet_stride=1, step_stride=10, capacity=100)
