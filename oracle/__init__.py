"""Python access to the plain FP64 CPU oracle (ldpm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the solver package.

Parity unpinned (no external reference exists for these; they follow the
documented readings, and the GPU path is compared against them): whole
trajectories of the inelastic workloads, and the reading that the facet law
takes a random perturbation's jump as an increment of its own (its
invariants are pinned: masking, rigid jumps, elastic work, consistency of
history and positions, energy balance).  The history across branch switches
and the e_max rule are pinned by closed forms along a tension - unloading -
compression - reloading path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libldpm_oracle.so")
_lib = None

_MAT_FIELDS = ("E0", "alpha", "sigma_t", "l_t", "r_st", "n_t", "r_s", "k_t",
               "sigma_c0", "Hc0_over_E0", "Hc1_over_E0", "kc0", "kc1", "kc2", "kc3",
               "Ed_over_E0", "beta", "mu0", "mu_inf", "sigma_N0")


class OraMat(C.Structure):
    _fields_ = [(k, C.c_double) for k in _MAT_FIELDS] + [("law", C.c_int32)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint8)


class OraSys(C.Structure):
    _fields_ = [("N", C.c_int64), ("T", C.c_int64), ("F", C.c_int64),
                ("x0", _dp), ("mass", _dp), ("inertia", _dp), ("cell_vol", _dp), ("cell_r", _dp),
                ("tet", _ip), ("fI", _ip), ("fJ", _ip), ("ftet", _ip),
                ("cI", _dp), ("n", _dp), ("m", _dp), ("A", _dp), ("len", _dp),
                ("dof_mode", _up), ("dof_prog", _ip), ("dof_scale", _dp),
                ("n_prog", C.c_int64), ("prog_off", _lp), ("prog_t", _dp), ("prog_v", _dp),
                ("body", _dp), ("dt", C.c_double), ("mat", OraMat), ("mass_block", _dp)]


class OraState(C.Structure):
    _fields_ = [("q", _dp), ("v", _dp), ("t", _dp), ("e", _dp), ("emax", _dp), ("fext", _dp),
                ("W_int", C.c_double), ("W_ext", C.c_double), ("W_kin", C.c_double),
                ("W_kin0", C.c_double), ("W_pert", C.c_double), ("step", C.c_int64)]


def use_library(path):
    """Load the oracle from another build of the same source (e.g. one
    optimised for the host, oracle.build.build_native) instead of the
    in-tree library; only before the library is first used."""
    global _LIB_PATH
    if _lib is not None and os.path.abspath(path) != os.path.abspath(_LIB_PATH):
        raise RuntimeError("the oracle library is already loaded")
    _LIB_PATH = path
    return lib()


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.ora_step.argtypes = [C.POINTER(OraSys), C.POINTER(OraState), C.c_int64, C.c_int]
        L.ora_step.restype = C.c_int
        L.ora_facet_law.argtypes = [C.POINTER(OraMat), C.c_double, _dp, _dp, C.c_double, _dp,
                                    C.c_double, _dp, _dp]
        L.ora_facet_law.restype = None
        L.ora_facet_strain.argtypes = [_dp, _dp, _dp, _dp, _dp, C.c_double, _dp]
        L.ora_tet_volstrain.argtypes = [_dp, _dp]
        L.ora_tet_volstrain.restype = C.c_double
        L.ora_elastic_internal_force.argtypes = [C.POINTER(OraSys), _dp, _dp]
        L.ora_all_strains.argtypes = [C.POINTER(OraSys), _dp, _dp]
        L.ora_all_volstrains.argtypes = [C.POINTER(OraSys), _dp, _dp]
        L.ora_max_threads.restype = C.c_int
        L.ora_perturb.argtypes = [C.POINTER(OraSys), C.POINTER(OraState), _dp]
        L.ora_perturb.restype = C.c_double
        L.ora_trial_force.argtypes = [C.POINTER(OraSys), C.POINTER(OraState)] + [_dp] * 6
        L.ora_trial_force.restype = None
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t)


def make_mat(md):
    m = OraMat()
    for k in _MAT_FIELDS:
        setattr(m, k, float(md[k]))
    m.law = int(md.get("law", 1))
    return m


class Oracle:
    """Holds one system (generator dict) and its FP64 state."""

    def __init__(self, sysd, nthreads=0):
        self.keep = {}
        g = lambda k, dt_: np.ascontiguousarray(sysd[k], dtype=dt_)
        self.arr = dict(
            x0=g("x0", np.float64), mass=g("mass", np.float64), inertia=g("inertia", np.float64),
            cell_vol=g("cell_vol", np.float64), cell_r=g("cell_r", np.float64),
            tet=g("tet_nodes", np.int32), fI=g("facet_I", np.int32), fJ=g("facet_J", np.int32),
            ftet=g("facet_tet", np.int32), cI=g("facet_cI", np.float64),
            n=g("facet_n", np.float64), m=g("facet_m", np.float64),
            A=g("facet_area", np.float64), len=g("facet_len", np.float64),
            dof_mode=g("dof_mode", np.uint8), dof_prog=g("dof_prog", np.int32),
            dof_scale=g("dof_scale", np.float64), prog_off=g("prog_off", np.int64),
            prog_t=g("prog_t", np.float64), prog_v=g("prog_v", np.float64),
            body=g("body_force", np.float64),
        )
        a = self.arr
        s = OraSys()
        s.N = a["x0"].shape[0]
        s.T = a["tet"].shape[0]
        s.F = a["fI"].shape[0]
        for k in ("x0", "mass", "inertia", "cell_vol", "cell_r", "cI", "n", "m", "A", "len",
                  "dof_scale", "prog_t", "prog_v", "body"):
            setattr(s, k, _ptr(a[k], _dp))
        for k in ("tet", "fI", "fJ", "ftet", "dof_prog"):
            setattr(s, k, _ptr(a[k], _ip))
        s.dof_mode = _ptr(a["dof_mode"], _up)
        s.n_prog = a["prog_off"].size - 1
        s.prog_off = _ptr(a["prog_off"], _lp)
        s.dt = float(sysd["dt"])
        s.mat = make_mat(sysd["material"])
        if sysd.get("mass_block") is not None:
            a["mass_block"] = np.ascontiguousarray(sysd["mass_block"], dtype=np.float64)
            if a["mass_block"].shape != (s.N, 21):
                raise ValueError("mass_block must have shape (N, 21)")
            s.mass_block = _ptr(a["mass_block"], _dp)
        self.sys = s
        self.N, self.T, self.F = int(s.N), int(s.T), int(s.F)
        self.nthreads = nthreads
        self.q = np.ascontiguousarray(sysd["q0"], dtype=np.float64).copy()
        self.v = np.ascontiguousarray(sysd["v0"], dtype=np.float64).copy()
        self.t = np.zeros((self.F, 3))
        self.e = np.zeros((self.F, 3))
        self.emax = np.zeros(self.F)
        self.fext = np.zeros((self.N, 6))
        st = OraState()
        st.q = _ptr(self.q, _dp)
        st.v = _ptr(self.v, _dp)
        st.t = _ptr(self.t, _dp)
        st.e = _ptr(self.e, _dp)
        st.emax = _ptr(self.emax, _dp)
        st.fext = _ptr(self.fext, _dp)
        self.st = st

    # -- state ----------------------------------------------------------
    @property
    def step_index(self):
        return int(self.st.step)

    def set_state(self, q, v, t, e, emax, fext, step, W=(0.0, 0.0, 0.0, 0.0), W_pert=0.0):
        self.q[...] = q
        self.v[...] = v
        self.t[...] = t
        self.e[...] = e
        self.emax[...] = emax
        self.fext[...] = fext
        self.st.step = int(step)
        self.st.W_int, self.st.W_ext, self.st.W_kin, self.st.W_kin0 = map(float, W)
        self.st.W_pert = float(W_pert)

    def energies(self):
        s = self.st
        return dict(W_int=s.W_int, W_ext=s.W_ext, W_kin=s.W_kin, W_kin0=s.W_kin0, W_pert=s.W_pert,
                    step=int(s.step),
                    err=energy_error(s.W_ext, s.W_int, s.W_kin, s.W_kin0, W_pert=s.W_pert))

    def step(self, n=1):
        rc = lib().ora_step(C.byref(self.sys), C.byref(self.st), int(n), int(self.nthreads))
        if rc != 0:
            raise FloatingPointError("oracle: non-finite state")
        return self

    # -- pieces ---------------------------------------------------------
    def strains(self, q=None):
        q = self.q if q is None else np.ascontiguousarray(q, dtype=np.float64)
        e = np.zeros((self.F, 3))
        lib().ora_all_strains(C.byref(self.sys), _ptr(q, _dp), _ptr(e, _dp))
        return e

    def volstrains(self, q=None):
        q = self.q if q is None else np.ascontiguousarray(q, dtype=np.float64)
        ev = np.zeros(self.T)
        lib().ora_all_volstrains(C.byref(self.sys), _ptr(q, _dp), _ptr(ev, _dp))
        return ev

    def elastic_internal_force(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        f = np.zeros((self.N, 6))
        lib().ora_elastic_internal_force(C.byref(self.sys), _ptr(q, _dp), _ptr(f, _dp))
        return f

    def perturb(self, delta):
        """Add delta (N, 6) to the free DoFs; the facet law takes the jump as
        an increment of its own (see ora_perturb).  Returns its work."""
        d = np.ascontiguousarray(delta, dtype=np.float64)
        if d.shape != (self.N, 6):
            raise ValueError("delta must have shape (N, 6)")
        return float(lib().ora_perturb(C.byref(self.sys), C.byref(self.st), _ptr(d, _dp)))

    def last_configuration(self):
        """q^{n-1} = q^n - dt v^{n-1/2}, the configuration at which the facet
        history was last evaluated (the undeformed one before the first step)."""
        if self.step_index == 0:
            return np.zeros_like(self.q)
        return self.q - float(self.sys.dt) * self.v

    def crack_opening(self):
        """Per-facet crack-opening vector and its magnitude, (F, 4):
        w_N, w_M, w_L, |w| (see crack_opening)."""
        md = self.sys.mat
        return crack_opening(self.e, self.t, self.arr["len"], md.E0, md.alpha)

    def volumetric_strain_field(self):
        """e_V of every tetrahedron at the configuration of the last law
        evaluation (zero before the first step)."""
        if self.step_index == 0:
            return np.zeros(self.T)
        return self.volstrains(self.last_configuration())

    def reaction_sum(self, prog_id):
        sel = self.arr["dof_prog"] == prog_id
        return float(self.fext[sel].sum())


def energy_error(W_ext, W_int, W_kin, W_kin0, tiny=1e-300, W_pert=0.0):
    """|W_ext + W_pert + W_kin0 - W_int - W_kin| / max(|W_ext + W_pert + W_kin0|, tiny);
    with W_kin0 = W_pert = 0 this is the paper's energy-balance measure
    divided by 100.  W_pert is the work of random perturbations, done on the
    specimen from outside like W_ext."""
    src = W_ext + W_pert + W_kin0
    den = max(abs(src), tiny)
    return abs(src - W_int - W_kin) / den


def crack_opening(e, t, length, E0, alpha):
    """Crack opening of each facet (numerical-examples section, comparison
    of crack patterns): the inelastic part of the facet strain times the
    facet length, w_a = l (e_a - t_a / E_a) with E = E0 diag(1, alpha, alpha),
    where only a positive (opening) inelastic normal strain counts,
    w_N = max(w_N, 0); total opening |w| = sqrt(w_N^2 + w_M^2 + w_L^2).
    e, t: (F, 3) strain and traction of the same law evaluation; returns
    (F, 4) = w_N, w_M, w_L, |w|."""
    e = np.asarray(e, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    L = np.asarray(length, dtype=np.float64)
    Ed = np.array([E0, alpha * E0, alpha * E0])
    w = L[:, None] * (e - t / Ed)
    w[:, 0] = np.maximum(w[:, 0], 0.0)
    out = np.empty((w.shape[0], 4))
    out[:, :3] = w
    out[:, 3] = np.sqrt(w[:, 0] ** 2 + w[:, 1] ** 2 + w[:, 2] ** 2)
    return out


def field_stats(x, ref, cap=None):
    """Pairwise comparison of two per-facet (or per-tetrahedron) fields as
    the paper compares crack patterns (numerical-examples section): Pearson's
    correlation coefficient and NRMSE = 100 / w~ * sqrt(mean (x - ref)^2),
    with w~ the maximum of the reference field.  cap (optional): both fields
    are limited to it first (the paper limits crack openings to 4 mm in the
    unconfined compression comparisons).  Definitions written out in FP64,
    two passes (means, then centred sums)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    if x.shape != r.shape or x.size == 0:
        raise ValueError("fields must have the same, non-zero size")
    if cap is not None and cap > 0 and np.isfinite(cap):
        x = np.minimum(x, cap)
        r = np.minimum(r, cap)
    n = x.size
    mx = x.sum() / n
    mr = r.sum() / n
    dx = x - mx
    dr = r - mr
    with np.errstate(divide="ignore", invalid="ignore"):
        pearson = float((dx * dr).sum() / np.sqrt((dx * dx).sum() * (dr * dr).sum()))
        rmse = float(np.sqrt(((x - r) ** 2).sum() / n))
        ref_max = float(r.max())
        nrmse = float(np.float64(100.0) * rmse / np.float64(ref_max))
    return dict(n=n, mean_x=float(mx), mean_ref=float(mr), pearson=pearson, rmse=rmse,
                ref_max=ref_max, nrmse=nrmse)


def facet_law(mat, length, e, e_old, eV, t_old, emax_old):
    """Single-facet constitutive update (strain driver)."""
    m = mat if isinstance(mat, OraMat) else make_mat(mat)
    e = np.ascontiguousarray(e, dtype=np.float64)
    eo = np.ascontiguousarray(e_old, dtype=np.float64)
    to = np.ascontiguousarray(t_old, dtype=np.float64)
    t = np.zeros(3)
    em = np.zeros(1)
    lib().ora_facet_law(C.byref(m), float(length), _ptr(e, _dp), _ptr(eo, _dp), float(eV),
                        _ptr(to, _dp), float(emax_old), _ptr(t, _dp), _ptr(em, _dp))
    return t, float(em[0])


def drive_facet(mat, length, path, eV_path=None):
    """Run the law along a strain path (K,3); returns tractions (K,3), e_max (K,)."""
    m = make_mat(mat)
    K = path.shape[0]
    t = np.zeros(3)
    e_old = np.zeros(3)
    em = 0.0
    T = np.zeros((K, 3))
    EM = np.zeros(K)
    for i in range(K):
        ev = 0.0 if eV_path is None else float(eV_path[i])
        t, em = facet_law(m, length, path[i], e_old, ev, t, em)
        e_old = np.array(path[i], dtype=float)
        T[i] = t
        EM[i] = em
    return T, EM


def facet_strain(qI, qJ, cI, n, m, length):
    e = np.zeros(3)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (qI, qJ, cI, n, m)]
    lib().ora_facet_strain(*[_ptr(x, _dp) for x in a], float(length), _ptr(e, _dp))
    return e


def tet_volstrain(x4, u4):
    x = np.ascontiguousarray(x4, dtype=np.float64)
    u = np.ascontiguousarray(u4, dtype=np.float64)
    return float(lib().ora_tet_volstrain(_ptr(x, _dp), _ptr(u, _dp)))


def max_threads():
    return int(lib().ora_max_threads())
