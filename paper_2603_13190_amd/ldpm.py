"""Thin Python binding of libldpm.so (the C-ABI declared in include/ldpm.h).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch provides device memory (through its caching allocator) and
the stream.  There is no fallback: if the library is missing or no GPU is
visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpm.so")

LDPM_OK, LDPM_ERR_ARG, LDPM_ERR_ALLOC, LDPM_ERR_DEVICE, LDPM_ERR_UNSTABLE, LDPM_ERR_STATE = range(6)
PREC = {"fp64": 0, "mixed": 1}
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_ALLOC", 3: "ERR_DEVICE", 4: "ERR_UNSTABLE", 5: "ERR_STATE"}

EXPORTS = ("ldpm_load_system", "ldpm_step", "ldpm_step_profiled", "ldpm_sync", "ldpm_read_state", "ldpm_energy",
           "ldpm_reaction", "ldpm_get_info", "ldpm_set_launch", "ldpm_get_launch", "ldpm_autotune",
           "ldpm_free", "ldpm_mlp_num_params", "ldpm_mlp_create", "ldpm_mlp_set_data",
           "ldpm_mlp_grad", "ldpm_mlp_train", "ldpm_mlp_forward", "ldpm_mlp_get_params",
           "ldpm_mlp_free", "ldpm_set_surrogate", "ldpm_surrogate_count", "ldpm_surrogate_stats",
           "ldpm_capture_begin",
           "ldpm_capture_end", "ldpm_crack_opening", "ldpm_volumetric_strain", "ldpm_compare_fields",
           "ldpm_compare_fields_noalloc",
           "ldpm_perturb", "ldpm_implicit_step", "ldpm_tessellate", "ldpm_element_lambda",
           "ldpm_stream_probe", "ldpm_last_error")

_MAT_FIELDS = ("E0", "alpha", "sigma_t", "l_t", "r_st", "n_t", "r_s", "k_t",
               "sigma_c0", "Hc0_over_E0", "Hc1_over_E0", "kc0", "kc1", "kc2", "kc3",
               "Ed_over_E0", "beta", "mu0", "mu_inf", "sigma_N0")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_up = C.POINTER(C.c_uint8)
_fp = C.POINTER(C.c_float)


class Material(C.Structure):
    _fields_ = [(k, C.c_double) for k in _MAT_FIELDS] + [("law", C.c_int32)]


class State(C.Structure):
    _fields_ = [("q", _dp), ("v", _dp), ("t", _dp), ("emax", _dp), ("fext", _dp),
                ("w_int", _dp), ("w_ext", _dp), ("w_kin", _dp), ("w_kin0", _dp),
                ("w_pert", _dp), ("step", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class SystemDesc(C.Structure):
    _fields_ = [("n_specimens", C.c_int32), ("particle_off", _lp), ("tet_off", _lp),
                ("n_particles", C.c_int64), ("n_tets", C.c_int64), ("n_facets", C.c_int64),
                ("x0", _dp), ("mass", _dp), ("rot_inertia", _dp), ("cell_vol", _dp), ("cell_r", _dp),
                ("tet_nodes", _ip), ("facet_I", _ip), ("facet_J", _ip),
                ("facet_cI", _dp), ("facet_n", _dp), ("facet_m", _dp),
                ("facet_area", _dp), ("facet_len", _dp),
                ("dof_mode", _up), ("dof_prog", _ip), ("dof_scale", _dp),
                ("n_programs", C.c_int32), ("prog_off", _lp), ("prog_t", _dp), ("prog_v", _dp),
                ("body_force", _dp), ("q0", _dp), ("v0", _dp), ("init_state", C.POINTER(State)),
                ("mat", C.POINTER(Material)), ("dt", C.c_double), ("precision", C.c_int32),
                ("stream", C.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", C.c_void_p), ("mass_block", _dp)]


class Energies(C.Structure):
    _fields_ = [("W_ext", C.c_double), ("W_int", C.c_double), ("W_kin", C.c_double),
                ("W_kin0", C.c_double), ("W_pert", C.c_double), ("err", C.c_double),
                ("step", C.c_int64), ("time", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_tets", C.c_int64), ("n_facets", C.c_int64),
                ("n_edges", C.c_int64), ("n_specimens", C.c_int64), ("step", C.c_int64),
                ("precision", C.c_int32), ("law", C.c_int32),
                ("facet_kernel_bytes", C.c_double), ("particle_kernel_bytes", C.c_double),
                ("device_bytes", C.c_size_t)]


class Launch(C.Structure):
    _fields_ = [("tets_per_block", C.c_int32), ("particle_threads", C.c_int32),
                ("xcd_remap", C.c_int32), ("persistent", C.c_int32), ("stream_facets", C.c_int32)]


def _launch_dict(c):
    return dict(tets_per_block=c.tets_per_block, particle_threads=c.particle_threads, xcd_remap=c.xcd_remap,
                persistent=c.persistent, stream_facets=c.stream_facets)


class TuneTrial(C.Structure):
    _fields_ = [("launch", Launch), ("us_per_step", C.c_double)]


class SurrogateDesc(C.Structure):
    _fields_ = [("params", _fp), ("x_mean", C.c_float * 9), ("x_scale", C.c_float * 9),
                ("y_scale", C.c_float * 3), ("y_dead", C.c_float * 3),
                ("y_tau", C.c_float), ("box_lo", C.c_float * 9), ("box_hi", C.c_float * 9),
                ("kappa_t", C.c_float), ("kappa_c", C.c_float), ("damage_max", C.c_float)]


class CaptureOpts(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("facet_stride", C.c_int32), ("facet_offset", C.c_int32),
                ("step_stride", C.c_int32), ("kappa_t", C.c_float), ("kappa_c", C.c_float),
                ("damage_max", C.c_float)]


class FieldStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean_x", C.c_double), ("mean_ref", C.c_double),
                ("pearson", C.c_double), ("rmse", C.c_double), ("ref_max", C.c_double),
                ("nrmse", C.c_double)]


class ImplicitOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("alpha_m", C.c_double), ("alpha_f", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("cg_tol", C.c_double), ("cg_max_iter", C.c_int32)]


class ImplicitStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("newton_iters", C.c_int64), ("cg_iters", C.c_int64),
                ("not_converged", C.c_int64), ("max_residual", C.c_double)]


class LdpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ldpm {_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libldpm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch's HIP runtime must be the one the library binds to (one
        # runtime per process; streams and allocations are shared with it):
        # load it first so libamdhip64.so.7 resolves to the copy in memory.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_13190_amd/build.py")
        L = C.CDLL(LIB_PATH)
        L.ldpm_load_system.argtypes = [C.POINTER(SystemDesc), C.POINTER(C.c_void_p)]
        L.ldpm_step.argtypes = [C.c_void_p, C.c_int64]
        L.ldpm_sync.argtypes = [C.c_void_p]
        L.ldpm_step_profiled.argtypes = [C.c_void_p, C.c_int64, _dp, _dp]
        L.ldpm_read_state.argtypes = [C.c_void_p, C.POINTER(State)]
        L.ldpm_energy.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Energies)]
        L.ldpm_reaction.argtypes = [C.c_void_p, C.c_int32, _dp]
        L.ldpm_get_info.argtypes = [C.c_void_p, C.POINTER(Info)]
        L.ldpm_set_launch.argtypes = [C.c_void_p, C.POINTER(Launch)]
        L.ldpm_get_launch.argtypes = [C.c_void_p, C.POINTER(Launch)]
        L.ldpm_autotune.argtypes = [C.c_void_p, C.c_int32, C.POINTER(Launch), _dp,
                                    C.POINTER(TuneTrial), C.c_int32, C.POINTER(C.c_int32)]
        L.ldpm_tessellate.argtypes = [C.POINTER(TessDesc), C.POINTER(TessOut), C.c_void_p]
        L.ldpm_element_lambda.argtypes = [C.POINTER(ElemDesc), _dp, C.c_void_p]
        L.ldpm_mlp_num_params.restype = C.c_int32
        L.ldpm_mlp_create.argtypes = [_fp, C.c_void_p, C.POINTER(C.c_void_p)]
        L.ldpm_mlp_set_data.argtypes = [C.c_void_p, _fp, _fp, C.c_int64]
        L.ldpm_mlp_grad.argtypes = [C.c_void_p, C.c_int32, C.c_int64, _fp, _fp]
        L.ldpm_mlp_train.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_float, _fp]
        L.ldpm_mlp_forward.argtypes = [C.c_void_p, _fp, C.c_int64, _fp]
        L.ldpm_mlp_get_params.argtypes = [C.c_void_p, _fp]
        L.ldpm_mlp_free.argtypes = [C.c_void_p]
        L.ldpm_mlp_free.restype = None
        L.ldpm_set_surrogate.argtypes = [C.c_void_p, C.POINTER(SurrogateDesc)]
        L.ldpm_surrogate_count.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.ldpm_surrogate_stats.argtypes = [C.c_void_p, C.POINTER(C.c_int64 * 7)]
        L.ldpm_capture_begin.argtypes = [C.c_void_p, C.POINTER(CaptureOpts)]
        L.ldpm_capture_end.argtypes = [C.c_void_p, _fp, C.c_int64, C.POINTER(C.c_int64)]
        L.ldpm_crack_opening.argtypes = [C.c_void_p, C.c_void_p]
        L.ldpm_volumetric_strain.argtypes = [C.c_void_p, C.c_void_p]
        L.ldpm_compare_fields.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_void_p,
                                          C.POINTER(FieldStats)]
        L.ldpm_compare_fields_noalloc.argtypes = L.ldpm_compare_fields.argtypes
        L.ldpm_perturb.argtypes = [C.c_void_p, _dp, _dp]
        L.ldpm_implicit_step.argtypes = [C.c_void_p, C.POINTER(ImplicitOpts), C.c_int64,
                                         C.POINTER(ImplicitStats)]
        L.ldpm_stream_probe.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.ldpm_free.argtypes = [C.c_void_p]
        L.ldpm_free.restype = None
        L.ldpm_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("ldpm_free", "ldpm_last_error", "ldpm_mlp_free", "ldpm_mlp_num_params"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != LDPM_OK:
        raise LdpmError(rc, lib().ldpm_last_error().decode())
    return rc


def _soa(a, dtype=np.float64):
    """(n, k) generator layout -> [k][n] contiguous."""
    a = np.asarray(a)
    if a.ndim == 1:
        return np.ascontiguousarray(a, dtype=dtype)
    return np.ascontiguousarray(a.T, dtype=dtype)


def _p(a, t):
    return a.ctypes.data_as(t)


class _TorchAllocator:
    """Device memory from torch's caching allocator on its current stream."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device, self.stream)
            except Exception:  # noqa: BLE001 - allocator failure is reported as NULL
                return None
            self.live[ptr] = nbytes
            return ptr

        def _free(ptr, ctx):
            if ptr in self.live:
                del self.live[ptr]
                # a handle collected while the interpreter shuts down finds
                # torch already torn down; the process releases the memory
                if not sys.is_finalizing():
                    torch.cuda.caching_allocator_delete(ptr)

        self.c_alloc = ALLOC_FN(_alloc)
        self.c_free = FREE_FN(_free)


def make_desc(sysd, precision="fp64"):
    """SystemDesc for a generator dict (host arrays only, no device work).
    Returns (desc, keepalive) - the arrays must outlive the load call."""
    N = int(sysd["x0"].shape[0])
    T = int(sysd["tet_nodes"].shape[0])
    F = int(sysd["facet_I"].shape[0])
    k = {}
    k["x0"] = _soa(sysd["x0"])
    k["mass"] = _soa(sysd["mass"])
    k["inertia"] = _soa(sysd["inertia"])
    k["cell_vol"] = _soa(sysd["cell_vol"])
    k["cell_r"] = _soa(sysd["cell_r"])
    k["tet"] = _soa(sysd["tet_nodes"], np.int32)
    k["fI"] = _soa(sysd["facet_I"], np.int32)
    k["fJ"] = _soa(sysd["facet_J"], np.int32)
    k["cI"] = _soa(sysd["facet_cI"])
    k["n"] = _soa(sysd["facet_n"])
    k["m"] = _soa(sysd["facet_m"])
    k["A"] = _soa(sysd["facet_area"])
    k["len"] = _soa(sysd["facet_len"])
    k["mode"] = _soa(sysd["dof_mode"], np.uint8)
    k["prog"] = _soa(sysd["dof_prog"], np.int32)
    k["scale"] = _soa(sysd["dof_scale"])
    k["poff"] = np.ascontiguousarray(sysd["prog_off"], dtype=np.int64)
    k["pt"] = np.ascontiguousarray(sysd["prog_t"], dtype=np.float64)
    k["pv"] = np.ascontiguousarray(sysd["prog_v"], dtype=np.float64)
    k["body"] = np.ascontiguousarray(sysd.get("body_force", np.zeros(3)), dtype=np.float64)
    k["q0"] = _soa(sysd["q0"])
    k["v0"] = _soa(sysd["v0"])
    nspec = 1
    if "particle_off" in sysd:
        k["po"] = np.ascontiguousarray(sysd["particle_off"], dtype=np.int64)
        k["to"] = np.ascontiguousarray(sysd["tet_off"], dtype=np.int64)
        nspec = int(k["po"].size - 1)
    mat = Material(**{f: float(sysd["material"][f]) for f in _MAT_FIELDS},
                   law=int(sysd["material"].get("law", 1)))
    k["mat"] = mat
    d = SystemDesc()
    d.n_specimens = nspec
    if "po" in k:
        d.particle_off = _p(k["po"], _lp)
        d.tet_off = _p(k["to"], _lp)
    d.n_particles, d.n_tets, d.n_facets = N, T, F
    d.x0 = _p(k["x0"], _dp)
    d.mass = _p(k["mass"], _dp)
    d.rot_inertia = _p(k["inertia"], _dp)
    d.cell_vol = _p(k["cell_vol"], _dp)
    d.cell_r = _p(k["cell_r"], _dp)
    d.tet_nodes = _p(k["tet"], _ip)
    d.facet_I = _p(k["fI"], _ip)
    d.facet_J = _p(k["fJ"], _ip)
    d.facet_cI = _p(k["cI"], _dp)
    d.facet_n = _p(k["n"], _dp)
    d.facet_m = _p(k["m"], _dp)
    d.facet_area = _p(k["A"], _dp)
    d.facet_len = _p(k["len"], _dp)
    d.dof_mode = _p(k["mode"], _up)
    d.dof_prog = _p(k["prog"], _ip)
    d.dof_scale = _p(k["scale"], _dp)
    d.n_programs = int(k["poff"].size - 1)
    d.prog_off = _p(k["poff"], _lp)
    d.prog_t = _p(k["pt"], _dp)
    d.prog_v = _p(k["pv"], _dp)
    d.body_force = _p(k["body"], _dp)
    d.q0 = _p(k["q0"], _dp)
    d.v0 = _p(k["v0"], _dp)
    d.mat = C.pointer(mat)
    d.dt = float(sysd["dt"])
    d.precision = PREC[precision]
    if sysd.get("mass_block") is not None:
        k["mblk"] = _soa(sysd["mass_block"])
        if k["mblk"].shape != (21, N):
            raise ValueError("mass_block must have shape (N, 21)")
        d.mass_block = _p(k["mblk"], _dp)
    return d, k


def try_load(desc):
    """Call ldpm_load_system; returns (status, message, handle or None)."""
    h = C.c_void_p()
    rc = lib().ldpm_load_system(C.byref(desc), C.byref(h))
    return rc, lib().ldpm_last_error().decode(), (h if rc == LDPM_OK else None)


class System:
    """One loaded LDPM system on the GPU.

    sysd: dict from paper_2603_13190_amd.specimen (particle-major arrays),
    precision: "fp64" or "mixed", init_state: dict from read_state() to
    resume, torch_alloc: take device memory from torch's caching allocator.
    """

    def __init__(self, sysd, precision="fp64", init_state: Optional[dict] = None,
                 torch_alloc=True, device=0):
        import torch  # device memory and stream provider

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the LDPM library needs a HIP device")
        torch.cuda.set_device(device)
        self.N = int(sysd["x0"].shape[0])
        self.T = int(sysd["tet_nodes"].shape[0])
        self.F = int(sysd["facet_I"].shape[0])
        self.nspec = int(len(sysd.get("particle_off", [0, self.N])) - 1)
        self.dt = float(sysd["dt"])
        self.precision = precision
        d, keep = make_desc(sysd, precision)
        if init_state is not None:
            self._init_arrays, st = self._state_struct(init_state, fill=True)
            d.init_state = C.pointer(st)
            keep["init"] = st
        self.stream = torch.cuda.current_stream(device)
        d.stream = C.c_void_p(self.stream.cuda_stream)
        self._alloc = None
        if torch_alloc:
            self._alloc = _TorchAllocator(torch, device)
            d.dev_alloc = self._alloc.c_alloc
            d.dev_free = self._alloc.c_free
        h = C.c_void_p()
        _check(lib().ldpm_load_system(C.byref(d), C.byref(h)))
        self.h = h
        self._keep = (keep, d)

    # ------------------------------------------------------------------
    def _state_struct(self, state=None, fill=False):
        N, T, F = self.N, self.T, self.F
        shapes = dict(q=(6, N), v=(6, N), t=(3, F), emax=(F,), fext=(6, N), w_int=(T,),
                      w_ext=(N,), w_kin=(N,), w_kin0=(self.nspec,), w_pert=(self.nspec,))
        arrs = {}
        st = State()
        for name, shp in shapes.items():
            if fill:
                if state is None or state.get(name) is None:
                    continue
                src = np.asarray(state[name], dtype=np.float64)
                a = np.ascontiguousarray(src.T if src.ndim == 2 else src)
                assert a.shape == shp, (name, a.shape, shp)
            else:
                a = np.zeros(shp)
            arrs[name] = a
            setattr(st, name, _p(a, _dp))
        st.step = int(state.get("step", 0)) if (fill and state is not None) else 0
        return arrs, st

    def step(self, n=1):
        _check(lib().ldpm_step(self.h, int(n)))
        return self

    def step_profiled(self, n):
        """n steps with per-kernel HIP-event timing; returns (facet_ms, particle_ms) sums."""
        a, b = C.c_double(), C.c_double()
        _check(lib().ldpm_step_profiled(self.h, int(n), C.byref(a), C.byref(b)))
        return a.value, b.value

    def sync(self):
        _check(lib().ldpm_sync(self.h))

    def read_state(self):
        """State in the generator's particle-major layout (q (N,6), t (F,3), ...)."""
        arrs, st = self._state_struct()
        _check(lib().ldpm_read_state(self.h, C.byref(st)))
        out = {k: (v.T.copy() if v.ndim == 2 else v.copy()) for k, v in arrs.items()}
        out["step"] = int(st.step)
        return out

    def energy(self, specimen=0):
        e = Energies()
        _check(lib().ldpm_energy(self.h, int(specimen), C.byref(e)))
        return dict(W_ext=e.W_ext, W_int=e.W_int, W_kin=e.W_kin, W_kin0=e.W_kin0, W_pert=e.W_pert,
                    err=e.err, step=int(e.step), time=e.time)

    def reaction(self, program):
        out = C.c_double()
        _check(lib().ldpm_reaction(self.h, int(program), C.byref(out)))
        return float(out.value)

    def info(self):
        i = Info()
        _check(lib().ldpm_get_info(self.h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in Info._fields_}

    def set_launch(self, tets_per_block=16, particle_threads=256, xcd_remap=1, persistent=0, stream_facets=None):
        """stream_facets None keeps the handle's current setting."""
        if stream_facets is None:
            stream_facets = self.get_launch()["stream_facets"]
        c = Launch(tets_per_block, particle_threads, xcd_remap, persistent, stream_facets)
        _check(lib().ldpm_set_launch(self.h, C.byref(c)))

    def get_launch(self):
        c = Launch()
        _check(lib().ldpm_get_launch(self.h, C.byref(c)))
        return _launch_dict(c)

    def autotune(self, steps_per_trial=100):
        """Time every launch shape on this system, keep the fastest.  Returns
        (best launch dict, us per step, list of (launch dict, us) trials)."""
        best = Launch()
        us = C.c_double()
        cap = 64
        arr = (TuneTrial * cap)()
        nt = C.c_int32()
        _check(lib().ldpm_autotune(self.h, int(steps_per_trial), C.byref(best), C.byref(us),
                                   arr, cap, C.byref(nt)))
        trials = [(_launch_dict(arr[i].launch), arr[i].us_per_step) for i in range(min(nt.value, cap))]
        return _launch_dict(best), us.value, trials

    def set_surrogate(self, params, x_mean, x_scale, y_scale, box_lo, box_hi,
                      kappa_t=1.1, kappa_c=0.9, damage_max=0.05, y_dead=(0.0, 0.0, 0.0), y_tau=0.0):
        """Install the MLP surrogate of the facet law (None removes it)."""
        if params is None:
            _check(lib().ldpm_set_surrogate(self.h, None))
            return
        p = np.ascontiguousarray(params, dtype=np.float32)
        d = SurrogateDesc()
        d.params = p.ctypes.data_as(_fp)
        for name, v in (("x_mean", x_mean), ("x_scale", x_scale), ("y_scale", y_scale),
                        ("y_dead", y_dead), ("box_lo", box_lo), ("box_hi", box_hi)):
            arr = getattr(d, name)
            for i, x in enumerate(np.asarray(v, dtype=np.float64)):
                arr[i] = float(x)
        d.kappa_t, d.kappa_c, d.damage_max = float(kappa_t), float(kappa_c), float(damage_max)
        d.y_tau = float(y_tau)
        _check(lib().ldpm_set_surrogate(self.h, C.byref(d)))

    def surrogate_count(self):
        n = C.c_int64()
        _check(lib().ldpm_surrogate_count(self.h, C.byref(n)))
        return int(n.value)

    def surrogate_stats(self):
        """Running counts since the surrogate was installed: facets handed
        back, facet-updates by the network, damaged facet-updates (damage in
        (1e-3, damage_max]) by either law, those of them by the network, and
        the facets handed back by the envelope, the feature box, the damage
        gate."""
        c = (C.c_int64 * 7)()
        _check(lib().ldpm_surrogate_stats(self.h, C.byref(c)))
        return dict(handed_back=c[0], network_updates=c[1], damaged_updates=c[2], damaged_network_updates=c[3],
                    handed_back_envelope=c[4], handed_back_box=c[5], handed_back_damage=c[6])

    def capture_begin(self, capacity, facet_stride=1, facet_offset=0, step_stride=1,
                      kappa_t=1.1, kappa_c=0.9, damage_max=0.05):
        o = CaptureOpts(int(capacity), int(facet_stride), int(facet_offset), int(step_stride),
                        float(kappa_t), float(kappa_c), float(damage_max))
        self._cap = int(capacity)
        _check(lib().ldpm_capture_begin(self.h, C.byref(o)))

    def capture_end(self):
        """Rows sorted by (step, facet): dict with x (n,9), y (n,3) (absolute
        residuals), s (n,) (|t_old + E de|), step, facet."""
        rows = np.zeros((self._cap, 16), dtype=np.float32)
        n = C.c_int64()
        _check(lib().ldpm_capture_end(self.h, rows.ctypes.data_as(_fp), self._cap, C.byref(n)))
        k = min(int(n.value), self._cap)
        rows = rows[:k]
        key = rows[:, 12:14].copy().view(np.int64).ravel()
        order = np.argsort(key, kind="stable")
        rows, key = rows[order], key[order]
        return dict(x=rows[:, :9].copy(), y=rows[:, 9:12].copy(), s=rows[:, 14].copy(), step=key >> 32,
                    facet=key & 0xffffffff, offered=int(n.value))

    def crack_opening(self, out=None):
        """Crack-opening vectors after the last step: device tensor (4, F)
        = w_N, w_M, w_L, |w| (enqueued on the handle's stream)."""
        import torch
        if out is None:
            out = torch.empty((4, self.F), dtype=torch.float64, device=self.stream.device)
        _check_out(out, (4, self.F))
        _check(lib().ldpm_crack_opening(self.h, C.c_void_p(out.data_ptr())))
        return out

    def volumetric_strain(self, out=None):
        """e_V per tetrahedron at the last evaluated configuration: device tensor (T,)."""
        import torch
        if out is None:
            out = torch.empty((self.T,), dtype=torch.float64, device=self.stream.device)
        _check_out(out, (self.T,))
        _check(lib().ldpm_volumetric_strain(self.h, C.c_void_p(out.data_ptr())))
        return out

    def perturb(self, delta):
        """Add delta (N, 6) (generator layout) to the free DoFs; returns the
        work of the jump."""
        d = np.asarray(delta, dtype=np.float64)
        if d.shape != (self.N, 6):
            raise ValueError("delta must have shape (N, 6)")
        d = np.ascontiguousarray(d.T)
        w = C.c_double()
        _check(lib().ldpm_perturb(self.h, _p(d, _dp), C.byref(w)))
        return float(w.value)

    def implicit_step(self, n, dt, alpha=0.0, rho_inf=None, tol=1e-8, max_iter=100, cg_tol=1e-10,
                      cg_max_iter=5000):
        """n implicit steps: HHT-alpha (alpha in [-1/3, 0]), or the
        generalised-alpha method when rho_inf is given; returns the iteration
        statistics."""
        if rho_inf is None:
            am, af = 0.0, -float(alpha)
        else:
            r = float(rho_inf)
            am, af = (2.0 * r - 1.0) / (r + 1.0), r / (r + 1.0)
        o = ImplicitOpts(float(dt), am, af, float(tol), int(max_iter), float(cg_tol), int(cg_max_iter))
        st = ImplicitStats()
        _check(lib().ldpm_implicit_step(self.h, C.byref(o), int(n), C.byref(st)))
        return {f: getattr(st, f) for f, _ in ImplicitStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().ldpm_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def _check_out(t, shape):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape):
        raise ValueError(f"output must be a contiguous float64 device tensor of shape {shape}")


def compare_fields(x, ref, cap=None, stream=None, noalloc=False):
    """Pearson's correlation and NRMSE (percent, normalised by max ref) of
    two device tensors of the same size (float64), optionally limited to cap
    first.  Returns a dict.  noalloc: ldpm_compare_fields_noalloc (its
    partials in the library's static device buffer) instead of
    ldpm_compare_fields."""
    import torch
    for t in (x, ref):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("fields must be contiguous float64 device tensors")
    if x.numel() != ref.numel():
        raise ValueError("fields must have the same size")
    st = torch.cuda.current_stream() if stream is None else stream
    o = FieldStats()
    L = lib()
    fn = L.ldpm_compare_fields_noalloc if noalloc else L.ldpm_compare_fields
    _check(fn(C.c_void_p(x.data_ptr()), C.c_void_p(ref.data_ptr()), int(x.numel()),
              float(cap) if cap is not None else 0.0, C.c_void_p(st.cuda_stream), C.byref(o)))
    return {f: getattr(o, f) for f, _ in FieldStats._fields_}


class TessDesc(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_tets", C.c_int64), ("x", _dp), ("diam", _dp),
                ("tet_nodes", _ip), ("rho", C.c_double)]


class TessOut(C.Structure):
    _fields_ = [("facet_I", _ip), ("facet_J", _ip), ("facet_cI", _dp), ("facet_n", _dp), ("facet_m", _dp),
                ("facet_area", _dp), ("facet_area0", _dp), ("facet_len", _dp), ("mass", _dp),
                ("cell_vol", _dp), ("rot_inertia", _dp), ("cell_r", _dp), ("cell_inertia", _dp),
                ("tet_node_cones", _dp)]


def tessellate(x, diam, tets, rho, cones=False, stream=None):
    """LDPM facets and cell mass properties from centres x (N, 3), diameters
    (N,), tetrahedra (T, 4) and density rho, computed on the GPU
    (ldpm_tessellate).  Returns the generator layout (the (F, 3) and (N, 3)
    arrays as transposed views): facet arrays (F,) / (F, 3) in tet-major
    order, mass (N,), inertia (N, 3) (diagonal of J),
    cell_inertia (N, 3, 3), cell_vol (N,), cell_r (N, 3); with cones=True
    also tet_node_cones (T, 4, 10)."""
    import torch  # noqa: F401  (HIP runtime and stream provider)
    x = np.asarray(x, dtype=np.float64)
    tets = np.asarray(tets)
    N, T = x.shape[0], tets.shape[0]
    if x.ndim != 2 or x.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
        raise ValueError("x must be (N, 3) and tets (T, 4)")
    if tets.size and (tets.min() < 0 or tets.max() >= N):
        raise ValueError("tetrahedron node out of range")
    F = 12 * T
    xs = _soa(x)
    dm = np.ascontiguousarray(diam, dtype=np.float64)
    if dm.shape != (N,):
        raise ValueError("diam must be (N,)")
    tn = _soa(tets, np.int32)
    d = TessDesc(N, T, _p(xs, _dp), _p(dm, _dp), _p(tn, _ip), float(rho))
    out = dict(facet_I=np.empty(F, np.int32), facet_J=np.empty(F, np.int32), facet_cI=np.empty((3, F)),
               facet_n=np.empty((3, F)), facet_m=np.empty((3, F)), facet_area=np.empty(F),
               facet_area0=np.empty(F), facet_len=np.empty(F), mass=np.empty(N), cell_vol=np.empty(N),
               rot_inertia=np.empty((3, N)), cell_r=np.empty((3, N)), cell_inertia=np.empty((6, N)))
    cone = np.empty((T, 4, 10)) if cones else None
    o = TessOut(*[_p(out[k], _ip if k in ("facet_I", "facet_J") else _dp) for k, _ in TessOut._fields_[:-1]],
                _p(cone, _dp) if cones else None)
    st = C.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib().ldpm_tessellate(C.byref(d), C.byref(o), st))
    J6 = out.pop("cell_inertia")
    Jf = np.empty((N, 3, 3))
    for p, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (1, 2), (0, 2))):
        Jf[:, i, j] = J6[p]
        Jf[:, j, i] = J6[p]
    # (F, 3) and (N, 3) arrays are transposed views of the library's [3][F]
    # and [3][N] outputs: no copy, and the loader's structure-of-arrays
    # conversion of a view is the original array again
    res = dict(facet_I=out["facet_I"], facet_J=out["facet_J"],
               facet_cI=out["facet_cI"].T, facet_n=out["facet_n"].T, facet_m=out["facet_m"].T,
               facet_area=out["facet_area"], facet_area0=out["facet_area0"], facet_len=out["facet_len"],
               mass=out["mass"], inertia=out["rot_inertia"].T, cell_inertia=Jf, cell_vol=out["cell_vol"],
               cell_r=out["cell_r"].T)
    if cones:
        res["tet_node_cones"] = cone
    return res


class ElemDesc(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("n_tets", C.c_int64), ("tet_nodes", _ip), ("facet_I", _ip),
                ("facet_J", _ip), ("facet_cI", _dp), ("facet_n", _dp), ("facet_area", _dp), ("facet_len", _dp),
                ("share", _dp), ("E0", C.c_double), ("alpha", C.c_double)]


STREAM_KINDS = {"copy": 0, "read": 1, "fill": 2, "mix": 3}


def stream_probe(kind, src, dst, nbytes, stream=None):
    """Enqueue one reference streaming kernel (ldpm_stream_probe) moving
    nbytes between the device tensors src and dst (src may be None for
    "fill"); the caller times it on `stream` (default: torch's current)."""
    import torch
    for t in (src, dst):
        if t is not None and not (t.is_cuda and t.is_contiguous()):
            raise ValueError("buffers must be contiguous device tensors")
    st = torch.cuda.current_stream() if stream is None else stream
    _check(lib().ldpm_stream_probe(STREAM_KINDS[kind], C.c_void_p(src.data_ptr() if src is not None else 0),
                                   C.c_void_p(dst.data_ptr()), int(nbytes), C.c_void_p(st.cuda_stream)))


def element_lambda_max(sysd, E0, alpha, share, stream=None):
    """Largest eigenvalue of each tetrahedron's mass-scaled elastic stiffness
    (ldpm_element_lambda) for a generator dict (facets tet-major) and the
    tetrahedra's mass shares (T, 4, 6).  Returns (T,)."""
    import torch  # noqa: F401  (HIP runtime and stream provider)
    x = np.asarray(sysd["x0"])
    tets = np.asarray(sysd["tet_nodes"])
    N, T = x.shape[0], tets.shape[0]
    k = dict(tn=_soa(tets, np.int32), fI=_soa(sysd["facet_I"], np.int32), fJ=_soa(sysd["facet_J"], np.int32),
             cI=_soa(sysd["facet_cI"]), n=_soa(sysd["facet_n"]), A=_soa(sysd["facet_area"]),
             L=_soa(sysd["facet_len"]), sh=np.ascontiguousarray(share, dtype=np.float64))
    if k["sh"].shape != (T, 4, 6):
        raise ValueError("share must be (T, 4, 6)")
    d = ElemDesc(N, T, _p(k["tn"], _ip), _p(k["fI"], _ip), _p(k["fJ"], _ip), _p(k["cI"], _dp), _p(k["n"], _dp),
                 _p(k["A"], _dp), _p(k["L"], _dp), _p(k["sh"], _dp), float(E0), float(alpha))
    lam = np.empty(T)
    st = C.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib().ldpm_element_lambda(C.byref(d), _p(lam, _dp), st))
    return lam


class Mlp:
    """GPU trainer of the facet-law surrogate (ldpm_mlp_* of the C-ABI)."""

    def __init__(self, params, stream=None):
        import torch  # noqa: F401  (HIP runtime and stream provider)
        L = lib()
        self.n_params = int(L.ldpm_mlp_num_params())
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        h = C.c_void_p()
        st = C.c_void_p(stream.cuda_stream) if stream is not None else None
        _check(L.ldpm_mlp_create(p.ctypes.data_as(_fp), st, C.byref(h)))
        self.h = h

    def set_data(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        assert x.shape[1] == 9 and y.shape[1] == 3 and x.shape[0] == y.shape[0]
        _check(lib().ldpm_mlp_set_data(self.h, x.ctypes.data_as(_fp), y.ctypes.data_as(_fp),
                                       int(x.shape[0])))
        self.n = x.shape[0]

    def grad(self, batch, offset=0):
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = C.c_float()
        _check(lib().ldpm_mlp_grad(self.h, int(batch), int(offset), g.ctypes.data_as(_fp), C.byref(loss)))
        return float(loss.value), g

    def train(self, steps, batch=4096, lr=1e-3):
        loss = C.c_float()
        _check(lib().ldpm_mlp_train(self.h, int(steps), int(batch), float(lr), C.byref(loss)))
        return float(loss.value)

    def forward(self, x):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], 3), dtype=np.float32)
        _check(lib().ldpm_mlp_forward(self.h, x.ctypes.data_as(_fp), int(x.shape[0]), y.ctypes.data_as(_fp)))
        return y

    def params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().ldpm_mlp_get_params(self.h, p.ctypes.data_as(_fp)))
        return p

    def close(self):
        if getattr(self, "h", None):
            lib().ldpm_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
