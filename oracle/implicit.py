"""Plain implicit HHT-alpha integration of the LDPM equations of motion, FP64.

TEST INFRASTRUCTURE ONLY: used by the tests and the CPU-baseline leg of the
benchmark, never by the solver package.

The paper's implicit solvers integrate M q'' + f_int(q) = f_ext with the
HHT (Hilber-Hughes-Taylor) alpha method or the generalised-alpha method and
Newton-type iterations (sections on the implementations and on the
time-integration schemes).  This module writes out the generalised-alpha
family with interpolated forces (Chung and Hulbert's parameters), of which
HHT-alpha is the member alpha_m = 0, alpha_f = -alpha:

  (1 - a_m) M a_{n+1} + a_m M a_n
      = (1 - a_f) (g(q_{n+1}) + f_{n+1}) + a_f (g(q_n) + f_n) + R_{n+1},
  q_{n+1} = q_n + dt v_n + dt^2 ((1/2 - beta) a_n + beta a_{n+1}),
  v_{n+1} = v_n + dt ((1 - gamma) a_n + gamma a_{n+1}),
  gamma = 1/2 - a_m + a_f, beta = (1 - a_m + a_f)^2 / 4;
  HHT: a_m = 0, a_f = -alpha, alpha in [-1/3, 0];
  generalised-alpha from the high-frequency spectral radius rho_inf in
  [0, 1]: a_m = (2 rho_inf - 1) / (rho_inf + 1), a_f = rho_inf / (rho_inf + 1),

with g = -f_int (the facet forces gathered as in the explicit step), f the
applied forces, and R the reactions of prescribed DoFs.  Each step is
solved by modified Newton on the free DoFs with the initial elastic
stiffness K0: K_eff = (1 - a_m) M / (beta dt^2) + (1 - a_f) K0, factorised
once (scipy sparse LU).  The facet laws are evaluated from the committed history
at every trial configuration and committed when the step is accepted.

Readings (the paper does not write these out):
- prescribed DoFs move by dt times their programmed velocity at mid-step,
  q_{n+1,P} = q_{n,P} + dt v_P(t_n + dt/2), and take a, v from the Newmark
  relations;
- the predictor keeps the acceleration, a^(0)_{n+1} = a_n;
- a step is accepted when ||R_F||_2 <= tol (||((1 - a_m) M a)_F||_2 +
  ||rhs_F||_2), rhs the other terms above, or after max_iter iterations
  (the paper's runs accept non-converged steps after a fixed number of
  iterations);
- reactions of prescribed DoFs: R = (1 - a_m) M a_{n+1} - rhs;
- a_0 solves M a_0 = g(q_0) + f(0) on the free DoFs (zero on prescribed);
- energies: W_int from the facet trapezoids of the accepted steps, W_kin =
  1/2 v^T M v, W_ext the trapezoid of (applied + reaction) forces over the
  displacement increments.
Lumped (diagonal) mass only.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from . import Oracle, _dp, _ptr, lib


def _skew(c):
    """[c]x with [c]x y = c x y, for a stack of vectors (k, 3)."""
    z = np.zeros(c.shape[0])
    return np.stack([np.stack([z, -c[:, 2], c[:, 1]], -1),
                     np.stack([c[:, 2], z, -c[:, 0]], -1),
                     np.stack([-c[:, 1], c[:, 0], z], -1)], -2)


def elastic_stiffness(sysd):
    """K0 (6N x 6N, CSR): sum over facets of (A / l) B^T D B with the jump
    [[u]] = B q = u_J - [c^J]x th_J - u_I + [c^I]x th_I (eq. strain1) and
    D = E0 (alpha 1 + (1 - alpha) n n^T), the elastic law written in the
    global frame (t = E0 diag(1, alpha, alpha) e)."""
    mat = sysd["material"]
    E0, al = float(mat["E0"]), float(mat["alpha"])
    I = np.asarray(sysd["facet_I"], dtype=np.int64)
    J = np.asarray(sysd["facet_J"], dtype=np.int64)
    n = np.asarray(sysd["facet_n"], dtype=np.float64)
    cI = np.asarray(sysd["facet_cI"], dtype=np.float64)
    L = np.asarray(sysd["facet_len"], dtype=np.float64)
    A = np.asarray(sysd["facet_area"], dtype=np.float64)
    F = I.size
    N = np.asarray(sysd["x0"]).shape[0]
    cJ = cI - L[:, None] * n
    eye = np.broadcast_to(np.eye(3), (F, 3, 3))
    B = np.concatenate([np.concatenate([-eye, _skew(cI)], 2), np.concatenate([eye, -_skew(cJ)], 2)], 2)  # (F,3,12)
    D = E0 * (al * np.eye(3)[None] + (1.0 - al) * n[:, :, None] * n[:, None, :])
    Kf = (A / L)[:, None, None] * np.einsum("fki,fkl,flj->fij", B, D, B)      # (F,12,12)
    dof = np.concatenate([6 * I[:, None] + np.arange(6), 6 * J[:, None] + np.arange(6)], 1)  # (F,12)
    rows = np.repeat(dof[:, :, None], 12, 2).ravel()
    cols = np.repeat(dof[:, None, :], 12, 1).ravel()
    K = sp.coo_matrix((Kf.ravel(), (rows, cols)), shape=(6 * N, 6 * N)).tocsr()
    return K


def gen_alpha_params(rho_inf):
    """(alpha_m, alpha_f) of the generalised-alpha method for rho_inf."""
    r = float(rho_inf)
    return (2.0 * r - 1.0) / (r + 1.0), r / (r + 1.0)


class HHT:
    """Generalised-alpha / HHT-alpha integrator on an Oracle's state (q, v
    are q_n, v_n).  alpha: HHT's alpha (alpha_f = -alpha) unless alpha_f is
    given; alpha_m = 0 is HHT."""

    def __init__(self, o: Oracle, sysd, dt, alpha=0.0, tol=1e-10, max_iter=100, alpha_m=0.0, alpha_f=None):
        if sysd.get("mass_block") is not None:
            raise ValueError("the implicit oracle takes the lumped diagonal mass only")
        am = float(alpha_m)
        af = -float(alpha) if alpha_f is None else float(alpha_f)
        if not (am <= af + 1e-15 and af <= 0.5 + 1e-15 and am >= -1.0):
            raise ValueError("need alpha_m <= alpha_f <= 1/2")
        self.o, self.dt = o, float(dt)
        self.am, self.af = am, af
        self.gamma = 0.5 - am + af
        self.beta = (1.0 - am + af) ** 2 / 4.0
        self.tol, self.max_iter = float(tol), int(max_iter)
        N = o.N
        self.M = np.concatenate([np.repeat(np.asarray(sysd["mass"])[:, None], 3, 1),
                                 np.asarray(sysd["inertia"])], 1)
        self.free = np.asarray(sysd["dof_mode"]) == 0
        self.prog = np.asarray(sysd["dof_prog"])
        self.scale = np.asarray(sysd["dof_scale"], dtype=np.float64)
        self.poff = np.asarray(sysd["prog_off"])
        self.pt = np.asarray(sysd["prog_t"], dtype=np.float64)
        self.pv = np.asarray(sysd["prog_v"], dtype=np.float64)
        b = np.asarray(sysd.get("body_force", np.zeros(3)), dtype=np.float64)
        self.body = np.zeros((N, 6))
        if np.any(b != 0):
            V = np.asarray(sysd["cell_vol"])
            r = np.asarray(sysd["cell_r"])
            self.body[:, :3] = V[:, None] * b
            self.body[:, 3:] = V[:, None] * np.cross(r, b)
        K0 = elastic_stiffness(sysd)
        fr = np.flatnonzero(self.free.ravel())
        self.fr = fr
        Keff = sp.diags((1.0 - am) * self.M.ravel()[fr] / (self.beta * self.dt ** 2)) + (1.0 - af) * K0[fr][:, fr]
        self.lu = sla.splu(Keff.tocsc())
        self.a = None
        self.g_n = None
        self.f_n = None
        self.iters = []

    # -- loads --------------------------------------------------------------
    def _prog(self, p, time):
        a, b = self.poff[p], self.poff[p + 1]
        if b <= a:
            return 0.0
        return float(np.interp(time, self.pt[a:b], self.pv[a:b]))

    def _program_values(self, time):
        vals = np.zeros(self.poff.size - 1)
        for p in range(vals.size):
            vals[p] = self._prog(p, time)
        return vals

    def applied(self, time):
        vals = self._program_values(time)
        f = self.body.copy()
        m = self.free & (self.prog >= 0)
        f[m] += self.scale[m] * vals[self.prog[m]]
        return f

    def prescribed_velocity(self, time):
        vals = self._program_values(time)
        v = np.zeros_like(self.scale)
        m = (~self.free) & (self.prog >= 0)
        v[m] = self.scale[m] * vals[self.prog[m]]
        return v

    # -- trial internal force -------------------------------------------
    def trial(self, q):
        o = self.o
        g = np.zeros((o.N, 6))
        t = np.zeros((o.F, 3))
        e = np.zeros((o.F, 3))
        em = np.zeros(o.F)
        dW = np.zeros(o.F)
        qq = np.ascontiguousarray(q, dtype=np.float64)
        lib().ora_trial_force(C.byref(o.sys), C.byref(o.st), _ptr(qq, _dp), _ptr(g, _dp), _ptr(t, _dp),
                              _ptr(e, _dp), _ptr(em, _dp), _ptr(dW, _dp))
        return g, t, e, em, dW

    # -- steps ----------------------------------------------------------
    def step(self, n=1):
        o, dt, am, af, be, ga = self.o, self.dt, self.am, self.af, self.beta, self.gamma
        M, free = self.M, self.free
        for _ in range(n):
            tn = o.step_index * dt
            if self.a is None:
                g0 = self.trial(o.q)[0]
                f0 = self.applied(tn)
                self.a = np.where(free, (g0 + f0) / M, 0.0)
                self.g_n, self.f_n = g0, f0
                if o.step_index == 0:
                    o.st.W_kin0 = 0.5 * float(np.sum(M * o.v * o.v))
                    o.st.W_kin = o.st.W_kin0
                    o.fext[...] = np.where(free, f0, 0.0)
            qn, vn, an = o.q.copy(), o.v.copy(), self.a
            f1 = self.applied(tn + dt)
            base = qn + dt * vn + dt * dt * (0.5 - be) * an
            q = qn + dt * vn + 0.5 * dt * dt * an
            q = np.where(free, q, qn + dt * self.prescribed_velocity(tn + 0.5 * dt))
            k = 0
            while True:
                a = (q - base) / (be * dt * dt)
                g, t, e, em, dW = self.trial(q)
                rhs = (1.0 - af) * (g + f1) + af * (self.g_n + self.f_n) - am * M * an
                Ma = (1.0 - am) * M * a
                Rf = (rhs - Ma)[free]
                ref = np.linalg.norm(Ma[free]) + np.linalg.norm(rhs[free])
                res = np.linalg.norm(Rf)
                if res <= self.tol * ref or k == self.max_iter:
                    break
                dq = self.lu.solve(Rf)
                qf = q.ravel().copy()
                qf[self.fr] += dq
                q = qf.reshape(q.shape)
                k += 1
            self.iters.append((k, res / ref if ref > 0 else 0.0))
            # accept: commit the trial history and advance
            v = vn + dt * ((1.0 - ga) * an + ga * a)
            react = np.where(free, 0.0, Ma - rhs)
            Ftot = np.where(free, f1, 0.0) + react
            o.st.W_ext += float(np.sum(0.5 * (o.fext + Ftot) * (q - qn)))
            o.st.W_int += float(np.sum(dW))
            o.t[...] = t
            o.e[...] = e
            o.emax[...] = em
            o.fext[...] = Ftot
            o.q[...] = q
            o.v[...] = v
            o.st.W_kin = 0.5 * float(np.sum(M * v * v))
            o.st.step = o.step_index + 1
            self.a, self.g_n, self.f_n = a, g, f1
        return self
