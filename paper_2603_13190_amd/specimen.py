"""Seeded synthetic LDPM specimens: the input generator.

This module produces what an LDPM preprocessor hands to a solver (paper,
Sec. "LDPM Mesh Generation": facet nodes, normals/tangents, projections,
areas) for synthetic concrete specimens, plus the loading programs and the
explicit stable time step.  It holds none of the time-stepping arithmetic
(strains, constitutive law, assembly, integration): those live in the solver
library and, independently, in the oracle.

Recipe (all seeded with ``numpy.random.default_rng(seed)``):

* particle diameters: inverse-CDF draws from the number distribution implied
  by a Fuller sieve curve (volume passing fraction (d/d_a)^n_F, n_F = 0.4,
  Sec. "Numerical examples") truncated to [d0, d_a]; the drawn aggregate
  volume is the specimen volume times the aggregate fraction of a mix with
  c = 375 kg/m3, w/c = 0.5 (same section), restricted to d >= d0;
* placement: random sequential addition, largest first, with a minimum gap
  of ``gap`` times the sum of radii;
* surface nodes of diameter d0 on corners, edges and faces (jittered grid);
* Delaunay tetrahedralisation of all centres (scipy / Qhull), degenerate
  tetrahedra removed, positive orientation, Morton ordering;
* tessellation into 12 triangular facets per tetrahedron (2 per edge): edge
  point at mid-gap between particle surfaces, face point at the centroid of
  the face's three edge points, tetrahedron point at the centroid of the four
  face points; facet = (edge point, face point, tetrahedron point);
* facet frame (n along I->J with I < J, m from the axis of smallest |n_i|,
  l = n x m), projected area A = A0 n.n0, centroid offset c^I;
* lumped mass and diagonal rotational inertia of each polyhedral cell about
  its particle centre, summed exactly over the cones (particle centre,
  facet triangle);
* stable time step from per-tetrahedron eigenvalue analysis (Sec.
  "Free vibrations": about 90 % of the critical step estimated at the level
  of the individual tetrahedron); the element bound is an upper bound of the
  assembled system's largest eigenvalue.

Units: mm, N, MPa, s, tonne (density 2.4e-9 t/mm^3).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import hashlib
import math
import os
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.spatial import Delaunay

# local edges of a tetrahedron and, for facet j = 2*e + s, the third node of
# the tetrahedron face that holds the facet
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def _facet_table():
    rows = []
    for a, b in EDGES:
        others = [c for c in range(4) if c not in (a, b)]
        for c in others:
            rows.append((a, b, c))
    return np.array(rows, dtype=np.int64)        # (12, 3): a, b, c


FACET_LOCAL = _facet_table()

# Material "M_B": paper's table of parameters with the elastic, tensile and
# compressive overrides of the synthetic workloads.
MATERIAL_MB = dict(
    E0=43700.0, alpha=0.29, sigma_t=4.0, l_t=120.0, r_st=2.6, n_t=0.4,
    r_s=0.0, k_t=0.0, sigma_c0=150.0, Hc0_over_E0=0.26, Hc1_over_E0=0.1,
    kc0=4.0, kc1=1.0, kc2=5.0, kc3=0.1, Ed_over_E0=1.0, beta=0.0,
    mu0=0.4, mu_inf=0.0, sigma_N0=600.0, law=1,
)
# Paper's table as printed (used by closed-form checks).
MATERIAL_PAPER = dict(
    E0=60273.0, alpha=0.25, sigma_t=3.44, l_t=500.0, r_st=2.6, n_t=0.4,
    r_s=0.0, k_t=0.0, sigma_c0=150.0, Hc0_over_E0=0.40, Hc1_over_E0=0.1,
    kc0=4.0, kc1=1.0, kc2=5.0, kc3=0.1, Ed_over_E0=1.0, beta=0.0,
    mu0=0.4, mu_inf=0.0, sigma_N0=600.0, law=1,
)
MATERIAL_KEYS = tuple(MATERIAL_MB.keys())
RHO = 2.4e-9            # t/mm^3 (2400 kg/m^3)


# --------------------------------------------------------------------------
# particle size distribution and placement
# --------------------------------------------------------------------------
def aggregate_fraction(c=375.0, wc=0.5, rho_c=3150.0, rho_w=1000.0, air=0.035):
    """Volume fraction of aggregate in a mix with cement content c [kg/m3]."""
    return 1.0 - c / rho_c - wc * c / rho_w - air


def fuller_diameters(rng, vol_target, d0, da, nF=0.4):
    """Draw diameters in [d0, da] until their volume reaches vol_target.

    Volume density of sizes ~ d^(nF-1) (Fuller curve), so the number density
    is ~ d^(nF-4); its CDF is inverted in closed form.
    """
    p = nF - 3.0
    a0, a1 = d0 ** p, da ** p
    out = []
    vol = 0.0
    while vol < vol_target:
        u = rng.random(4096)
        d = (a0 - u * (a0 - a1)) ** (1.0 / p)
        cv = np.cumsum(np.pi / 6.0 * d ** 3)
        k = np.searchsorted(cv, vol_target - vol)
        if k < d.size:
            out.append(d[: k + 1])
            vol += cv[k]
            break
        out.append(d)
        vol += cv[-1]
    return np.concatenate(out)


class _Grid:
    """Uniform hash grid for minimum-distance checks during placement."""

    def __init__(self, cell):
        self.cell = cell
        self.cells: Dict[Tuple[int, int, int], List[int]] = {}
        self.x: List[np.ndarray] = []
        self.r: List[float] = []

    def key(self, x):
        return (int(math.floor(x[0] / self.cell)), int(math.floor(x[1] / self.cell)),
                int(math.floor(x[2] / self.cell)))

    def ok(self, x, r, gap):
        kx, ky, kz = self.key(x)
        for i in (kx - 1, kx, kx + 1):
            for j in (ky - 1, ky, ky + 1):
                for k in (kz - 1, kz, kz + 1):
                    lst = self.cells.get((i, j, k))
                    if not lst:
                        continue
                    for p in lst:
                        y = self.x[p]
                        dd = (x[0] - y[0]) ** 2 + (x[1] - y[1]) ** 2 + (x[2] - y[2]) ** 2
                        lim = (r + self.r[p]) * (1.0 + gap)
                        if dd < lim * lim:
                            return False
        return True

    def add(self, x, r):
        self.x.append(x)
        self.r.append(r)
        self.cells.setdefault(self.key(x), []).append(len(self.x) - 1)


@dataclasses.dataclass
class Shape:
    kind: str                  # "box" or "cylinder"
    size: Tuple[float, ...]    # box: (Lx, Ly, Lz); cylinder: (D, H)

    def volume(self):
        if self.kind == "box":
            return float(np.prod(self.size))
        D, H = self.size
        return math.pi * D * D / 4.0 * H

    def sample_inside(self, rng, margin, n):
        """n uniform points whose distance to the surface is >= margin."""
        if self.kind == "box":
            lo = np.full(3, margin)
            hi = np.asarray(self.size) - margin
            if np.any(hi <= lo):
                return np.empty((0, 3))
            return lo + rng.random((n, 3)) * (hi - lo)
        D, H = self.size
        R = D / 2.0 - margin
        if R <= 0 or H - 2 * margin <= 0:
            return np.empty((0, 3))
        rr = R * np.sqrt(rng.random(n))
        ph = 2 * np.pi * rng.random(n)
        z = margin + rng.random(n) * (H - 2 * margin)
        return np.stack([D / 2 + rr * np.cos(ph), D / 2 + rr * np.sin(ph), z], axis=1)


def surface_nodes(shape: Shape, d0, rng, spacing=1.4, jitter=0.1):
    """Nodes of diameter d0 on the specimen surface (corners, edges, faces)."""
    s = spacing * d0
    pts = []
    if shape.kind == "box":
        L = np.asarray(shape.size, dtype=float)
        n = np.maximum(np.round(L / s).astype(int), 1)
        # corners
        for cx in (0.0, L[0]):
            for cy in (0.0, L[1]):
                for cz in (0.0, L[2]):
                    pts.append((cx, cy, cz))
        # edges
        for ax in range(3):
            o1, o2 = [a for a in range(3) if a != ax]
            t = np.arange(1, n[ax]) / n[ax] * L[ax]
            for v1 in (0.0, L[o1]):
                for v2 in (0.0, L[o2]):
                    tt = t + rng.uniform(-jitter, jitter, t.size) * s
                    p = np.zeros((t.size, 3))
                    p[:, ax] = tt
                    p[:, o1] = v1
                    p[:, o2] = v2
                    pts.extend(map(tuple, p))
        # faces
        for ax in range(3):
            o1, o2 = [a for a in range(3) if a != ax]
            g1 = np.arange(1, n[o1]) / n[o1] * L[o1]
            g2 = np.arange(1, n[o2]) / n[o2] * L[o2]
            G1, G2 = np.meshgrid(g1, g2, indexing="ij")
            G1 = G1.ravel()
            G2 = G2.ravel()
            for v in (0.0, L[ax]):
                p = np.zeros((G1.size, 3))
                p[:, ax] = v
                p[:, o1] = G1 + rng.uniform(-jitter, jitter, G1.size) * s
                p[:, o2] = G2 + rng.uniform(-jitter, jitter, G2.size) * s
                pts.extend(map(tuple, p))
        return np.array(pts, dtype=float)
    # cylinder: axis z, centre (D/2, D/2)
    D, H = shape.size
    R = D / 2.0
    c = np.array([R, R])
    nphi = max(int(round(2 * np.pi * R / s)), 8)
    nz = max(int(round(H / s)), 1)
    phi0 = np.arange(nphi) / nphi * 2 * np.pi
    # rims
    for z in (0.0, H):
        ph = phi0 + rng.uniform(-jitter, jitter, nphi) * s / R
        pts.extend(zip(c[0] + R * np.cos(ph), c[1] + R * np.sin(ph), np.full(nphi, z)))
    # lateral surface
    for iz in range(1, nz):
        z = iz / nz * H
        ph = phi0 + (0.5 * (iz % 2)) * 2 * np.pi / nphi + rng.uniform(-jitter, jitter, nphi) * s / R
        zz = z + rng.uniform(-jitter, jitter, nphi) * s
        pts.extend(zip(c[0] + R * np.cos(ph), c[1] + R * np.sin(ph), zz))
    # end discs: concentric rings
    nr = max(int(round(R / s)), 1)
    for z in (0.0, H):
        pts.append((c[0], c[1], z))
        for ir in range(1, nr):
            rr = ir / nr * R
            nring = max(int(round(2 * np.pi * rr / s)), 3)
            ph = np.arange(nring) / nring * 2 * np.pi + rng.uniform(0, 2 * np.pi)
            ph = ph + rng.uniform(-jitter, jitter, nring) * s / rr
            r2 = rr + rng.uniform(-jitter, jitter, nring) * s
            pts.extend(zip(c[0] + r2 * np.cos(ph), c[1] + r2 * np.sin(ph), np.full(nring, z)))
    return np.array(pts, dtype=float)


def place_particles(shape: Shape, d0, da, rng, gap=0.1, nF=0.4, max_tries=200,
                    vol_fraction=None, native=None):
    """Random sequential addition of Fuller-distributed particles.

    Returns (centres (n,3), diameters (n,)) of interior particles, placed so
    that they keep the minimum gap from each other and from the surface
    nodes (distance to the surface >= r + d0/2 (1 + gap)).  Every particle
    draws its max_tries candidates at once, so the random stream does not
    depend on which are accepted.  native (None: when available): the
    acceptance loop in C (gen/placement.c), which accepts exactly the same
    candidates as the Python loop."""
    if vol_fraction is None:
        vol_fraction = aggregate_fraction() * (1.0 - (d0 / da) ** nF)
    d = fuller_diameters(rng, vol_fraction * shape.volume(), d0, da, nF)
    d = np.sort(d)[::-1]
    cell = da * (1.0 + gap)
    L = None
    if native is not False:
        from . import gen
        L = gen.lib()
        if L is None and native:
            raise RuntimeError("the native placement library could not be built")
    xs, ds = [], []
    if L is not None:
        ext = shape.size if shape.kind == "box" else (shape.size[0], shape.size[0], shape.size[1])
        h = L.place_create(cell, float(ext[0]), float(ext[1]), float(ext[2]), int(d.size))
        if not h:
            raise MemoryError("placement grid")
        try:
            for di in d:
                r = 0.5 * di
                margin = r + 0.5 * d0 * (1.0 + gap) + gap * d0
                cand = np.ascontiguousarray(shape.sample_inside(rng, margin, max_tries), dtype=np.float64)
                if cand.shape[0] == 0:
                    continue
                k = L.place_try(h, cand.ctypes.data_as(C.POINTER(C.c_double)), cand.shape[0], r, gap)
                if k == -2:
                    raise RuntimeError("placement grid overflow")
                if k >= 0:
                    xs.append(cand[k])
                    ds.append(di)
        finally:
            L.place_free(h)
        return np.array(xs, dtype=float).reshape(-1, 3), np.array(ds, dtype=float)
    grid = _Grid(cell)
    for di in d:
        r = 0.5 * di
        margin = r + 0.5 * d0 * (1.0 + gap) + gap * d0
        cand = shape.sample_inside(rng, margin, max_tries)
        for x in cand:
            if grid.ok(x, r, gap):
                grid.add(x, r)
                xs.append(x)
                ds.append(di)
                break
    return np.array(xs, dtype=float).reshape(-1, 3), np.array(ds, dtype=float)


# --------------------------------------------------------------------------
# mesh and tessellation
# --------------------------------------------------------------------------
def _morton_keys(x, bits=10):
    lo = x.min(axis=0)
    span = np.maximum(x.max(axis=0) - lo, 1e-30)
    q = np.clip(((x - lo) / span * ((1 << bits) - 1)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(x.shape[0], dtype=np.int64)
    for b in range(bits):
        for ax in range(3):
            key |= ((q[:, ax] >> b) & 1) << (3 * b + ax)
    return key


def delaunay_tets(x, rel_vol_tol=1e-6):
    """Delaunay tetrahedra of the centres, positive orientation, slivers with
    volume below rel_vol_tol * mean volume removed."""
    tri = Delaunay(x)
    tets = tri.simplices.astype(np.int64)
    p = x[tets]
    v6 = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
    neg = v6 < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    v6 = np.abs(v6)
    keep = v6 > rel_vol_tol * v6.mean()
    return tets[keep]


def tet_quality(x, tets):
    """6 sqrt(2) V / L_max^3: 1 for a regular tetrahedron, -> 0 for slivers."""
    p = x[tets]
    V = np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])) / 6
    L = np.zeros(tets.shape[0])
    for a, b in EDGES:
        L = np.maximum(L, np.linalg.norm(p[:, a] - p[:, b], axis=1))
    return 6.0 * np.sqrt(2.0) * V / L ** 3


def _triple_key(tri, n):
    """One int64 per row of sorted node triples (values < n <= 2^21)."""
    t = tri.astype(np.int64)
    return (t[:, 0] * n + t[:, 1]) * n + t[:, 2]


def peel_boundary_slivers(x, tets, is_surf, qmin=0.05, max_iter=50):
    """Remove, layer by layer, boundary tetrahedra whose four nodes all lie on
    the specimen surface and whose quality is below qmin: the Delaunay
    tetrahedralisation of points on a curved surface leaves thin slivers
    spanning the hull.  Each layer removes, at once, every such tetrahedron
    with a face that no other remaining tetrahedron shares.  Only the fixed
    set of surface-only low-quality tetrahedra can ever go, so the face
    multiplicities are counted once and decremented as tetrahedra are
    removed."""
    T = tets.shape[0]
    if T == 0:
        return tets
    faces = np.concatenate([np.sort(tets[:, [b for b in range(4) if b != miss]], axis=1)
                            for miss in range(4)])
    _, inv, cnt = np.unique(_triple_key(faces, x.shape[0]), return_inverse=True, return_counts=True)
    face_of = inv.ravel().reshape(4, T)          # unique face id of face `miss` of tet t
    alive = np.ones(T, bool)
    cand = np.flatnonzero(is_surf[tets].all(axis=1) & (tet_quality(x, tets) < qmin))
    for _ in range(max_iter):
        if not alive.any() or cand.size == 0:
            break
        on_bnd = (cnt[face_of[:, cand]] == 1).any(axis=0)
        bad = cand[on_bnd]
        if bad.size == 0:
            break
        alive[bad] = False
        np.subtract.at(cnt, face_of[:, bad].ravel(), 1)
        cand = cand[~on_bnd]
    return tets[alive]


def frame_from_normal(n):
    """Tangent m: normalised n x a, a the axis of smallest |n_i| (lowest index
    on ties); second tangent l = n x m."""
    ax = np.argmin(np.abs(n), axis=1)
    a = np.zeros_like(n)
    a[np.arange(n.shape[0]), ax] = 1.0
    m = np.cross(n, a)
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    return m


def tessellate(x, diam, tets):
    """12 facets per tetrahedron (tet-major order, facet 12*t + j)."""
    T = tets.shape[0]
    r = 0.5 * diam
    # edge points, (T, 6, 3)
    E = np.empty((T, 6, 3))
    for e, (a, b) in enumerate(EDGES):
        xa = x[tets[:, a]]
        xb = x[tets[:, b]]
        dv = xb - xa
        ln = np.linalg.norm(dv, axis=1)
        ra = r[tets[:, a]]
        rb = r[tets[:, b]]
        s = (ln + ra - rb) / 2.0                      # mid-gap distance from a
        s = np.clip(s, 0.05 * ln, 0.95 * ln)
        E[:, e] = xa + dv * (s / ln)[:, None]
    eidx = {}
    for e, (a, b) in enumerate(EDGES):
        eidx[(a, b)] = e
        eidx[(b, a)] = e
    # face points keyed by the missing node
    Fp = np.empty((T, 4, 3))
    for miss in range(4):
        nodes = [c for c in range(4) if c != miss]
        es = [eidx[(nodes[0], nodes[1])], eidx[(nodes[0], nodes[2])], eidx[(nodes[1], nodes[2])]]
        Fp[:, miss] = (E[:, es[0]] + E[:, es[1]] + E[:, es[2]]) / 3.0
    Tp = Fp.mean(axis=1)
    # facets
    a_loc = FACET_LOCAL[:, 0]
    b_loc = FACET_LOCAL[:, 1]
    c_loc = FACET_LOCAL[:, 2]
    miss = np.array([[k for k in range(4) if k not in row] for row in FACET_LOCAL])[:, 0]
    e_of = np.array([eidx[(a, b)] for a, b in zip(a_loc, b_loc)])
    P0 = E[:, e_of]                    # (T,12,3)
    P1 = Fp[:, miss]                   # face (a,b,c) misses node d
    P2 = np.broadcast_to(Tp[:, None, :], P0.shape)
    ga = tets[:, a_loc]
    gb = tets[:, b_loc]
    I = np.minimum(ga, gb)
    J = np.maximum(ga, gb)
    xI = x[I]
    xJ = x[J]
    dv = xJ - xI
    ln = np.linalg.norm(dv, axis=2)
    n = dv / ln[..., None]
    cr = 0.5 * np.cross(P1 - P0, P2 - P0)          # vector area of the triangle
    sgn = np.sign(np.einsum("tkj,tkj->tk", cr, n))
    sgn[sgn == 0] = 1.0
    avec = cr * sgn[..., None]                     # oriented along n
    A = np.einsum("tkj,tkj->tk", avec, n)          # projected area A0 n0.n
    A0 = np.linalg.norm(avec, axis=2)
    xk = (P0 + P1 + P2) / 3.0
    cI = xk - xI
    F = 12 * T
    n_f = n.reshape(F, 3)
    m_f = frame_from_normal(n_f)
    out = dict(
        facet_I=I.reshape(F).astype(np.int32), facet_J=J.reshape(F).astype(np.int32),
        facet_tet=np.repeat(np.arange(T, dtype=np.int32), 12),
        facet_cI=cI.reshape(F, 3), facet_n=n_f, facet_m=m_f,
        facet_area=A.reshape(F), facet_len=ln.reshape(F), facet_area0=A0.reshape(F),
    )
    tri = dict(P0=P0, P1=P1, P2=P2, avec=avec, xk=xk, I=I, J=J)
    return out, tri


def cell_mass_properties(x, tets, tri, rho):
    """Mass, diagonal rotational inertia about the centre, cell volume,
    centroid offset and full inertia tensor (about the centre) of every
    polyhedral cell (exact cone sums)."""
    N = x.shape[0]
    P0, P1, P2, avec, I, J = tri["P0"], tri["P1"], tri["P2"], tri["avec"], tri["I"], tri["J"]
    vol = np.zeros(N)
    mom1 = np.zeros((N, 3))
    mom2 = np.zeros((N, 3, 3))
    cr = np.cross(P1 - P0, P2 - P0)
    orient = np.sign(np.einsum("tkj,tkj->tk", cr, avec))       # +1 if (P0,P1,P2) is ccw about avec
    for side, node in ((+1.0, I), (-1.0, J)):
        xo = x[node]
        p1 = P0 - xo
        p2 = P1 - xo
        p3 = P2 - xo
        det = np.einsum("tkj,tkj->tk", np.cross(p1, p2), p3)
        # signed cone volume: positive when the facet lies beyond the centre
        # along the cell's outward normal (toward J for the I cell)
        V = side * orient * det / 6.0
        s = p1 + p2 + p3
        S = (np.einsum("tki,tkj->tkij", p1, p1) + np.einsum("tki,tkj->tkij", p2, p2)
             + np.einsum("tki,tkj->tkij", p3, p3) + np.einsum("tki,tkj->tkij", s, s))
        S *= (V / 20.0)[..., None, None]
        nf = node.reshape(-1)
        np.add.at(vol, nf, V.reshape(-1))
        np.add.at(mom1, nf, (V[..., None] * s / 4.0).reshape(-1, 3))
        np.add.at(mom2, nf, S.reshape(-1, 3, 3))
    mass = rho * vol
    tr = np.trace(mom2, axis1=1, axis2=2)
    inertia = rho * (tr[:, None] - np.einsum("nii->ni", mom2))
    r_off = mom1 / np.maximum(vol, 1e-300)[:, None]
    J = rho * (tr[:, None, None] * np.eye(3)[None] - mom2)
    return mass, inertia, vol, r_off, J


def element_mass_share(x, tets, tri, rho):
    """Per-tetrahedron share of the lumped mass/inertia of its 4 nodes (T,4,6)."""
    T = tets.shape[0]
    P0, P1, P2, avec, I, J = tri["P0"], tri["P1"], tri["P2"], tri["avec"], tri["I"], tri["J"]
    cr = np.cross(P1 - P0, P2 - P0)
    orient = np.sign(np.einsum("tkj,tkj->tk", cr, avec))
    out = np.zeros((T, 4, 6))
    ga = tets[:, FACET_LOCAL[:, 0]]
    for side, node in ((+1.0, I), (-1.0, J)):
        xo = x[node]
        p1, p2, p3 = P0 - xo, P1 - xo, P2 - xo
        det = np.einsum("tkj,tkj->tk", np.cross(p1, p2), p3)
        V = side * orient * det / 6.0
        s = p1 + p2 + p3
        S = (np.einsum("tki,tkj->tkij", p1, p1) + np.einsum("tki,tkj->tkij", p2, p2)
             + np.einsum("tki,tkj->tkij", p3, p3) + np.einsum("tki,tkj->tkij", s, s))
        S *= (V / 20.0)[..., None, None]
        tr = np.trace(S, axis1=2, axis2=3)
        Idiag = rho * (tr[..., None] - np.einsum("tkii->tki", S))
        # local index of `node` within its tetrahedron
        loc = np.where(node == ga, FACET_LOCAL[None, :, 0], FACET_LOCAL[None, :, 1])
        for j in range(12):
            li = loc[:, j]
            out[np.arange(T), li, 0:3] += (rho * V[:, j])[:, None]
            out[np.arange(T), li, 3:6] += Idiag[:, j]
    return out


def _skew(c):
    z = np.zeros(c.shape[:-1])
    return np.stack([np.stack([z, -c[..., 2], c[..., 1]], -1),
                     np.stack([c[..., 2], z, -c[..., 0]], -1),
                     np.stack([-c[..., 1], c[..., 0], z], -1)], -2)


class _TetStiffness:
    """Elastic stiffness of tetrahedra s0..s1 (t, 24, 24), DoFs ordered
    (local node, u_x, u_y, u_z, th_x, th_y, th_z).

    Facet k couples the 6-DoF blocks of its nodes I and J through
    B = [-1, S(c^I) | 1, -S(c^J)] (jump = B q) and D = E0 (alpha 1 + (1 - alpha) n n^T):
    K_tet = sum_k (A_k / l_k) B^T D B."""

    def __init__(self, sysd, E0, alpha):
        tets = sysd["tet_nodes"].astype(np.int64)
        T = tets.shape[0]
        self.T = T
        fI = sysd["facet_I"].reshape(T, 12)
        ga = tets[:, FACET_LOCAL[:, 0]]
        self.locI = np.where(fI == ga, FACET_LOCAL[None, :, 0], FACET_LOCAL[None, :, 1])
        self.locJ = np.where(fI == ga, FACET_LOCAL[None, :, 1], FACET_LOCAL[None, :, 0])
        self.cI = sysd["facet_cI"].reshape(T, 12, 3)
        self.n = sysd["facet_n"].reshape(T, 12, 3)
        self.ln = sysd["facet_len"].reshape(T, 12)
        self.A = sysd["facet_area"].reshape(T, 12)
        self.E0, self.alpha = E0, alpha

    def __call__(self, s0, s1):
        E0, alpha = self.E0, self.alpha
        cI, n, ln, A, locI, locJ = self.cI, self.n, self.ln, self.A, self.locI, self.locJ
        eye3 = np.eye(3)
        t = s1 - s0
        rows = np.arange(t)
        K = np.zeros((t, 4, 6, 4, 6))
        for j in range(12):
            nn = n[s0:s1, j]
            cj = cI[s0:s1, j] - ln[s0:s1, j, None] * nn
            GI = np.concatenate([np.broadcast_to(-eye3, (t, 3, 3)), _skew(cI[s0:s1, j])], axis=2)
            GJ = np.concatenate([np.broadcast_to(eye3, (t, 3, 3)), -_skew(cj)], axis=2)
            D = E0 * (alpha * eye3[None] + (1 - alpha) * nn[:, :, None] * nn[:, None, :])
            D *= (A[s0:s1, j] / ln[s0:s1, j])[:, None, None]
            DI, DJ = D @ GI, D @ GJ
            GIt, GJt = GI.transpose(0, 2, 1), GJ.transpose(0, 2, 1)
            li, lj = locI[s0:s1, j], locJ[s0:s1, j]
            K[rows, li, :, li, :] += GIt @ DI
            K[rows, li, :, lj, :] += GIt @ DJ
            K[rows, lj, :, li, :] += GJt @ DI
            K[rows, lj, :, lj, :] += GJt @ DJ
        return K.reshape(t, 24, 24)


def element_lambda_max(sysd, E0, alpha, chunk=8192, workers=None):
    """Largest eigenvalue of each tetrahedron's elastic operator with its
    share of the lumped mass; the max over tetrahedra bounds the assembled
    system's largest eigenvalue from above.  Chunks run on a thread pool
    (the batched products and eigvalsh release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    ks = _TetStiffness(sysd, E0, alpha)
    T = ks.T
    mshare = sysd["_elem_mass"]
    lam = np.empty(T)

    def one(s0):
        s1 = min(T, s0 + chunk)
        t = s1 - s0
        K = ks(s0, s1)
        wgt = 1.0 / np.sqrt(mshare[s0:s1].reshape(t, 24))
        Kh = K * wgt[:, :, None] * wgt[:, None, :]
        lam[s0:s1] = np.linalg.eigvalsh(Kh)[:, -1]

    starts = range(0, T, chunk)
    nw = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=nw) as ex:
        list(ex.map(one, starts))
    return lam


def global_stiffness(sysd, chunk=8192):
    """Assembled elastic stiffness (6N x 6N, scipy CSR) from the
    tetrahedra's matrices; used to compare stable steps across mass
    representations."""
    import scipy.sparse as sp
    mat = sysd["material"]
    ks = _TetStiffness(sysd, mat["E0"], mat["alpha"])
    tets = sysd["tet_nodes"].astype(np.int64)
    N = sysd["x0"].shape[0]
    rows, cols, vals = [], [], []
    for s0 in range(0, ks.T, chunk):
        s1 = min(ks.T, s0 + chunk)
        K = ks(s0, s1)
        dof = (6 * tets[s0:s1, :, None] + np.arange(6)[None, None, :]).reshape(-1, 24)
        rows.append(np.repeat(dof[:, :, None], 24, axis=2).ravel())
        cols.append(np.repeat(dof[:, None, :], 24, axis=1).ravel())
        vals.append(K.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(6 * N, 6 * N)).tocsr()
    return 0.5 * (K + K.T)


def mass_matrix(sysd):
    """Assembled mass (6N x 6N, scipy CSR): the per-cell blocks of
    `mass_block` when present, else the diagonal (mass, inertia)."""
    import scipy.sparse as sp
    N = sysd["x0"].shape[0]
    if sysd.get("mass_block") is not None:
        iu = np.triu_indices(6)
        B = np.zeros((N, 6, 6))
        B[:, iu[0], iu[1]] = sysd["mass_block"]
        B[:, iu[1], iu[0]] = sysd["mass_block"]
        return sp.block_diag(list(B), format="csr")
    d = np.empty((N, 6))
    d[:, :3] = np.asarray(sysd["mass"])[:, None]
    d[:, 3:] = sysd["inertia"]
    return sp.diags(d.ravel()).tocsr()


def lambda_max(sysd):
    """Largest eigenvalue of K phi = lambda M phi of the assembled system."""
    import scipy.sparse.linalg as sla
    K = global_stiffness(sysd)
    M = mass_matrix(sysd)
    return float(sla.eigsh(K, k=1, M=M, which="LA", tol=1e-9, return_eigenvectors=False)[0])


def boundary_triangles(tets):
    """Faces that belong to exactly one tetrahedron (outward orientation)."""
    faces = []
    for miss in range(4):
        nodes = [c for c in range(4) if c != miss]
        f = tets[:, nodes]
        # orient outward: the missing node must be on the negative side
        faces.append(np.concatenate([f, tets[:, miss:miss + 1]], axis=1))
    F = np.concatenate(faces, axis=0)
    key = np.sort(F[:, :3], axis=1)
    _, inv, cnt = np.unique(_triple_key(key, int(tets.max()) + 1), return_inverse=True, return_counts=True)
    once = cnt[inv.ravel()] == 1
    return F[once]


# --------------------------------------------------------------------------
# specimen assembly
# --------------------------------------------------------------------------
def build_geometry(shape: Shape, d0, da, seed, gap=0.1, rho=RHO, vol_fraction=None, device=False):
    """Seeded particles, Delaunay tetrahedra (host), then the tessellation
    and cell integrals: NumPy on the host, or ldpm_tessellate on the GPU
    when device=True (same construction, same layout)."""
    rng = np.random.default_rng(seed)
    xs = surface_nodes(shape, d0, rng)
    ds = np.full(xs.shape[0], d0)
    xi, di = place_particles(shape, d0, da, rng, gap=gap, vol_fraction=vol_fraction)
    x = np.concatenate([xs, xi], axis=0)
    diam = np.concatenate([ds, di])
    is_surf = np.concatenate([np.ones(xs.shape[0], bool), np.zeros(xi.shape[0], bool)])
    # Morton order of nodes
    order = np.argsort(_morton_keys(x), kind="stable")
    x, diam, is_surf = x[order], diam[order], is_surf[order]
    tets = delaunay_tets(x)
    tets = peel_boundary_slivers(x, tets, is_surf)
    # drop nodes not referenced by any tetrahedron
    used = np.zeros(x.shape[0], bool)
    used[tets.ravel()] = True
    remap = -np.ones(x.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.sum())
    x, diam, is_surf = x[used], diam[used], is_surf[used]
    tets = remap[tets]
    # Morton order of tetrahedra by centroid
    cen = x[tets].mean(axis=1)
    tets = tets[np.argsort(_morton_keys(cen), kind="stable")]
    if device:
        from . import ldpm
        g = ldpm.tessellate(x, diam, tets, rho, cones=True)
        c = g.pop("tet_node_cones")
        tr = c[..., 4:7].sum(-1)
        em = np.concatenate([np.repeat(rho * c[..., :1], 3, -1), rho * (tr[..., None] - c[..., 4:7])], -1)
        sysd = dict(x0=x, diam=diam, is_surface=is_surf, tet_nodes=tets.astype(np.int32), **g)
        sysd["_elem_mass"] = em
        return sysd
    fac, tri = tessellate(x, diam, tets)
    mass, inertia, cvol, roff, cJ = cell_mass_properties(x, tets, tri, rho)
    sysd = dict(x0=x, diam=diam, is_surface=is_surf, tet_nodes=tets.astype(np.int32),
                mass=mass, inertia=inertia, cell_vol=cvol, cell_r=roff, cell_inertia=cJ, **fac)
    sysd["_elem_mass"] = element_mass_share(x, tets, tri, rho)
    sysd["_tri"] = tri
    return sysd


def stable_dt(sysd, mat, fraction=0.8, device=False):
    """fraction x 2 / sqrt(max element eigenvalue); the element eigenvalues
    on the host (LAPACK) or, with device=True, on the GPU
    (ldpm_element_lambda)."""
    if device:
        from . import ldpm
        lam = ldpm.element_lambda_max(sysd, mat["E0"], mat["alpha"], sysd["_elem_mass"])
    else:
        lam = element_lambda_max(sysd, mat["E0"], mat["alpha"])
    return fraction * 2.0 / math.sqrt(lam.max()), lam


@dataclasses.dataclass
class Programs:
    """Piecewise-linear time programs (t_i, value_i); constant beyond ends."""
    t: List[np.ndarray] = dataclasses.field(default_factory=list)
    v: List[np.ndarray] = dataclasses.field(default_factory=list)

    def add(self, t, v):
        self.t.append(np.asarray(t, float))
        self.v.append(np.asarray(v, float))
        return len(self.t) - 1

    def pack(self):
        off = np.zeros(len(self.t) + 1, dtype=np.int64)
        for i, t in enumerate(self.t):
            off[i + 1] = off[i] + t.size
        tt = np.concatenate(self.t) if self.t else np.zeros(0)
        vv = np.concatenate(self.v) if self.v else np.zeros(0)
        return off, tt, vv


def finalize(sysd, mat, dof_mode, dof_prog, dof_scale, progs: Programs, v0, dt,
             name, meta=None):
    off, pt, pv = progs.pack()
    N = sysd["x0"].shape[0]
    out = {k: v for k, v in sysd.items() if not k.startswith("_")}
    out.update(dict(
        dof_mode=dof_mode.astype(np.uint8), dof_prog=dof_prog.astype(np.int32),
        dof_scale=dof_scale.astype(np.float64), prog_off=off, prog_t=pt, prog_v=pv,
        v0=v0.astype(np.float64), q0=np.zeros((N, 6)), dt=float(dt),
        body_force=np.zeros(3), material=dict(mat), name=name,
        meta=dict(meta or {}),
    ))
    out["meta"].update(N=int(N), T=int(sysd["tet_nodes"].shape[0]),
                       F=int(sysd["facet_I"].shape[0]))
    return out


def _box_faces(x, L, tol):
    return dict(xmin=np.abs(x[:, 0]) < tol, xmax=np.abs(x[:, 0] - L[0]) < tol,
                ymin=np.abs(x[:, 1]) < tol, ymax=np.abs(x[:, 1] - L[1]) < tol,
                zmin=np.abs(x[:, 2]) < tol, zmax=np.abs(x[:, 2] - L[2]) < tol)


def elastic_vibration_cube(edge=50.0, d0=4.0, da=8.0, seed=1, v0_amp=10.0,
                           mat=None, dt_fraction=0.8, device=False):
    """Elastic cube, all DoFs of the base fixed, initial sinusoidal velocity
    v_x = v0 sin(pi z / 2H), no damping."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    mat["law"] = 0
    shape = Shape("box", (edge, edge, edge))
    g = build_geometry(shape, d0, da, seed, device=device)
    x = g["x0"]
    N = x.shape[0]
    faces = _box_faces(x, shape.size, 1e-9)
    mode = np.zeros((N, 6), np.uint8)
    prog = -np.ones((N, 6), np.int32)
    scale = np.zeros((N, 6))
    mode[faces["zmin"]] = 1
    v0 = np.zeros((N, 6))
    v0[:, 0] = v0_amp * np.sin(np.pi * x[:, 2] / (2 * edge))
    v0[faces["zmin"]] = 0.0
    dt, lam = stable_dt(g, mat, dt_fraction, device=device)
    return finalize(g, mat, mode, prog, scale, Programs(), v0, dt,
                    f"elastic_cube{edge:g}_s{seed}",
                    dict(d0=d0, da=da, seed=seed, lam_max=float(lam.max()),
                         height=edge, area=edge * edge, load_prog=-1))


def tension_cube(edge=100.0, d0=4.0, da=10.0, seed=1, rate=1e-2, ramp=1e-3,
                 mat=None, dt_fraction=0.8, n_steps=200000, device=False):
    """Uniaxial tension: bottom face u=0, theta_x=theta_y=0; top face the same
    except u_z following a velocity program ramped over `ramp` seconds to
    rate * height."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    shape = Shape("box", (edge, edge, edge))
    g = build_geometry(shape, d0, da, seed, device=device)
    x = g["x0"]
    N = x.shape[0]
    faces = _box_faces(x, shape.size, 1e-9)
    mode = np.zeros((N, 6), np.uint8)
    prog = -np.ones((N, 6), np.int32)
    scale = np.zeros((N, 6))
    P = Programs()
    pid = P.add([0.0, ramp, 1e9], [0.0, 1.0, 1.0])
    for f in ("zmin", "zmax"):
        mode[faces[f], 0:5] = 1
    top = faces["zmax"]
    prog[top, 2] = pid
    scale[top, 2] = rate * edge
    v0 = np.zeros((N, 6))
    dt, lam = stable_dt(g, mat, dt_fraction, device=device)
    return finalize(g, mat, mode, prog, scale, P, v0, dt, f"tension_cube{edge:g}_s{seed}",
                    dict(d0=d0, da=da, seed=seed, rate=rate, lam_max=float(lam.max()),
                         height=edge, area=edge * edge, load_prog=pid, n_steps=n_steps))


def confined_compression_cube(edge=150.0, d0=4.0, da=12.0, seed=1, pressure=20.0,
                              final_strain=2e-2, n_steps=300000, mat=None,
                              dt_fraction=0.8, ramp_frac=0.1, device=False):
    """Lateral pressure as nodal forces (p times a third of each boundary
    triangle's area on the four lateral faces, ramped over the first
    ramp_frac of the run), then a top velocity; bottom u_z = 0."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    shape = Shape("box", (edge, edge, edge))
    g = build_geometry(shape, d0, da, seed, device=device)
    x = g["x0"]
    N = x.shape[0]
    L = shape.size
    faces = _box_faces(x, L, 1e-9)
    dt, lam = stable_dt(g, mat, dt_fraction, device=device)
    t_end = n_steps * dt
    t_ramp = ramp_frac * t_end
    mode = np.zeros((N, 6), np.uint8)
    prog = -np.ones((N, 6), np.int32)
    scale = np.zeros((N, 6))
    P = Programs()
    p_force = P.add([0.0, t_ramp, 1e9], [0.0, 1.0, 1.0])
    p_vel = P.add([0.0, t_ramp, t_ramp + 0.05 * (t_end - t_ramp), 1e9], [0.0, 0.0, 1.0, 1.0])
    bt = boundary_triangles(g["tet_nodes"].astype(np.int64))
    p = x[bt[:, :3]]
    cr = 0.5 * np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    inward = x[bt[:, 3]] - p.mean(axis=1)
    sg = np.sign(np.einsum("ij,ij->i", cr, inward))
    cr_out = -cr * sg[:, None]                     # outward vector area
    area = np.linalg.norm(cr_out, axis=1)
    nout = cr_out / area[:, None]
    force = np.zeros((N, 3))
    lateral = (np.abs(nout[:, 2]) < 0.5)
    for k in range(3):
        np.add.at(force, bt[lateral, k], -(pressure * area[lateral] / 3.0)[:, None] * nout[lateral])
    loaded = np.linalg.norm(force, axis=1) > 0
    for ax in range(2):
        sel = loaded & (np.abs(force[:, ax]) > 0)
        prog[sel, ax] = p_force
        scale[sel, ax] = force[sel, ax]
    bot, top = faces["zmin"], faces["zmax"]
    mode[bot, 2] = 1
    mode[top, 2] = 1
    mode[bot | top, 3:5] = 1
    v_top = -final_strain * edge / (t_end - t_ramp)
    prog[top, 2] = p_vel
    scale[top, 2] = v_top
    # pin one bottom-centre node laterally to remove rigid modes
    cen = np.argmin(np.where(bot, np.linalg.norm(x[:, :2] - np.asarray(L[:2]) / 2, axis=1), np.inf))
    mode[cen, 0:2] = 1
    mode[cen, 5] = 1
    v0 = np.zeros((N, 6))
    return finalize(g, mat, mode, prog, scale, P, v0, dt, f"confined_cube{edge:g}_s{seed}",
                    dict(d0=d0, da=da, seed=seed, pressure=pressure, lam_max=float(lam.max()),
                         height=edge, area=edge * edge, load_prog=p_vel, n_steps=n_steps))


def sliding_compression_cube(edge, d0=4.0, da=8.0, seed=0, rate=2.5e-2, ramp=1e-3,
                             mat=None, dt=None, dt_fraction=0.8, device=False):
    """Unconfined compression between frictionless platens: u_z prescribed on
    top (velocity) and bottom (zero); theta_x, theta_y fixed there; u_x, u_y,
    theta_z free except at the face-centre nodes."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    shape = Shape("box", (edge, edge, edge))
    g = build_geometry(shape, d0, da, seed, device=device)
    x = g["x0"]
    N = x.shape[0]
    L = shape.size
    faces = _box_faces(x, L, 1e-9)
    mode = np.zeros((N, 6), np.uint8)
    prog = -np.ones((N, 6), np.int32)
    scale = np.zeros((N, 6))
    P = Programs()
    pid = P.add([0.0, ramp, 1e9], [0.0, 1.0, 1.0])
    bot, top = faces["zmin"], faces["zmax"]
    for f in (bot, top):
        mode[f, 2] = 1
        mode[f, 3:5] = 1
        cen = np.argmin(np.where(f, np.linalg.norm(x[:, :2] - np.asarray(L[:2]) / 2, axis=1), np.inf))
        mode[cen, 0:2] = 1
        mode[cen, 5] = 1
    prog[top, 2] = pid
    scale[top, 2] = -rate * edge
    v0 = np.zeros((N, 6))
    dts, lam = stable_dt(g, mat, dt_fraction, device=device)
    return finalize(g, mat, mode, prog, scale, P, v0, dts if dt is None else dt,
                    f"sliding_cube{edge:g}_s{seed}",
                    dict(d0=d0, da=da, seed=seed, rate=rate, lam_max=float(lam.max()),
                         height=edge, area=edge * edge, load_prog=pid))


def concat_specimens(specs: List[dict], dt=None):
    """Concatenate independent specimens into one batched system (disjoint
    node sets, program ids offset); all advance with the same time step."""
    out = {}
    N_off = [0]
    T_off = [0]
    F_off = [0]
    P_off = [0]
    for s in specs:
        N_off.append(N_off[-1] + s["x0"].shape[0])
        T_off.append(T_off[-1] + s["tet_nodes"].shape[0])
        F_off.append(F_off[-1] + s["facet_I"].shape[0])
        P_off.append(P_off[-1] + s["prog_off"].size - 1)
    cat = lambda k: np.concatenate([s[k] for s in specs], axis=0)
    for k in ("x0", "diam", "is_surface", "mass", "inertia", "cell_vol", "cell_r",
              "facet_cI", "facet_n", "facet_m", "facet_area", "facet_len", "facet_area0",
              "dof_mode", "dof_scale", "v0", "q0"):
        out[k] = cat(k)
    for k in ("cell_inertia", "mass_block"):
        if all(k in s for s in specs):
            out[k] = cat(k)
    out["tet_nodes"] = np.concatenate([s["tet_nodes"] + N_off[i] for i, s in enumerate(specs)]).astype(np.int32)
    out["facet_I"] = np.concatenate([s["facet_I"] + N_off[i] for i, s in enumerate(specs)]).astype(np.int32)
    out["facet_J"] = np.concatenate([s["facet_J"] + N_off[i] for i, s in enumerate(specs)]).astype(np.int32)
    out["facet_tet"] = np.concatenate([s["facet_tet"] + T_off[i] for i, s in enumerate(specs)]).astype(np.int32)
    out["dof_prog"] = np.concatenate([np.where(s["dof_prog"] >= 0, s["dof_prog"] + P_off[i], -1)
                                      for i, s in enumerate(specs)]).astype(np.int32)
    offs = [0]
    pts, pvs = [], []
    for s in specs:
        o = s["prog_off"]
        for p in range(o.size - 1):
            pts.append(s["prog_t"][o[p]:o[p + 1]])
            pvs.append(s["prog_v"][o[p]:o[p + 1]])
            offs.append(offs[-1] + o[p + 1] - o[p])
    out["prog_off"] = np.array(offs, dtype=np.int64)
    out["prog_t"] = np.concatenate(pts) if pts else np.zeros(0)
    out["prog_v"] = np.concatenate(pvs) if pvs else np.zeros(0)
    out["dt"] = float(min(s["dt"] for s in specs) if dt is None else dt)
    out["body_force"] = np.zeros(3)
    out["material"] = dict(specs[0]["material"])
    out["name"] = f"batch{len(specs)}"
    out["particle_off"] = np.array(N_off, dtype=np.int64)
    out["tet_off"] = np.array(T_off, dtype=np.int64)
    out["facet_off"] = np.array(F_off, dtype=np.int64)
    out["meta"] = dict(N=N_off[-1], T=T_off[-1], F=F_off[-1], n_specimens=len(specs))
    return out


def system_hash(sysd):
    h = hashlib.sha1()
    for k in sorted(sysd.keys()):
        v = sysd[k]
        if isinstance(v, np.ndarray):
            h.update(k.encode())
            h.update(np.ascontiguousarray(v).tobytes())
    h.update(repr(sorted(sysd["material"].items())).encode())
    h.update(repr(sysd["dt"]).encode())
    return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# small fixtures
# --------------------------------------------------------------------------
def system_from_points(x, diam, tets=None, mat=None, rho=RHO, dt=None, name="points"):
    """A free-floating system (no prescribed DoFs) on explicit centres."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    x = np.asarray(x, float)
    diam = np.asarray(diam, float)
    if tets is None:
        tets = delaunay_tets(x)
    else:
        tets = np.asarray(tets, np.int64).copy()
        p = x[tets]
        v6 = np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])
        neg = v6 < 0
        tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    fac, tri = tessellate(x, diam, tets)
    mass, inertia, cvol, roff, cJ = cell_mass_properties(x, tets, tri, rho)
    g = dict(x0=x, diam=diam, is_surface=np.zeros(x.shape[0], bool),
             tet_nodes=tets.astype(np.int32), mass=mass, inertia=inertia, cell_vol=cvol,
             cell_r=roff, cell_inertia=cJ, **fac)
    g["_elem_mass"] = element_mass_share(x, tets, tri, rho)
    N = x.shape[0]
    if dt is None:
        dt, _ = stable_dt(g, mat, 0.8)
    return finalize(g, mat, np.zeros((N, 6), np.uint8), -np.ones((N, 6), np.int32),
                    np.zeros((N, 6)), Programs(), np.zeros((N, 6)), dt, name)


def single_tet(mat=None):
    x = np.array([[0.0, 0.0, 0.0], [10.0, 0.5, 0.2], [1.0, 9.0, 0.7], [0.8, 1.2, 9.5]])
    diam = np.array([4.0, 5.0, 4.5, 6.0])
    return system_from_points(x, diam, tets=[[0, 1, 2, 3]], mat=mat, name="single_tet")


def few_particle(n=12, seed=3, mat=None):
    """n jittered points in a ~20 mm box, Delaunay-meshed, free-floating."""
    rng = np.random.default_rng(seed)
    side = int(math.ceil(n ** (1 / 3)))
    g = np.stack(np.meshgrid(*[np.arange(side)] * 3, indexing="ij"), -1).reshape(-1, 3)[:n]
    x = g * 7.0 + rng.uniform(-1.2, 1.2, g.shape)
    diam = rng.uniform(3.0, 4.5, n)
    return system_from_points(x, diam, mat=mat, name=f"few{n}_s{seed}")


def _sliding_one(args):
    edge, seed, d0, da, rate = args
    return sliding_compression_cube(edge, d0=d0, da=da, seed=seed, rate=rate)


def batch_sliding_compression(n=64, seed=0, edge_range=(50.0, 100.0), d0=4.0, da=8.0,
                              rate=2.5e-2, workers=None):
    """n seeded realisations of unconfined compression with sliding platens,
    cube edges drawn uniformly from edge_range, concatenated into one batched
    system advancing with the smallest stable step of the set."""
    import concurrent.futures as cf
    import os
    rng = np.random.default_rng(seed)
    edges = rng.uniform(edge_range[0], edge_range[1], n)
    jobs = [(float(e), int(seed * 1000 + i), d0, da, rate) for i, e in enumerate(edges)]
    workers = workers or min(16, os.cpu_count() or 1, n)
    if workers > 1:
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            specs = list(ex.map(_sliding_one, jobs))
    else:
        specs = [_sliding_one(j) for j in jobs]
    out = concat_specimens(specs)
    out["name"] = f"batch_sliding{n}_s{seed}"
    out["meta"].update(edges=edges.tolist(), specimen_F=[s["meta"]["F"] for s in specs],
                       load_progs=[int(s["meta"]["load_prog"]) for s in specs], rate=rate)
    return out


def cylinder_cycle(D=100.0, H=200.0, d0=2.0, da=4.0, seed=1, eps_t=1.2e-4, eps_c=1.0e-3,
                   cycles=2, rate=0.2, mat=None, dt_fraction=0.8, device=False):
    """Cylinder (axis z) cycled between tension and compression: bottom face
    u_z = 0, theta_x = theta_y = 0 (centre node pinned laterally); top face
    theta_x = theta_y = 0 and u_z following a triangle wave of nominal strain
    rate `rate` between +eps_t H (about 0.9 of the tensile peak strain) and
    -eps_c H (about half of the compressive peak), `cycles` times."""
    mat = dict(MATERIAL_MB if mat is None else mat)
    shape = Shape("cylinder", (D, H))
    g = build_geometry(shape, d0, da, seed, device=device)
    x = g["x0"]
    N = x.shape[0]
    tol = 1e-9
    bot = np.abs(x[:, 2]) < tol
    top = np.abs(x[:, 2] - H) < tol
    mode = np.zeros((N, 6), np.uint8)
    prog = -np.ones((N, 6), np.int32)
    scale = np.zeros((N, 6))
    P = Programs()
    # triangle wave of the top displacement -> piecewise-constant velocity
    v = rate * H
    legs = []
    for _ in range(cycles):
        legs += [eps_t * H, -eps_c * H]
    t_pts, v_pts = [0.0], [v]
    u, t = 0.0, 0.0
    leg_end = []
    for target in legs:
        dur = abs(target - u) / v
        sgn = 1.0 if target > u else -1.0
        t_pts += [t + 1e-12, t + dur]
        v_pts += [sgn * v, sgn * v]
        t, u = t + dur, target
        leg_end.append(t)
    t_pts = np.array(t_pts[1:])
    v_pts = np.array(v_pts[1:])
    pid = P.add(np.concatenate([[0.0], t_pts, [t + 1e-9, 1e9]]),
                np.concatenate([[v_pts[0]], v_pts, [0.0, 0.0]]) / v)
    for f in (bot, top):
        mode[f, 2] = 1
        mode[f, 3:5] = 1
    cen = np.argmin(np.where(bot, np.linalg.norm(x[:, :2] - D / 2, axis=1), np.inf))
    mode[cen, 0:2] = 1
    mode[cen, 5] = 1
    prog[top, 2] = pid
    scale[top, 2] = v
    dt, lam = stable_dt(g, mat, dt_fraction, device=device)
    return finalize(g, mat, mode, prog, scale, P, np.zeros((N, 6)), dt, f"cylinder{D:g}x{H:g}_s{seed}",
                    dict(d0=d0, da=da, seed=seed, lam_max=float(lam.max()), height=H,
                         area=np.pi * D * D / 4, load_prog=pid, total_time=float(t),
                         n_steps=int(np.ceil(t / dt)), eps_t=eps_t, eps_c=eps_c, rate=rate,
                         leg_end_steps=[int(np.ceil(te / dt)) for te in leg_end]))


def perturbation(n_particles, eta, seed, index):
    """Random jump of every DoF (displacements and rotations) of n_particles
    particles, uniform in [-eta/2, eta/2], shape (N, 6): the random vector of
    the paper's perturbation study (section on time step, convergence
    criteria and stability).  Draw `index` of the sequence `seed`; the solver
    applies it to the free DoFs only."""
    if not eta >= 0.0:
        raise ValueError("eta must be non-negative")
    rng = np.random.default_rng([int(seed), int(index)])
    return rng.uniform(-0.5 * eta, 0.5 * eta, size=(int(n_particles), 6))


def synthetic_state(sysd, seed, strain, noise=0.3, t_normal=(-60.0, 4.0), t_shear=3.0,
                    emax_max=4e-4, step=1000):
    """A seeded, loaded state with facet history, for checks at full size that
    cannot afford a trajectory on the CPU: translations u = strain . x0 plus
    noise (relative amplitude `noise` of the strain times 4 mm, rotations
    likewise per mm), random mid-step velocities whose step increment dt v is
    about a tenth of the noise, facet tractions drawn uniformly (normal in
    t_normal, each shear component in +-t_shear, MPa) and e_max uniformly in
    [0, emax_max], independently of the strains.  Returns a dict with q, v
    (N, 6), t (F, 3), emax (F,), fext (N, 6) zero, and step."""
    rng = np.random.default_rng(seed)
    x = np.asarray(sysd["x0"], dtype=np.float64)
    N = x.shape[0]
    F = int(np.asarray(sysd["facet_I"]).shape[0])
    eps = np.asarray(strain, dtype=np.float64).reshape(3, 3)
    amp = noise * float(np.abs(eps).max()) * 4.0
    q = np.zeros((N, 6))
    q[:, :3] = x @ eps.T + amp * rng.standard_normal((N, 3))
    q[:, 3:] = 0.5 * (eps - eps.T)[[2, 0, 1], [1, 2, 0]] + (amp / 4.0) * rng.standard_normal((N, 3))
    v = (0.1 * amp / float(sysd["dt"])) * rng.standard_normal((N, 6))
    v[:, 3:] /= 4.0
    t = np.empty((F, 3))
    t[:, 0] = rng.uniform(t_normal[0], t_normal[1], F)
    t[:, 1:] = rng.uniform(-t_shear, t_shear, (F, 2))
    emax = rng.uniform(0.0, emax_max, F)
    return dict(q=q, v=v, t=t, emax=emax, fext=np.zeros((N, 6)), step=int(step))


def _upper21(M):
    """Upper triangle, row-major, of a stack of symmetric 6 x 6 matrices."""
    iu = np.triu_indices(6)
    return np.ascontiguousarray(M[:, iu[0], iu[1]])


def _rescale_dt(base, var):
    base = {k: v for k, v in base.items() if k != "mass_block"}
    r = lambda_max(base) / lambda_max(var)
    var["dt"] = float(base["dt"]) * math.sqrt(min(r, 1.0))
    var["meta"] = dict(var.get("meta", {}), dt_scale=math.sqrt(min(r, 1.0)),
                       lambda_ratio=r)


def mass_variant(sysd, kind):
    """The specimen with another mass representation (eq. balance and the
    section on the implementations' mass matrices):

    - "lumped": the diagonal of each cell's rigid-body mass block (mass,
      diagonal of the inertia tensor about the particle centre); the
      generator's default;
    - "cell_block": the full 6 x 6 rigid-body block of each cell about its
      particle centre, [[m 1, -[c]x], [[c]x, J]] with c = m r (first moment,
      r the centroid offset) and J the full inertia tensor, as `mass_block`
      (N, 21: upper triangle, row-major, DoFs u_x, u_y, u_z, th_x, th_y,
      th_z); its diagonal stays in mass / inertia;
    - "sphere": point masses from an equal split of each tetrahedron's mass
      (rho V_tet / 4 to each vertex) and an isotropic rotational inertia of
      a solid sphere of the particle's diameter, m d^2 / 10.
    The time step is scaled by sqrt(lambda_max(lumped) / lambda_max(variant))
    of the assembled systems, when that is below 1, so that the stability
    margin of the given step carries over.
    Returns a new dict (arrays shared where unchanged)."""
    out = dict(sysd)
    out.pop("mass_block", None)
    if kind == "lumped":
        return out
    if kind == "cell_block":
        m = np.asarray(sysd["mass"], dtype=np.float64)
        c = m[:, None] * np.asarray(sysd["cell_r"], dtype=np.float64)
        J = np.asarray(sysd["cell_inertia"], dtype=np.float64)
        N = m.size
        M = np.zeros((N, 6, 6))
        M[:, 0, 0] = M[:, 1, 1] = M[:, 2, 2] = m
        cx = np.zeros((N, 3, 3))
        cx[:, 0, 1], cx[:, 0, 2] = -c[:, 2], c[:, 1]
        cx[:, 1, 0], cx[:, 1, 2] = c[:, 2], -c[:, 0]
        cx[:, 2, 0], cx[:, 2, 1] = -c[:, 1], c[:, 0]
        M[:, :3, 3:] = -cx
        M[:, 3:, :3] = cx
        M[:, 3:, 3:] = J
        out["mass_block"] = _upper21(M)
        out["inertia"] = np.ascontiguousarray(np.einsum("nii->ni", J))
        _rescale_dt(sysd, out)
        return out
    if kind == "sphere":
        x = np.asarray(sysd["x0"], dtype=np.float64)
        tets = np.asarray(sysd["tet_nodes"], dtype=np.int64)
        p = x[tets]
        V = np.abs(np.einsum("ij,ij->i", np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0]), p[:, 3] - p[:, 0])) / 6.0
        rho = float(sysd["mass"].sum() / sysd["cell_vol"].sum())
        m = np.zeros(x.shape[0])
        np.add.at(m, tets.ravel(), np.repeat(rho * V / 4.0, 4))
        d = np.asarray(sysd["diam"], dtype=np.float64)
        out["mass"] = m
        out["inertia"] = np.repeat((m * d ** 2 / 10.0)[:, None], 3, axis=1)
        _rescale_dt(sysd, out)
        return out
    raise ValueError(f"unknown mass representation {kind!r}")
