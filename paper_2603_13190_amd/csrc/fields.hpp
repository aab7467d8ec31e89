// Device side of the post-processing and perturbation calls: crack-opening
// vectors, tetrahedron volumetric strains, the random-perturbation jump and
// the deterministic comparison of two fields (Pearson's correlation and
// NRMSE).  None of these runs inside a step; all are one pass over their
// data.  Included once, by ldpm.hip, after step_kernels.hpp.
#pragma once

// geometry of facet f in FP64: frame, centroid offsets, length, area and
// the two particles
struct FacetGeo {
    double n[3], m[3], l[3], cI[3], cJ[3];
    double len, area;
    int64_t I, J;
};

template <typename R>
__device__ __forceinline__ FacetGeo facet_geo(const FacetArgs<R>& fa, const int32_t* __restrict__ tet, int64_t T,
                                              int64_t f)
{
    FacetGeo g;
    const int32_t rc = fa.rec[f];
    const R* fr = fa.frame + (int64_t)(rc & 0x0fffffff) * 8;
    const int aI = (rc >> 28) & 3, aJ = (rc >> 30) & 3;
    const int64_t t = f / 12;
    g.I = tet[(int64_t)aI * T + t];
    g.J = tet[(int64_t)aJ * T + t];
    const int64_t F = fa.F;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        g.n[c] = (double)fr[c];
        g.m[c] = (double)fr[3 + c];
        g.cI[c] = (double)fa.geo[quad_index<R>(F, f, c)];
    }
    g.len = (double)fr[6];
    g.area = (double)fa.geo[quad_index<R>(F, f, 3)];
    g.l[0] = g.n[1] * g.m[2] - g.n[2] * g.m[1];
    g.l[1] = g.n[2] * g.m[0] - g.n[0] * g.m[2];
    g.l[2] = g.n[0] * g.m[1] - g.n[1] * g.m[0];
#pragma unroll
    for (int c = 0; c < 3; c++) g.cJ[c] = g.cI[c] - g.len * g.n[c];
    return g;
}

// e = P^T [[x]] / len for generalised displacements a (particle I) and b
// (particle J), each 6 values (translation, rotation) with stride st
// (eq. strain1)
__device__ __forceinline__ void rel_strain(const FacetGeo& g, const double* a, const double* b, int64_t st,
                                           double e[3])
{
    const double aT[3] = {a[3 * st], a[4 * st], a[5 * st]};
    const double bT[3] = {b[3 * st], b[4 * st], b[5 * st]};
    double d[3];
    d[0] = b[0] - a[0] + (bT[1] * g.cJ[2] - bT[2] * g.cJ[1]) - (aT[1] * g.cI[2] - aT[2] * g.cI[1]);
    d[1] = b[st] - a[st] + (bT[2] * g.cJ[0] - bT[0] * g.cJ[2]) - (aT[2] * g.cI[0] - aT[0] * g.cI[2]);
    d[2] = b[2 * st] - a[2 * st] + (bT[0] * g.cJ[1] - bT[1] * g.cJ[0]) - (aT[0] * g.cI[1] - aT[1] * g.cI[0]);
    e[0] = (g.n[0] * d[0] + g.n[1] * d[1] + g.n[2] * d[2]) / g.len;
    e[1] = (g.m[0] * d[0] + g.m[1] * d[1] + g.m[2] * d[2]) / g.len;
    e[2] = (g.l[0] * d[0] + g.l[1] * d[1] + g.l[2] * d[2]) / g.len;
}

// strain of facet f at the configuration of the last law evaluation,
// q^{n-1} = q^n - dt v^{n-1/2} (node records hold q^n and v^{n-1/2})
__device__ __forceinline__ void last_strain(const FacetGeo& g, const double* __restrict__ node, double dt,
                                            double e[3])
{
    double eq[3], ev[3];
    rel_strain(g, node + g.I * 16, node + g.J * 16, 1, eq);
    rel_strain(g, node + g.I * 16 + 6, node + g.J * 16 + 6, 1, ev);
#pragma unroll
    for (int c = 0; c < 3; c++) e[c] = eq[c] - dt * ev[c];
}

// Crack opening of every facet: w = len (e - E^{-1} t), E = E0 diag(1, a, a),
// w_N = max(w_N, 0); out [4][F] = w_N, w_M, w_L, |w|.  first: no law
// evaluation yet (the history belongs to the undeformed state).  One block
// per TB tetrahedra: the 4 TB node records (q, v) are staged in LDS once
// and read by the tets' 12 facets, one lane per facet.
template <typename R, int TB>
__global__ __launch_bounds__(12 * TB) void k_crack(NodeArgs na, FacetArgs<R> fa, double E0, double aE0, double dt,
                                                   int first, double* __restrict__ out)
{
    constexpr int NS = 4 * TB;
    __shared__ double s_u[6][NS];  // q - dt v: the configuration of the last law evaluation
    const int tid = threadIdx.x;
    const int64_t T = na.T, F = fa.F;
    const int64_t tet0 = (int64_t)blockIdx.x * TB;
    // facet data first (independent of the staging)
    const int tl = tid / 12;
    const bool valid = tet0 + tl < T;
    const int64_t f = (tet0 + tl) * 12 + (tid % 12);
    int32_t rc = 0;
    double n[3] = {0, 0, 0}, m[3] = {0, 0, 0}, cI[3] = {0, 0, 0}, t[3] = {0, 0, 0}, len = 1.0;
    if (valid) {
        rc = fa.rec[f];
        const R* fr = fa.frame + (int64_t)(rc & 0x0fffffff) * 8;
        R g[4], h[4];
        ld_quad<0>(fa.geo, F, f, g[0], g[1], g[2], g[3]);
        ld_quad<0>((const R*)fa.hist, F, f, h[0], h[1], h[2], h[3]);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            n[c] = (double)fr[c];
            m[c] = (double)fr[3 + c];
            cI[c] = (double)g[c];
            t[c] = (double)h[c];
        }
        len = (double)fr[6];
    }
    if (tid < NS) {
        const int ttl = tid % TB, a = tid / TB;
        if (tet0 + ttl < T) {
            const double* r = na.node + (int64_t)na.tet[(int64_t)a * T + tet0 + ttl] * 16;
#pragma unroll
            for (int c = 0; c < 6; c++) s_u[c][tid] = first ? 0.0 : r[c] - dt * r[6 + c];
        }
    }
    __syncthreads();
    if (!valid) return;
    const int aI = (rc >> 28) & 3, aJ = (rc >> 30) & 3;
    const int sI = aI * TB + tl, sJ = aJ * TB + tl;
    const double l[3] = {n[1] * m[2] - n[2] * m[1], n[2] * m[0] - n[0] * m[2], n[0] * m[1] - n[1] * m[0]};
    const double cJ[3] = {cI[0] - len * n[0], cI[1] - len * n[1], cI[2] - len * n[2]};
    double uI[6], uJ[6];
#pragma unroll
    for (int c = 0; c < 6; c++) {
        uI[c] = s_u[c][sI];
        uJ[c] = s_u[c][sJ];
    }
    // [[u]] = u_J + th_J x c^J - u_I - th_I x c^I (eq. strain1)
    double d[3];
    d[0] = uJ[0] - uI[0] + (uJ[4] * cJ[2] - uJ[5] * cJ[1]) - (uI[4] * cI[2] - uI[5] * cI[1]);
    d[1] = uJ[1] - uI[1] + (uJ[5] * cJ[0] - uJ[3] * cJ[2]) - (uI[5] * cI[0] - uI[3] * cI[2]);
    d[2] = uJ[2] - uI[2] + (uJ[3] * cJ[1] - uJ[4] * cJ[0]) - (uI[3] * cI[1] - uI[4] * cI[0]);
    const double e0 = (n[0] * d[0] + n[1] * d[1] + n[2] * d[2]) / len;
    const double e1 = (m[0] * d[0] + m[1] * d[1] + m[2] * d[2]) / len;
    const double e2 = (l[0] * d[0] + l[1] * d[1] + l[2] * d[2]) / len;
    double wN = len * (e0 - t[0] / E0);
    const double wM = len * (e1 - t[1] / aE0);
    const double wL = len * (e2 - t[2] / aE0);
    wN = wN > 0.0 ? wN : 0.0;
    out[f] = wN;
    out[F + f] = wM;
    out[2 * F + f] = wL;
    out[3 * F + f] = sqrt(wN * wN + wM * wM + wL * wL);
}

// e_V = (1/3) sum_a grad N_a . u_a of every tetrahedron (appendix,
// compressive behaviour), with
//   u = q^n - dt v^{n-1/2} (+ jump d [6][N], if given),
// i.e. at the configuration of the last law evaluation.
// With J = [x1 - x0, x2 - x0, x3 - x0] the rows of J^{-1} are
// (b x c, c x a, a x b) / det, so 3 e_V = tr(U J^{-1}).
__global__ __launch_bounds__(256) void k_volstrain(NodeArgs na, double dt, int first, const double* __restrict__ d,
                                                   double* __restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t T = na.T, N = na.N;
    if (t >= T) return;
    if (first && !d) {
        out[t] = 0.0;
        return;
    }
    double x[4][3], u[4][3];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int64_t nd = na.tet[(int64_t)a * T + t];
        const double* r = na.node + nd * 16;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            x[a][c] = r[12 + c];
            u[a][c] = first ? 0.0 : r[c] - dt * r[6 + c];
            if (d) u[a][c] += d[(int64_t)c * N + nd];
        }
    }
    double A[3], B[3], Cc[3], Ua[3], Ub[3], Uc[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        A[c] = x[1][c] - x[0][c];
        B[c] = x[2][c] - x[0][c];
        Cc[c] = x[3][c] - x[0][c];
        Ua[c] = u[1][c] - u[0][c];
        Ub[c] = u[2][c] - u[0][c];
        Uc[c] = u[3][c] - u[0][c];
    }
    const double bc[3] = {B[1] * Cc[2] - B[2] * Cc[1], B[2] * Cc[0] - B[0] * Cc[2], B[0] * Cc[1] - B[1] * Cc[0]};
    const double ca[3] = {Cc[1] * A[2] - Cc[2] * A[1], Cc[2] * A[0] - Cc[0] * A[2], Cc[0] * A[1] - Cc[1] * A[0]};
    const double ab[3] = {A[1] * B[2] - A[2] * B[1], A[2] * B[0] - A[0] * B[2], A[0] * B[1] - A[1] * B[0]};
    const double det = A[0] * bc[0] + A[1] * bc[1] + A[2] * bc[2];
    const double tr = (Ua[0] * bc[0] + Ua[1] * bc[1] + Ua[2] * bc[2]) + (Ub[0] * ca[0] + Ub[1] * ca[1] + Ub[2] * ca[2]) +
                      (Uc[0] * ab[0] + Uc[1] * ab[1] + Uc[2] * ab[2]);
    out[t] = tr / det / 3.0;
}

// prescribed DoFs take no part in a perturbation: d[id] = 0 where mode != 0
__global__ __launch_bounds__(256) void k_mask_free(const uint8_t* __restrict__ mode, int64_t n6,
                                                   double* __restrict__ d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n6 && mode[i] != 0) d[i] = 0.0;
}

// The facet law takes the jump d as a strain increment of its own, from the
// configuration of the last evaluation to that configuration plus the jump;
// evj [T]: e_V after the jump.  One thread per tetrahedron, its 12 facets in
// order; the traction work of the jump goes to w_int and to wj [T].
template <typename R, int LAW>
__global__ __launch_bounds__(256) void k_jump(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                              const double* __restrict__ d, const double* __restrict__ evj,
                                              double dt, double* __restrict__ wint, double* __restrict__ wj)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t T = na.T, N = na.N, F = fa.F;
    if (t >= T) return;
    const R eV = (R)evj[t];
    double W = 0.0;
    for (int k = 0; k < 12; k++) {
        const int64_t f = t * 12 + k;
        const FacetGeo g = facet_geo(fa, na.tet, T, f);
        double e[3], de[3];
        last_strain(g, na.node, dt, e);
        rel_strain(g, d + g.I, d + g.J, N, de);
        R er[3], der[3], tv[3], told[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            er[c] = (R)(e[c] + de[c]);
            der[c] = (R)de[c];
            tv[c] = fa.hist[quad_index<R>(F, f, c)];
            told[c] = tv[c];
        }
        R em = fa.hist[quad_index<R>(F, f, 3)];
        facet_law<R, LAW>(mat, (R)g.len, er, der, eV, tv, em);
        double w = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) w += 0.5 * ((double)told[c] + (double)tv[c]) * de[c];
        W += g.area * g.len * w;
#pragma unroll
        for (int c = 0; c < 3; c++) fa.hist[quad_index<R>(F, f, c)] = tv[c];
        fa.hist[quad_index<R>(F, f, 3)] = em;
    }
    wint[t] += W;
    wj[t] = W;
}

// q^n += d for every DoF (d already masked)
__global__ __launch_bounds__(256) void k_add_jump(double* __restrict__ node, const double* __restrict__ d, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * N) return;
    const int64_t c = i / N, p = i - c * N;
    node[p * 16 + c] += d[i];
}

// out[0] = sum of x[a..b) in a fixed order (one block)
__global__ __launch_bounds__(RED_THREADS) void k_range_sum(const double* __restrict__ x, int64_t a, int64_t b,
                                                           double* __restrict__ out)
{
    double s = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += RED_THREADS) s += x[i];
    s = block_sum_fixed(s);
    if (threadIdx.x == 0) out[0] = s;
}

// ---------------------------------------------------------------------------
// field comparison: count, means, centred second moments and co-moment,
// sum of squared differences and the maximum of the reference; per lane
// from shifted sums, then merged pairwise (Chan et al.'s combination) in a
// fixed tree
// ---------------------------------------------------------------------------
struct Moments {
    double n, mx, mr, sxx, srr, sxr, sse, rmax;
};

__device__ __forceinline__ Moments mom_merge(const Moments& A, const Moments& B)
{
    if (B.n == 0.0) return A;
    if (A.n == 0.0) return B;
    Moments o;
    o.n = A.n + B.n;
    const double dx = B.mx - A.mx, dr = B.mr - A.mr;
    const double fb = B.n / o.n, w = A.n * fb;  // nA nB / n
    o.mx = A.mx + dx * fb;
    o.mr = A.mr + dr * fb;
    o.sxx = A.sxx + B.sxx + dx * dx * w;
    o.srr = A.srr + B.srr + dr * dr * w;
    o.sxr = A.sxr + B.sxr + dx * dr * w;
    o.sse = A.sse + B.sse;
    o.rmax = A.rmax > B.rmax ? A.rmax : B.rmax;
    return o;
}

constexpr int CMP_THREADS = 256;
constexpr int CMP_MAX_BLOCKS = 2048;

__device__ Moments block_merge(Moments m)
{
    __shared__ Moments s[CMP_THREADS];
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = CMP_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = mom_merge(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    const Moments r = s[0];
    __syncthreads();
    return r;
}

// one partial per block; thread i of block b takes elements
// i + CMP_THREADS b + CMP_THREADS G k, k = 0, 1, ... (coalesced), and sums
// them shifted by its first pair (no division per element; the shift keeps
// the centred sums well conditioned), then forms its moments
__global__ __launch_bounds__(CMP_THREADS) void k_cmp_partial(const double* __restrict__ x,
                                                             const double* __restrict__ r, int64_t n, double cap,
                                                             int use_cap, Moments* __restrict__ part)
{
    double cnt = 0.0, kx = 0.0, kr = 0.0, sx = 0.0, sr = 0.0, sxx = 0.0, srr = 0.0, sxr = 0.0, sse = 0.0;
    double rmax = -INFINITY;
    const int64_t stride = (int64_t)gridDim.x * CMP_THREADS;
    const int64_t i0 = (int64_t)blockIdx.x * CMP_THREADS + threadIdx.x;
    if (i0 < n) {
        kx = x[i0];
        kr = r[i0];
        if (use_cap) {
            kx = kx < cap ? kx : cap;
            kr = kr < cap ? kr : cap;
        }
    }
    for (int64_t i = i0; i < n; i += stride) {
        double a = x[i], b = r[i];
        if (use_cap) {
            a = a < cap ? a : cap;
            b = b < cap ? b : cap;
        }
        const double da = a - kx, db = b - kr;
        cnt += 1.0;
        sx += da;
        sr += db;
        sxx += da * da;
        srr += db * db;
        sxr += da * db;
        sse += (a - b) * (a - b);
        rmax = b > rmax ? b : rmax;
    }
    Moments m{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY};
    if (cnt > 0.0) {
        const double inv = 1.0 / cnt;
        m.n = cnt;
        m.mx = kx + sx * inv;
        m.mr = kr + sr * inv;
        m.sxx = sxx - sx * sx * inv;
        m.srr = srr - sr * sr * inv;
        m.sxr = sxr - sx * sr * inv;
        m.sse = sse;
        m.rmax = rmax;
    }
    m = block_merge(m);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// merge the G partials (thread i takes i, i + CMP_THREADS, ... in order)
// and finish: out = n, mean_x, mean_ref, pearson, rmse, ref_max, nrmse
__global__ __launch_bounds__(CMP_THREADS) void k_cmp_final(const Moments* __restrict__ part, int G,
                                                           double* __restrict__ out)
{
    Moments m{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, -INFINITY};
    for (int i = threadIdx.x; i < G; i += CMP_THREADS) m = mom_merge(m, part[i]);
    m = block_merge(m);
    if (threadIdx.x == 0) {
        const double rmse = sqrt(m.sse / m.n);
        out[0] = m.n;
        out[1] = m.mx;
        out[2] = m.mr;
        out[3] = m.sxr / sqrt(m.sxx * m.srr);
        out[4] = rmse;
        out[5] = m.rmax;
        out[6] = 100.0 * rmse / m.rmax;
    }
}
