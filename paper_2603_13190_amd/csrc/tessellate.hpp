// Device side of the on-device tessellation: from particle centres,
// diameters and tetrahedra, the 12 LDPM facets of every tetrahedron and the
// cone integrals of the polyhedral cells.  Included once, by ldpm.hip.
//
// Construction (the paper's preprocessor is not available; this is the
// construction the input generator documents): an edge point at mid-gap
// between the particle surfaces, clamped to [0.05, 0.95] of the edge; face
// points at the centroid of the face's edge points; the tetrahedron point
// at the centroid of the face points; facet = (edge point, point of the face
// through the edge and the third node, tetrahedron point).
#pragma once

struct TessIn {
    const double* __restrict__ x;    // [3][N]
    const double* __restrict__ diam; // [N]
    const int32_t* __restrict__ tet; // [4][T]
    int64_t N, T;
};

struct TessOut {
    int32_t *I, *J;        // [F]
    double *cI, *n, *m;    // [3][F]
    double *A, *A0, *len;  // [F]
    double* cone;          // [T][4][10]: the tet's part of each node's cell: V, V s / 4 (3),
                           // S (xx yy zz xy yz xz) about the node
};

__device__ __forceinline__ void cross3d(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// A group of 16 lanes per tetrahedron, lane k < 12 of the group builds facet
// k (so a wave's stores of one output array cover 48 consecutive facets).
// The tetrahedron's 6 edge points and 4 face points are evaluated once each,
// by different lanes of the group, and exchanged by shuffles.  Each facet's
// two cone integrals go to LDS; lanes then sum the 6 facets of each tet
// node in ascending facet order into the node's cone record.
constexpr int kTessTets = 16;  // tetrahedra per 256-lane block
// divisions by constants become products with their rounded reciprocals
// (one rounding more than a division: far below the 1e-12 parity bar)
constexpr double kThird = 1.0 / 3.0;

template <int N_>
__device__ __forceinline__ void pick3(const double (&src)[N_][3], int i, double dst[3])
{
#pragma unroll
    for (int c = 0; c < 3; c++) dst[c] = src[0][c];
#pragma unroll
    for (int j = 1; j < N_; j++)
        if (i == j) {
#pragma unroll
            for (int c = 0; c < 3; c++) dst[c] = src[j][c];
        }
}

__device__ __forceinline__ void facet_nodes(int k, int& a, int& b, int& cc)
{
    const int e = k >> 1;
    a = e < 3 ? 0 : (e < 5 ? 1 : 2);
    b = e == 0 ? 1 : (e == 1 || e == 3 ? 2 : 3);
    // third node: the lower of the two remaining nodes first
    const int lo = (a != 0 && b != 0) ? 0 : ((a != 1 && b != 1) ? 1 : 2);
    const int hi = 6 - a - b - lo;
    cc = (k & 1) ? hi : lo;
}

__global__ __launch_bounds__(256) void k_tessellate(TessIn in, TessOut out)
{
    __shared__ double s_c[kTessTets][12][2][10];
    const int g = threadIdx.x >> 4, k = threadIdx.x & 15;
    const int64_t t = (int64_t)blockIdx.x * kTessTets + g;
    const int64_t T = in.T, N = in.N, F = 12 * T;
    const bool tv = t < T;
    int64_t id[4] = {0, 0, 0, 0};
    double x[4][3], r[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        if (tv) id[a] = in.tet[(int64_t)a * T + t];
#pragma unroll
        for (int c = 0; c < 3; c++) x[a][c] = tv ? in.x[(int64_t)c * N + id[a]] : 0.0;
        r[a] = tv ? 0.5 * in.diam[id[a]] : 1.0;
    }
    if (!tv) {  // keep the arithmetic finite in idle groups
        x[1][0] = x[2][1] = x[3][2] = 1.0;
    }
    // shared points of the tetrahedron, one evaluation per lane of the
    // group: lane j holds edge point j mod 6 and face point j mod 4 (the
    // face without node j mod 4); the others are read by shuffles
    const int base = (int)(threadIdx.x & 63) & ~15;
    double epv[3], fpv[3], tp[3];
    {
        const int e = k % 6;
        const int a = e < 3 ? 0 : (e < 5 ? 1 : 2);
        const int b = e == 0 ? 1 : ((e == 1 || e == 3) ? 2 : 3);
        double xa[3], xb[3];
        pick3(x, a, xa);
        pick3(x, b, xb);
        const double ra = a == 0 ? r[0] : (a == 1 ? r[1] : r[2]);
        const double rb = b == 1 ? r[1] : (b == 2 ? r[2] : r[3]);
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; c++) d[c] = xb[c] - xa[c];
        const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double sl = 0.5 * (L + ra - rb);
        sl = sl < 0.05 * L ? 0.05 * L : (sl > 0.95 * L ? 0.95 * L : sl);
#pragma unroll
        for (int c = 0; c < 3; c++) epv[c] = xa[c] + d[c] * (sl / L);
    }
    {
        // face without node `miss`: its edges in the order of the three
        // remaining nodes (u, v), (u, w), (v, w)
        const int miss = k & 3;
        const int f0 = miss == 0 ? 3 : (miss == 1 ? 1 : 0);
        const int f1 = miss == 0 ? 4 : (miss == 3 ? 1 : 2);
        const int f2 = miss == 0 ? 5 : (miss == 1 ? 5 : (miss == 2 ? 4 : 3));
#pragma unroll
        for (int c = 0; c < 3; c++)
            fpv[c] = (__shfl(epv[c], base + f0) + __shfl(epv[c], base + f1) + __shfl(epv[c], base + f2)) * kThird;
#pragma unroll
        for (int c = 0; c < 3; c++)
            tp[c] = (__shfl(fpv[c], base + 0) + __shfl(fpv[c], base + 1) + __shfl(fpv[c], base + 2) +
                     __shfl(fpv[c], base + 3)) * 0.25;
    }

    const int kk = k < 12 ? k : 0;
    int a, b, cc;
    facet_nodes(kk, a, b, cc);
    const bool swap = id[b] < id[a];  // I = min, J = max of the particle ids
    const int aI = swap ? b : a, aJ = swap ? a : b;
    double P0[3], P1[3], xI[3], xJ[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        P0[c] = __shfl(epv[c], base + (kk >> 1));
        P1[c] = __shfl(fpv[c], base + (6 - a - b - cc));
    }
    pick3(x, aI, xI);
    pick3(x, aJ, xJ);
    double dv[3];
#pragma unroll
    for (int c = 0; c < 3; c++) dv[c] = xJ[c] - xI[c];
    const double L = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const double iL = 1.0 / L;
    const double n[3] = {dv[0] * iL, dv[1] * iL, dv[2] * iL};
    double u1[3], u2[3], cr[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        u1[c] = P1[c] - P0[c];
        u2[c] = tp[c] - P0[c];
    }
    cross3d(u1, u2, cr);
    double av[3] = {0.5 * cr[0], 0.5 * cr[1], 0.5 * cr[2]};
    const double sg = (av[0] * n[0] + av[1] * n[1] + av[2] * n[2]) < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int c = 0; c < 3; c++) av[c] *= sg;
    if (tv && k < 12) {
        const int64_t f = t * 12 + k;
        out.I[f] = (int32_t)id[aI];
        out.J[f] = (int32_t)id[aJ];
        out.A[f] = av[0] * n[0] + av[1] * n[1] + av[2] * n[2];
        out.A0[f] = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
        out.len[f] = L;
        // tangent m = normalise(n x e_k), e_k the axis of the smallest |n_k|
        const double a0 = fabs(n[0]), a1 = fabs(n[1]), a2 = fabs(n[2]);
        const int ax = (a0 <= a1 && a0 <= a2) ? 0 : (a1 <= a2 ? 1 : 2);
        const double ek[3] = {ax == 0 ? 1.0 : 0.0, ax == 1 ? 1.0 : 0.0, ax == 2 ? 1.0 : 0.0};
        double m[3];
        cross3d(n, ek, m);
        const double imn = 1.0 / sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            out.n[c * F + f] = n[c];
            out.m[c * F + f] = m[c] * imn;
            out.cI[c * F + f] = (P0[c] + P1[c] + tp[c]) * kThird - xI[c];
        }
    }
    // cones (centre, triangle) of the I cell (side 0, outward +n) and of the
    // J cell (side 1, outward -n); the triangle winds about the oriented
    // area, so the sign of its volume is sg
    if (k < 12) {
#pragma unroll
        for (int side = 0; side < 2; side++) {
            const double* xo = side == 0 ? xI : xJ;
            const double sgn = side == 0 ? sg : -sg;
            double q1[3], q2[3], q3[3], q12[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                q1[c] = P0[c] - xo[c];
                q2[c] = P1[c] - xo[c];
                q3[c] = tp[c] - xo[c];
            }
            cross3d(q1, q2, q12);
            const double V = sgn * (q12[0] * q3[0] + q12[1] * q3[1] + q12[2] * q3[2]) * (1.0 / 6.0);
            const double s3[3] = {q1[0] + q2[0] + q3[0], q1[1] + q2[1] + q3[1], q1[2] + q2[2] + q3[2]};
            double* o = s_c[g][k][side];
            o[0] = V;
#pragma unroll
            for (int c = 0; c < 3; c++) o[1 + c] = V * s3[c] / 4.0;
            constexpr int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int p = 0; p < 6; p++) {
                const int i = ii[p], j = jj[p];
                o[4 + p] = (q1[i] * q1[j] + q2[i] * q2[j] + q3[i] * q3[j] + s3[i] * s3[j]) * (V * (1.0 / 20.0));
            }
        }
    }
    __syncthreads();
    if (!tv) return;
    // node records: value v = (node na, component q), 40 per tetrahedron
    for (int v = k; v < 40; v += 16) {
        const int na = v / 10, q = v - 10 * na;
        double acc = 0.0;
#pragma unroll
        for (int kf = 0; kf < 12; kf++) {
            int fa, fb, fc;
            facet_nodes(kf, fa, fb, fc);
            if (fa == na || fb == na) {
                const bool sw = id[fb] < id[fa];
                const int fI = sw ? fb : fa;
                acc += s_c[g][kf][fI == na ? 0 : 1][q];
            }
        }
        out.cone[t * 40 + v] = acc;
    }
}

// cell properties: a group of 16 lanes per particle, lane q < 10 sums
// component q of the particle's cone records, found through the incidence
// list inc (record index 4 t + a, ascending t), so that the group reads each
// 80-byte record in one pass; the sums are shared in the group by shuffles.  mass = rho V,
// J = rho (tr(S) 1 - S), r = (first moment) / V.
constexpr int kCellGroup = 16;

__global__ __launch_bounds__(256) void k_cells(const int32_t* __restrict__ ptr, const int32_t* __restrict__ inc,
                                               const double* __restrict__ cone,
                                               int64_t N, double rho, double* __restrict__ mass,
                                               double* __restrict__ vol, double* __restrict__ rcell,
                                               double* __restrict__ Jd, double* __restrict__ J6)
{
    const int q = threadIdx.x & (kCellGroup - 1);
    const int64_t I = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kCellGroup;
    // whole groups leave together: the shuffles below stay within a group
    if (I >= N) return;
    double acc = 0.0;
    if (q < 10)
        for (int32_t p = ptr[I]; p < ptr[I + 1]; p++) acc += cone[(int64_t)inc[p] * 10 + q];
    double sv[10];
#pragma unroll
    for (int j = 0; j < 10; j++) sv[j] = __shfl(acc, j, kCellGroup);
    const double V = sv[0];
    const double tr = sv[4] + sv[5] + sv[6];
    const double iv = V > 0.0 ? 1.0 / V : 0.0;
    if (q == 0) {
        mass[I] = rho * V;
        vol[I] = V;
    }
    if (q < 3) {
        const double s1 = q == 0 ? sv[1] : (q == 1 ? sv[2] : sv[3]);
        const double sd = q == 0 ? sv[4] : (q == 1 ? sv[5] : sv[6]);
        rcell[q * N + I] = s1 * iv;
        Jd[q * N + I] = rho * (tr - sd);
    }
    // J6: xx yy zz xy yz xz
    if (q < 6) {
        const double sq = q == 1 ? sv[5] : (q == 2 ? sv[6] : sv[4]);
        const double so = q == 3 ? sv[7] : (q == 4 ? sv[8] : sv[9]);
        J6[q * N + I] = q < 3 ? rho * (tr - sq) : -rho * so;
    }
}
