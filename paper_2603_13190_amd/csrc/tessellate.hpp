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
    const int32_t* __restrict__ pos; // [4T]: incidence position of tet node (t, a)
    int64_t N, T;
};

struct TessOut {
    int32_t *I, *J;        // [F]
    double *cI, *n, *m;    // [3][F]
    double *A, *A0, *len;  // [F]
    double* cone;          // [4T][10] in incidence order: V, V s / 4 (3), S (xx yy zz xy yz xz)
};

// edges (a, b) and, for facet k = 2 e + j, the third node c of its face;
// compile-time tables so that the unrolled loops index registers only
constexpr int kEdgeA[6] = {0, 0, 0, 1, 1, 2};
constexpr int kEdgeB[6] = {1, 2, 3, 2, 3, 3};
constexpr int kThird[12] = {2, 3, 1, 3, 1, 2, 0, 3, 0, 2, 0, 1};

__device__ __forceinline__ void cross3d(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// one lane per tetrahedron
__global__ __launch_bounds__(128) void k_tessellate(TessIn in, TessOut out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t T = in.T, N = in.N, F = 12 * T;
    if (t >= T) return;
    int64_t id[4];
    double x[4][3], r[4];
#pragma unroll
    for (int a = 0; a < 4; a++) {
        id[a] = in.tet[(int64_t)a * T + t];
#pragma unroll
        for (int c = 0; c < 3; c++) x[a][c] = in.x[(int64_t)c * N + id[a]];
        r[a] = 0.5 * in.diam[id[a]];
    }
    double ep[6][3];
#pragma unroll
    for (int e = 0; e < 6; e++) {
        const int a = kEdgeA[e], b = kEdgeB[e];
        double d[3];
#pragma unroll
        for (int c = 0; c < 3; c++) d[c] = x[b][c] - x[a][c];
        const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double s = 0.5 * (L + r[a] - r[b]);
        s = s < 0.05 * L ? 0.05 * L : (s > 0.95 * L ? 0.95 * L : s);
#pragma unroll
        for (int c = 0; c < 3; c++) ep[e][c] = x[a][c] + d[c] * (s / L);
    }
    // face point of the face without node `miss`: its edges, in the order
    // of the three remaining nodes (u, v), (u, w), (v, w)
    double fp[4][3];
    const int fe[4][3] = {{3, 4, 5}, {1, 2, 5}, {0, 2, 4}, {0, 1, 3}};
#pragma unroll
    for (int miss = 0; miss < 4; miss++)
#pragma unroll
        for (int c = 0; c < 3; c++)
            fp[miss][c] = (ep[fe[miss][0]][c] + ep[fe[miss][1]][c] + ep[fe[miss][2]][c]) / 3.0;
    double tp[3];
#pragma unroll
    for (int c = 0; c < 3; c++) tp[c] = (fp[0][c] + fp[1][c] + fp[2][c] + fp[3][c]) / 4.0;
    double acc[4][10];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int k = 0; k < 10; k++) acc[a][k] = 0.0;
#pragma unroll
    for (int k = 0; k < 12; k++) {
        const int e = k >> 1;
        const int a = kEdgeA[e], b = kEdgeB[e], cc = kThird[k];
        const int dmiss = 6 - a - b - cc;
        const int aI = id[a] < id[b] ? a : b, aJ = id[a] < id[b] ? b : a;
        const double* P0 = ep[e];
        const double* P1 = fp[dmiss];
        const double* P2 = tp;
        double dv[3];
#pragma unroll
        for (int c = 0; c < 3; c++) dv[c] = x[aJ][c] - x[aI][c];
        const double L = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
        const double n[3] = {dv[0] / L, dv[1] / L, dv[2] / L};
        double u1[3], u2[3], cr[3];
#pragma unroll
        for (int c = 0; c < 3; c++) {
            u1[c] = P1[c] - P0[c];
            u2[c] = P2[c] - P0[c];
        }
        cross3d(u1, u2, cr);
        double av[3] = {0.5 * cr[0], 0.5 * cr[1], 0.5 * cr[2]};
        const double an = av[0] * n[0] + av[1] * n[1] + av[2] * n[2];
        const double sg = an < 0.0 ? -1.0 : 1.0;
#pragma unroll
        for (int c = 0; c < 3; c++) av[c] *= sg;
        const int64_t f = t * 12 + k;
        out.I[f] = (int32_t)id[aI];
        out.J[f] = (int32_t)id[aJ];
        out.A[f] = av[0] * n[0] + av[1] * n[1] + av[2] * n[2];
        out.A0[f] = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
        out.len[f] = L;
        // tangent m = normalise(n x e_k), e_k the axis of the smallest |n_k|
        const double a0 = fabs(n[0]), a1 = fabs(n[1]), a2 = fabs(n[2]);
        const int ax = (a0 <= a1 && a0 <= a2) ? 0 : (a1 <= a2 ? 1 : 2);
        double ek[3] = {0.0, 0.0, 0.0};
        ek[ax] = 1.0;
        double m[3];
        cross3d(n, ek, m);
        const double mn = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
#pragma unroll
        for (int c = 0; c < 3; c++) {
            out.n[c * F + f] = n[c];
            out.m[c * F + f] = m[c] / mn;
            out.cI[c * F + f] = (P0[c] + P1[c] + P2[c]) / 3.0 - x[aI][c];
        }
        // cones (centre, triangle): signed volume, first and second moments;
        // the triangle winds about the oriented area when cr . av > 0
        const double orient = sg;
#pragma unroll
        for (int side = 0; side < 2; side++) {
            const int an_ = side == 0 ? aI : aJ;
            const double sgn = side == 0 ? 1.0 : -1.0;
            double q1[3], q2[3], q3[3], q12[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                q1[c] = P0[c] - x[an_][c];
                q2[c] = P1[c] - x[an_][c];
                q3[c] = P2[c] - x[an_][c];
            }
            cross3d(q1, q2, q12);
            const double V = sgn * orient * (q12[0] * q3[0] + q12[1] * q3[1] + q12[2] * q3[2]) / 6.0;
            const double s3[3] = {q1[0] + q2[0] + q3[0], q1[1] + q2[1] + q3[1], q1[2] + q2[2] + q3[2]};
            double* A_ = acc[an_];
            A_[0] += V;
#pragma unroll
            for (int c = 0; c < 3; c++) A_[1 + c] += V * s3[c] / 4.0;
            const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int p = 0; p < 6; p++) {
                const int i = ii[p], j = jj[p];
                A_[4 + p] += (q1[i] * q1[j] + q2[i] * q2[j] + q3[i] * q3[j] + s3[i] * s3[j]) * (V / 20.0);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 4; a++) {
        double* o = out.cone + (int64_t)in.pos[4 * t + a] * 10;
#pragma unroll
        for (int k = 0; k < 10; k++) o[k] = acc[a][k];
    }
}

// cell properties: the cone records of each particle summed in incidence
// (ascending tetrahedron) order; mass = rho V, J = rho (tr(S) 1 - S),
// r = (first moment) / V.  cell[11][N]: V, m1 (3), S (6), then derived
// outputs are written separately.
__global__ __launch_bounds__(256) void k_cells(const int32_t* __restrict__ ptr, const double* __restrict__ cone,
                                               int64_t N, double rho, double* __restrict__ mass,
                                               double* __restrict__ vol, double* __restrict__ rcell,
                                               double* __restrict__ Jd, double* __restrict__ J6)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= N) return;
    double s[10];
#pragma unroll
    for (int k = 0; k < 10; k++) s[k] = 0.0;
    for (int32_t q = ptr[I]; q < ptr[I + 1]; q++)
#pragma unroll
        for (int k = 0; k < 10; k++) s[k] += cone[(int64_t)q * 10 + k];
    const double V = s[0];
    const double tr = s[4] + s[5] + s[6];
    mass[I] = rho * V;
    vol[I] = V;
    const double iv = V > 0.0 ? 1.0 / V : 0.0;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        rcell[c * N + I] = s[1 + c] * iv;
        Jd[c * N + I] = rho * (tr - s[4 + c]);
    }
    // J6: xx yy zz xy yz xz
    J6[0 * N + I] = rho * (tr - s[4]);
    J6[1 * N + I] = rho * (tr - s[5]);
    J6[2 * N + I] = rho * (tr - s[6]);
    J6[3 * N + I] = -rho * s[7];
    J6[4 * N + I] = -rho * s[8];
    J6[5 * N + I] = -rho * s[9];
}
