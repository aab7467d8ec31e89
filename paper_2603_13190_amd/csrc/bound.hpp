// Element bound of the stable explicit step on the device: for every
// tetrahedron the largest eigenvalue of W K_e W, K_e its elastic stiffness
// (the sum over its 12 facets of (A / l) B^T D B, B = [-1, [c^I]x] at the
// facet's I node and [1, -[c^J]x] at its J node, c^J = c^I - l n,
// D = E0 (alpha 1 + (1 - alpha) n n^T)) and W = diag(share)^(-1/2) from its
// share of the lumped masses of its four nodes.  Included once, by ldpm.hip.
//
// One wave per tetrahedron: the 24 x 24 matrix is assembled in LDS (facet by
// facet, the 144 entries of a facet's block spread over the lanes), scaled,
// and diagonalised by cyclic Jacobi rotations in round-robin order: in round
// r the 24 indices form 12 disjoint pairs, (23, r) and ((r + k) mod 23,
// (r - k) mod 23) for k = 1..11, so the 12 rotations of a round commute and
// are applied together, block by 2 x 2 block of (row pair, column pair) in
// one pass over the matrix; 23 rounds make a sweep, in which every pair occurs
// once.  Sweeps stop when the off-diagonal part is below 1e-12 of the
// matrix's Frobenius norm for all tetrahedra of the block; the diagonal then
// holds the eigenvalues.
#pragma once

constexpr int EB_WAVES = 4;     // tetrahedra per 256-lane block
constexpr int EB_N = 24;        // DoFs per tetrahedron
constexpr int EB_PITCH = 25;    // LDS row pitch
constexpr int EB_SWEEPS = 12;   // cap; convergence is quadratic and usually takes 5 to 7

struct ElemIn {
    const int32_t* __restrict__ tet;    // [4][T]
    const int32_t* __restrict__ fI;     // [F], F = 12 T, tet-major
    const int32_t* __restrict__ fJ;     // [F]
    const double* __restrict__ cI;      // [3][F]
    const double* __restrict__ n;       // [3][F]
    const double* __restrict__ A;       // [F]
    const double* __restrict__ len;     // [F]
    const double* __restrict__ share;   // [T][4][6]
    double E0, alpha;
    int64_t T;
};

// column d of G at one facet end with offset c: d < 3: sg * (-e_d);
// d >= 3: sg * (c x e_{d-3}), i.e. (0, c2, -c1), (-c2, 0, c0), (c1, -c0, 0);
// written with selects so that no register array is indexed at run time
__device__ __forceinline__ void eb_column(int d, double sg, double c0, double c1, double c2, double g[3])
{
    g[0] = d == 0 ? -sg : (d == 4 ? -sg * c2 : (d == 5 ? sg * c1 : 0.0));
    g[1] = d == 1 ? -sg : (d == 3 ? sg * c2 : (d == 5 ? -sg * c0 : 0.0));
    g[2] = d == 2 ? -sg : (d == 3 ? -sg * c1 : (d == 4 ? sg * c0 : 0.0));
}

__global__ __launch_bounds__(256) void k_elem_lambda(ElemIn in, double* __restrict__ lam)
{
    __shared__ double sA[EB_WAVES][EB_N * EB_PITCH];
    __shared__ double sCS[EB_WAVES][12][2];
    __shared__ int sDone[EB_WAVES];
    const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const int64_t t = (int64_t)blockIdx.x * EB_WAVES + w;
    const bool valid = t < in.T;
    const int64_t T = in.T, F = 12 * in.T;
    double* Am = sA[w];
    for (int e = l; e < EB_N * EB_PITCH; e += 64) Am[e] = 0.0;
    int32_t ids[4] = {-1, -1, -1, -1};
    if (valid)
#pragma unroll
        for (int a = 0; a < 4; a++) ids[a] = in.tet[(int64_t)a * T + t];
    __syncthreads();
    // ---- assembly, facet by facet (the entries of one facet are distinct) ----
    for (int k = 0; k < 12; k++) {
        if (valid) {
            const int64_t f = t * 12 + k;
            const int32_t I = in.fI[f], J = in.fJ[f];
            const int aI = I == ids[0] ? 0 : (I == ids[1] ? 1 : (I == ids[2] ? 2 : 3));
            const int aJ = J == ids[0] ? 0 : (J == ids[1] ? 1 : (J == ids[2] ? 2 : 3));
            const double nn[3] = {in.n[f], in.n[F + f], in.n[2 * F + f]};
            const double L = in.len[f];
            const double ci[3] = {in.cI[f], in.cI[F + f], in.cI[2 * F + f]};
            const double cj[3] = {ci[0] - L * nn[0], ci[1] - L * nn[1], ci[2] - L * nn[2]};
            const double wk = in.A[f] / L * in.E0;
            for (int e = l; e < 144; e += 64) {
                const int r = e / 12, c = e % 12;
                const int sr = r / 6, sc = c / 6;
                double gr[3], gc[3];
                // B_I = G(c^I); B_J = -G(c^J): the end's sign multiplies its column
                eb_column(r % 6, sr ? -1.0 : 1.0, sr ? cj[0] : ci[0], sr ? cj[1] : ci[1], sr ? cj[2] : ci[2], gr);
                eb_column(c % 6, sc ? -1.0 : 1.0, sc ? cj[0] : ci[0], sc ? cj[1] : ci[1], sc ? cj[2] : ci[2], gc);
                const double gg = gr[0] * gc[0] + gr[1] * gc[1] + gr[2] * gc[2];
                const double ngr = nn[0] * gr[0] + nn[1] * gr[1] + nn[2] * gr[2];
                const double ngc = nn[0] * gc[0] + nn[1] * gc[1] + nn[2] * gc[2];
                const int row = 6 * (sr ? aJ : aI) + r % 6, col = 6 * (sc ? aJ : aI) + c % 6;
                Am[row * EB_PITCH + col] += wk * (in.alpha * gg + (1.0 - in.alpha) * ngr * ngc);
            }
        }
        __syncthreads();
    }
    // ---- mass scaling W K W ----
    if (valid) {
        const double* sh = in.share + t * 24;
        for (int e = l; e < EB_N * EB_N; e += 64) {
            const int i = e / EB_N, j = e % EB_N;
            Am[i * EB_PITCH + j] = Am[i * EB_PITCH + j] / sqrt(sh[i]) / sqrt(sh[j]);
        }
    }
    __syncthreads();
    // ---- cyclic Jacobi, round-robin pairs; the block stops when every
    //      wave's off-diagonal norm is below 1e-12 of its matrix norm (the
    //      error of the separated largest eigenvalue is quadratic in it) ----
    for (int sweep = 0; sweep < EB_SWEEPS; sweep++) {
        {
            double off = 0.0, all = 0.0;
            for (int e = l; e < EB_N * EB_N; e += 64) {
                const int i = e / EB_N, j = e % EB_N;
                const double v = Am[i * EB_PITCH + j];
                all += v * v;
                if (i != j) off += v * v;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                off += __shfl_xor(off, o);
                all += __shfl_xor(all, o);
            }
            if (l == 0) sDone[w] = off <= 1e-24 * all;
            __syncthreads();
            bool done = true;
#pragma unroll
            for (int k = 0; k < EB_WAVES; k++) done = done && sDone[k];
            __syncthreads();
            if (done) break;
        }
        for (int r = 0; r < 23; r++) {
            if (l < 12) {
                const int p = l == 0 ? 23 : (r + l) % 23, q = l == 0 ? r : (r - l + 23) % 23;
                const double app = Am[p * EB_PITCH + p], aqq = Am[q * EB_PITCH + q], apq = Am[p * EB_PITCH + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double th = (aqq - app) / (2.0 * apq);
                    const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(tt * tt + 1.0);
                    s = tt * c;
                }
                sCS[w][l][0] = c;
                sCS[w][l][1] = s;
            }
            __syncthreads();
            // A <- J^T A J, one 2 x 2 block (row pair k, column pair m) per
            // item: the pairs partition the indices, so every entry belongs
            // to one block; rows are rotated first, then columns
            for (int e = l; e < 144; e += 64) {
                const int k = e / 12, m = e % 12;
                const int p = k == 0 ? 23 : (r + k) % 23, q = k == 0 ? r : (r - k + 23) % 23;
                const int pp = m == 0 ? 23 : (r + m) % 23, qq = m == 0 ? r : (r - m + 23) % 23;
                const double ck = sCS[w][k][0], sk = sCS[w][k][1], cm = sCS[w][m][0], sm = sCS[w][m][1];
                const double b00 = Am[p * EB_PITCH + pp], b01 = Am[p * EB_PITCH + qq];
                const double b10 = Am[q * EB_PITCH + pp], b11 = Am[q * EB_PITCH + qq];
                const double x00 = ck * b00 - sk * b10, x01 = ck * b01 - sk * b11;
                const double x10 = sk * b00 + ck * b10, x11 = sk * b01 + ck * b11;
                Am[p * EB_PITCH + pp] = cm * x00 - sm * x01;
                Am[p * EB_PITCH + qq] = sm * x00 + cm * x01;
                Am[q * EB_PITCH + pp] = cm * x10 - sm * x11;
                Am[q * EB_PITCH + qq] = sm * x10 + cm * x11;
            }
            __syncthreads();
        }
    }
    // ---- the largest diagonal entry ----
    double d = l < EB_N ? Am[l * EB_PITCH + l] : -1.0e300;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
    if (valid && l == 0) lam[t] = d;
}
