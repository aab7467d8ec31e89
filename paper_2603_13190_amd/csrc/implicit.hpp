// Device side of the implicit generalised-alpha / HHT-alpha integrator: per-DoF vector kernels,
// the deterministic gather of tet-node records into particle vectors, the
// particle blocks of the initial elastic stiffness, and the conjugate-gradient
// kernels of the modified-Newton solves.  Vectors are [6][N] doubles.
// Included once, by ldpm.hip, after step_kernels.hpp.
#pragma once

constexpr int IM_THREADS = 256;
constexpr int IM_MAX_BLOCKS = 1024;

// fixed-order block sum of three values (IM_THREADS lanes)
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c)
{
    __shared__ double s[3][IM_THREADS];
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    s[2][threadIdx.x] = c;
    __syncthreads();
    for (int w = IM_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
            s[2][threadIdx.x] += s[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    a = s[0][0];
    b = s[1][0];
    c = s[2][0];
    __syncthreads();
}

// partials [3][G] -> out[0..2] (one block, fixed order)
__global__ __launch_bounds__(IM_THREADS) void k_im_reduce3(const double* __restrict__ part, int G,
                                                           double* __restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < G; i += IM_THREADS) {
        a += part[i];
        b += part[G + i];
        c += part[2 * G + i];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
    }
}

// out[k][I] = sum of the NV-value tet-node records of particle I (CSR
// order, PG lanes per particle, the same summation structure as the step's
// gather)
template <typename R, int NV = 6>
__global__ __launch_bounds__(256) void k_im_gather(const int32_t* __restrict__ ptr, const R* __restrict__ contrib,
                                                   int64_t N, double* __restrict__ out)
{
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t I = gt / PG;
    const int lane = (int)(gt % PG);
    if (I >= N) return;
    double f[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) f[k] = 0.0;
    const int32_t s0 = ptr[I], s1 = ptr[I + 1];
    for (int32_t s = s0 + lane; s < s1; s += PG) {
        const R* c = contrib + (int64_t)s * NV;
#pragma unroll
        for (int k = 0; k < NV; k++) f[k] += (double)c[k];
    }
#pragma unroll
    for (int off = PG / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < NV; k++) f[k] += __shfl_xor(f[k], off, PG);
    }
#pragma unroll
    for (int k = 0; k < NV; k++)
        if (k % PG == lane) out[(int64_t)k * N + I] = f[k];
}

// The 6 x 6 block of the initial elastic stiffness that couples a particle's
// DoFs with themselves, per tet node (t, a) in incidence order: for every
// facet of tet t at node a, (A / l) G^T D G with G = [-1, [c]x] (c = c^I at
// the facet's I node, c^J = c^I - l n at its J node, where B_J = -G and the
// sign cancels) and D = E0 (alpha 1 + (1 - alpha) n n^T).  21 values: the
// upper triangle row by row, DoFs (u_x, u_y, u_z, th_x, th_y, th_z).
template <typename R>
__global__ __launch_bounds__(256) void k_im_block_k0(const FacetArgs<R> fa, const int32_t* __restrict__ pos, int64_t T,
                                                     double E0, double alpha, double* __restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= 4 * T) return;
    const int64_t t = s >> 2;
    const int a = (int)(s & 3);
    const int64_t F = fa.F;
    double K[21];
#pragma unroll
    for (int p = 0; p < 21; p++) K[p] = 0.0;
    for (int k = 0; k < 12; k++) {
        const int64_t f = t * 12 + k;
        const int32_t rc = fa.rec[f];
        const int aI = (rc >> 28) & 3, aJ = (rc >> 30) & 3;
        if (aI != a && aJ != a) continue;
        const R* fr = fa.frame + (int64_t)(rc & 0x0fffffff) * 8;
        const double n[3] = {(double)fr[0], (double)fr[1], (double)fr[2]};
        const double len = (double)fr[6];
        double c[3];
#pragma unroll
        for (int i = 0; i < 3; i++) c[i] = (double)fa.geo[quad_index<R>(F, f, i)];
        if (aJ == a)
#pragma unroll
            for (int i = 0; i < 3; i++) c[i] -= len * n[i];
        const double w = (double)fa.geo[quad_index<R>(F, f, 3)] / len * E0;
        // columns of G: -e_j for the translations, c x e_j for the rotations
        double g[6][3];
#pragma unroll
        for (int j = 0; j < 3; j++) {
#pragma unroll
            for (int i = 0; i < 3; i++) g[j][i] = i == j ? -1.0 : 0.0;
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            g[3 + j][j] = 0.0;
            g[3 + j][j1] = c[j2];   // (c x e_j)_{j+1} = c_{j+2}
            g[3 + j][j2] = -c[j1];  // (c x e_j)_{j+2} = -c_{j+1}
        }
        double ng[6];
#pragma unroll
        for (int j = 0; j < 6; j++) ng[j] = n[0] * g[j][0] + n[1] * g[j][1] + n[2] * g[j][2];
        int p = 0;
#pragma unroll
        for (int i = 0; i < 6; i++)
#pragma unroll
            for (int j = i; j < 6; j++) {
                const double gg = g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2];
                K[p++] += w * (alpha * gg + (1.0 - alpha) * ng[i] * ng[j]);
            }
    }
    const int64_t o = (int64_t)pos[s] * 21;
#pragma unroll
    for (int p = 0; p < 21; p++) out[o + p] = K[p];
}

// applied generalised forces of the free DoFs at `time` (zero on prescribed
// DoFs), and prescribed velocities at `time_mid` (zero on free DoFs)
__global__ __launch_bounds__(256) void k_im_loads(const uint8_t* __restrict__ mode, const int32_t* __restrict__ prog,
                                                  const double* __restrict__ scale, const double* __restrict__ body,
                                                  ProgArgs pr, double time, double time_mid, int64_t n6,
                                                  double* __restrict__ f, double* __restrict__ vp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n6) return;
    const int32_t pg = prog[i];
    if (mode[i] == 0) {
        double a = body ? body[i] : 0.0;
        if (pg >= 0) a += scale[i] * prog_at(pr, pg, time);
        f[i] = a;
        if (vp) vp[i] = 0.0;
    } else {
        f[i] = 0.0;
        if (vp) vp[i] = pg >= 0 ? scale[i] * prog_at(pr, pg, time_mid) : 0.0;
    }
}

// node records of a trial configuration: q slot = q, v slot = q - q_n (the
// facet kernel, launched with dt = 1, then takes e(q) - e(q_n) as the strain
// increment from the committed history)
__global__ __launch_bounds__(256) void k_im_nodes(double* __restrict__ node, const double* __restrict__ q,
                                                  const double* __restrict__ qn, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * N) return;
    const int64_t c = i / N, p = i - c * N;
    node[p * 16 + c] = q[i];
    node[p * 16 + 6 + c] = qn ? q[i] - qn[i] : 0.0;
}

// predictor: q = q_n + dt v_n + dt^2/2 a_n on free DoFs, q_n + dt v_P(t + dt/2)
// on prescribed ones
__global__ __launch_bounds__(256) void k_im_predict(const uint8_t* __restrict__ mode, const double* __restrict__ qn,
                                                    const double* __restrict__ vn, const double* __restrict__ an,
                                                    const double* __restrict__ vp, double dt, int64_t n6,
                                                    double* __restrict__ q)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n6) return;
    q[i] = mode[i] == 0 ? qn[i] + dt * vn[i] + 0.5 * dt * dt * an[i] : qn[i] + dt * vp[i];
}

// generalised-alpha parameters: am = alpha_m, af = alpha_f (HHT: am = 0,
// af = -alpha)
struct ImArgs {
    const uint8_t* __restrict__ mode;
    const double* __restrict__ M;      // [6][N] lumped diagonal
    const double *qn, *vn, *an, *gn, *fn, *f1;
    double dt, am, af, beta, gamma;
    int64_t N;
};

// a = (q - q_n - dt v_n - dt^2 (1/2 - beta) a_n) / (beta dt^2),
// rhs = (1 - af)(g + f1) + af (g_n + f_n) - am M a_n,
// R = rhs - (1 - am) M a on free DoFs;
// block partials of |R_F|^2, |((1 - am) M a)_F|^2, |rhs_F|^2
__global__ __launch_bounds__(IM_THREADS) void k_im_residual(ImArgs ia, const double* __restrict__ q,
                                                            const double* __restrict__ g, double* __restrict__ Rv,
                                                            double* __restrict__ part)
{
    double rr = 0.0, mm = 0.0, hh = 0.0;
    const int64_t n6 = 6 * ia.N;
    const int64_t stride = (int64_t)gridDim.x * IM_THREADS;
    const double bdt2 = ia.beta * ia.dt * ia.dt;
    for (int64_t i = (int64_t)blockIdx.x * IM_THREADS + threadIdx.x; i < n6; i += stride) {
        const double base = ia.qn[i] + ia.dt * ia.vn[i] + ia.dt * ia.dt * (0.5 - ia.beta) * ia.an[i];
        const double a = (q[i] - base) / bdt2;
        const double rhs =
            (1.0 - ia.af) * (g[i] + ia.f1[i]) + ia.af * (ia.gn[i] + ia.fn[i]) - ia.am * ia.M[i] * ia.an[i];
        const double ma = (1.0 - ia.am) * ia.M[i] * a;
        double r = 0.0;
        if (ia.mode[i] == 0) {
            r = rhs - ma;
            rr += r * r;
            mm += ma * ma;
            hh += rhs * rhs;
        }
        Rv[i] = r;
    }
    block_sum3(rr, mm, hh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rr;
        part[gridDim.x + blockIdx.x] = mm;
        part[2 * gridDim.x + blockIdx.x] = hh;
    }
}

// accept the step: a, v, reactions on prescribed DoFs, external work
// (trapezoid of applied + reaction forces over q - q_n, per particle in DoF
// order), kinetic energy, and the new committed vectors
__global__ __launch_bounds__(256) void k_im_accept(ImArgs ia, const double* __restrict__ q,
                                                   const double* __restrict__ g, double* __restrict__ fext,
                                                   double* __restrict__ wext, double* __restrict__ wkin,
                                                   double* __restrict__ node, double* __restrict__ qn_o,
                                                   double* __restrict__ vn_o, double* __restrict__ an_o,
                                                   double* __restrict__ gn_o, double* __restrict__ fn_o,
                                                   int32_t* __restrict__ flag)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = ia.N;
    if (I >= N) return;
    const double bdt2 = ia.beta * ia.dt * ia.dt;
    double dwe = 0.0, wk = 0.0;
    bool bad = false;
    for (int d = 0; d < 6; d++) {
        const int64_t i = d * N + I;
        const double qq = q[i];
        const double base = ia.qn[i] + ia.dt * ia.vn[i] + ia.dt * ia.dt * (0.5 - ia.beta) * ia.an[i];
        const double a = (qq - base) / bdt2;
        const double v = ia.vn[i] + ia.dt * ((1.0 - ia.gamma) * ia.an[i] + ia.gamma * a);
        const double rhs =
            (1.0 - ia.af) * (g[i] + ia.f1[i]) + ia.af * (ia.gn[i] + ia.fn[i]) - ia.am * ia.M[i] * ia.an[i];
        const double ma = (1.0 - ia.am) * ia.M[i] * a;
        const double Ft = ia.mode[i] == 0 ? ia.f1[i] : ma - rhs;
        dwe += 0.5 * (fext[i] + Ft) * (qq - ia.qn[i]);
        wk += 0.5 * ia.M[i] * v * v;
        fext[i] = Ft;
        node[I * 16 + d] = qq;
        node[I * 16 + 6 + d] = v;
        qn_o[i] = qq;
        vn_o[i] = v;
        an_o[i] = a;
        gn_o[i] = g[i];
        fn_o[i] = ia.f1[i];
        bad = bad || !isfinite(v);
    }
    wext[I] += dwe;
    wkin[I] = wk;
    if (bad) flag[0] = 1;
}

// q += x on free DoFs
__global__ __launch_bounds__(256) void k_im_add(const uint8_t* __restrict__ mode, const double* __restrict__ x,
                                                int64_t n6, double* __restrict__ q)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n6 && mode[i] == 0) q[i] += x[i];
}

// ---------------------------------------------------------------------------
// conjugate gradients on K_eff = cM M + cK K0 over the free DoFs with a
// block-Jacobi preconditioner (the inverse 6 x 6 particle blocks of K_eff);
// K0 p = -gather(facet kernel of the elastic law at p)
// scalars: sc[0] = r.z, sc[1] = alpha_cg, sc[2] = beta_cg, sc[3] = r.r,
// sc[4] = r.r of the right-hand side, sc[8 + parity] = r.z
// ---------------------------------------------------------------------------
struct CgArgs {
    const uint8_t* __restrict__ mode;
    const double* __restrict__ M;
    const double* __restrict__ binv;  // [36][N] inverse particle blocks of K_eff (zero on prescribed DoFs)
    double *x, *r, *z, *p, *Ap, *sc, *part;
    double cM, cK;
    int64_t N;
};

// z = B^-1 r for one particle (B its block of K_eff; rows of prescribed DoFs
// are zero, so z vanishes there)
__device__ __forceinline__ void block_precond(const double* __restrict__ binv, int64_t N, int64_t I,
                                              const double r[6], double z[6])
{
#pragma unroll
    for (int i = 0; i < 6; i++) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < 6; j++) v += binv[(int64_t)(6 * i + j) * N + I] * r[j];
        z[i] = v;
    }
}

// x = 0, r = R, z = B^-1 r, p = z; node_p slots = p; partials r.z, r.r
// (one thread per particle, grid-stride)
__global__ __launch_bounds__(IM_THREADS) void k_cg_init(CgArgs cg, const double* __restrict__ R,
                                                        double* __restrict__ node_p)
{
    double rz = 0.0, rr = 0.0, zz = 0.0;
    const int64_t N = cg.N;
    const int64_t stride = (int64_t)gridDim.x * IM_THREADS;
    for (int64_t I = (int64_t)blockIdx.x * IM_THREADS + threadIdx.x; I < N; I += stride) {
        double r[6], z[6];
#pragma unroll
        for (int c = 0; c < 6; c++) r[c] = cg.mode[c * N + I] == 0 ? R[c * N + I] : 0.0;
        block_precond(cg.binv, N, I, r, z);
#pragma unroll
        for (int c = 0; c < 6; c++) {
            const int64_t i = c * N + I;
            cg.x[i] = 0.0;
            cg.r[i] = r[c];
            cg.z[i] = z[c];
            cg.p[i] = z[c];
            node_p[I * 16 + c] = z[c];
            rz += r[c] * z[c];
            rr += r[c] * r[c];
        }
    }
    block_sum3(rz, rr, zz);
    if (threadIdx.x == 0) {
        cg.part[blockIdx.x] = rz;
        cg.part[gridDim.x + blockIdx.x] = rr;
        cg.part[2 * gridDim.x + blockIdx.x] = 0.0;
    }
}

// sc[2] = rz_new / sc[0]; sc[0] = rz_new; sc[3] = r.r  (first: only store);
// used after k_cg_init
__global__ __launch_bounds__(IM_THREADS) void k_cg_beta(CgArgs cg, int G, int first)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < G; i += IM_THREADS) {
        a += cg.part[i];
        b += cg.part[G + i];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) {
        cg.sc[2] = (!first && cg.sc[0] != 0.0) ? a / cg.sc[0] : 0.0;
        cg.sc[0] = a;
        cg.sc[3] = b;
        if (first) {
            cg.sc[4] = b;  // r.r of the right-hand side
            cg.sc[8] = a;  // r.z in the parity-0 slot the first update reads
        }
    }
}

// One CG iteration is four kernels: the elastic facet kernel at p, then
//   k_cg_gather_apply  y = -K0 p per particle, Ap = cM M p - cK y, partials of p.Ap;
//   k_cg_update        alpha from the p.Ap partials, x += alpha p,
//                      r -= alpha Ap, z = B^-1 r (particle blocks), partials
//                      of r.z and r.r;
//   k_cg_newp          beta from the r.z partials, p = z + beta p.
// Every block reduces the previous kernel's partials itself, in the same
// fixed order, so all blocks hold the same scalar and no reduction kernel
// runs in between.  r.z alternates between sc[8] and sc[9] (par = iteration
// parity), so that the block that stores the new value never overwrites the
// one the other blocks are still reading.  partA has IM_MAX_BLOCKS slots,
// partB 2 x IM_MAX_BLOCKS (r.z, then r.r).

// the gather of k_im_gather (PG lanes per particle, same summation order),
// over particle groups grid-stride, then the operator on the group's 6 DoFs
template <typename R>
__global__ __launch_bounds__(256) void k_cg_gather_apply(CgArgs cg, const int32_t* __restrict__ ptr,
                                                         const R* __restrict__ contrib, double* __restrict__ partA)
{
    const int64_t N = cg.N;
    constexpr int GROUPS = 256 / PG;
    const int lane = (int)(threadIdx.x % PG);
    double pap = 0.0, u0 = 0.0, u1 = 0.0;
    for (int64_t I0 = (int64_t)blockIdx.x * GROUPS; I0 < N; I0 += (int64_t)gridDim.x * GROUPS) {
        const int64_t I = I0 + threadIdx.x / PG;
        double f[6] = {0, 0, 0, 0, 0, 0};
        if (I < N) {
            const int32_t s0 = ptr[I], s1 = ptr[I + 1];
            for (int32_t q = s0 + lane; q < s1; q += PG) {
                const R* c = contrib + (int64_t)q * 6;
#pragma unroll
                for (int k = 0; k < 6; k++) f[k] += (double)c[k];
            }
        }
#pragma unroll
        for (int off = PG / 2; off > 0; off >>= 1) {
#pragma unroll
            for (int k = 0; k < 6; k++) f[k] += __shfl_xor(f[k], off, PG);
        }
        if (I < N && lane < 6) {
            double y = f[0];
#pragma unroll
            for (int k = 1; k < 6; k++) y = (lane == k) ? f[k] : y;
            const int64_t i = (int64_t)lane * N + I;
            const double ap = cg.mode[i] == 0 ? cg.cM * cg.M[i] * cg.p[i] - cg.cK * y : 0.0;
            cg.Ap[i] = ap;
            pap += cg.p[i] * ap;
        }
    }
    block_sum3(pap, u0, u1);
    if (threadIdx.x == 0) partA[blockIdx.x] = pap;
}

// alpha = r.z / p.Ap; x += alpha p, r -= alpha Ap, z = B^-1 r; partials r.z, r.r.
// 8 lanes per particle: lane c < 6 updates DoF c and gets the particle's
// other new residuals by shuffles (no lane reads what another one writes).
constexpr int CG_LANES = 8;

__global__ __launch_bounds__(IM_THREADS) void k_cg_update(CgArgs cg, const double* __restrict__ partA, int GA,
                                                          double* __restrict__ partB, int par)
{
    double pap = 0.0, u0 = 0.0, u1 = 0.0;
    for (int i = threadIdx.x; i < GA; i += IM_THREADS) pap += partA[i];
    block_sum3(pap, u0, u1);
    const double al = pap != 0.0 ? cg.sc[8 + par] / pap : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) cg.sc[1] = al;
    double rz = 0.0, rr = 0.0, u = 0.0;
    const int64_t N = cg.N;
    constexpr int PER_BLOCK = IM_THREADS / CG_LANES;
    const int c = (int)(threadIdx.x % CG_LANES);
    const int base = (int)(threadIdx.x & 63) & ~(CG_LANES - 1);
    for (int64_t I0 = (int64_t)blockIdx.x * PER_BLOCK; I0 < N; I0 += (int64_t)gridDim.x * PER_BLOCK) {
        const int64_t I = I0 + threadIdx.x / CG_LANES;
        const bool act = I < N && c < 6;
        const int64_t i = (int64_t)c * N + I;
        double r = 0.0;
        if (act) {
            r = cg.r[i];  // zero on prescribed DoFs since k_cg_init
            if (cg.mode[i] == 0) {
                cg.x[i] += al * cg.p[i];
                r -= al * cg.Ap[i];
            }
        }
        double z = 0.0;
#pragma unroll
        for (int j = 0; j < 6; j++) {
            const double rj = __shfl(r, base + j);
            if (act) z += cg.binv[(int64_t)(6 * c + j) * N + I] * rj;
        }
        if (act) {
            cg.r[i] = r;
            cg.z[i] = z;
            rz += r * z;
            rr += r * r;
        }
    }
    block_sum3(rz, rr, u);
    if (threadIdx.x == 0) {
        partB[blockIdx.x] = rz;
        partB[IM_MAX_BLOCKS + blockIdx.x] = rr;
    }
}

// sc[3] = r.r from the update's partials (one block; the host's stopping test)
__global__ __launch_bounds__(IM_THREADS) void k_cg_rr(CgArgs cg, const double* __restrict__ partB, int G)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < G; i += IM_THREADS) {
        a += partB[i];
        b += partB[IM_MAX_BLOCKS + i];
    }
    block_sum3(a, b, c);
    if (threadIdx.x == 0) cg.sc[3] = b;
}

// beta = r.z_new / r.z_old; p = z + beta p (free DoFs), written also to the
// q slots of node_p; block 0 stores r.z_new in the other parity slot
__global__ __launch_bounds__(IM_THREADS) void k_cg_newp(CgArgs cg, const double* __restrict__ partB, int G,
                                                        double* __restrict__ node_p, int par)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < G; i += IM_THREADS) {
        a += partB[i];
        b += partB[IM_MAX_BLOCKS + i];
    }
    block_sum3(a, b, c);
    const double rz_old = cg.sc[8 + par];
    const double be = rz_old != 0.0 ? a / rz_old : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cg.sc[8 + (par ^ 1)] = a;
        cg.sc[0] = a;
        cg.sc[2] = be;
        cg.sc[3] = b;
    }
    const int64_t n6 = 6 * cg.N;
    const int64_t stride = (int64_t)gridDim.x * IM_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * IM_THREADS + threadIdx.x; i < n6; i += stride) {
        const double p = cg.mode[i] == 0 ? cg.z[i] + be * cg.p[i] : 0.0;
        cg.p[i] = p;
        const int64_t cc = i / cg.N, pI = i - cc * cg.N;
        node_p[pI * 16 + cc] = p;
    }
}

// q_n, v_n from the node records
__global__ __launch_bounds__(256) void k_im_unpack(const double* __restrict__ node, int64_t N, double* __restrict__ q,
                                                   double* __restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * N) return;
    const int64_t c = i / N, p = i - c * N;
    q[i] = node[p * 16 + c];
    v[i] = node[p * 16 + 6 + c];
}

// node records <- q, v
__global__ __launch_bounds__(256) void k_im_pack(double* __restrict__ node, const double* __restrict__ q,
                                                 const double* __restrict__ v, int64_t N)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * N) return;
    const int64_t c = i / N, p = i - c * N;
    node[p * 16 + c] = q[i];
    node[p * 16 + 6 + c] = v[i];
}

// Inverse of each particle's 6 x 6 block of K_eff = cM M + cK K0 on its free
// DoFs (rows and columns of prescribed DoFs replaced by the identity, and
// zero in the result), by Cholesky; binv[(6 i + j) N + I].  A block that is
// not positive definite (not expected: K_eff is SPD on the free DoFs) falls
// back to its inverse diagonal.
__global__ __launch_bounds__(256) void k_im_block_inv(const double* __restrict__ M, const uint8_t* __restrict__ mode,
                                                      const double* __restrict__ blk, double cM, double cK,
                                                      int64_t N, double* __restrict__ binv)
{
    const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= N) return;
    bool fr[6];
#pragma unroll
    for (int i = 0; i < 6; i++) fr[i] = mode[i * N + I] == 0;
    double A[6][6];
    int p = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i; j < 6; j++) {
            double v = cK * blk[(int64_t)p * N + I];
            if (i == j) v += cM * M[i * N + I];
            if (!fr[i] || !fr[j]) v = i == j ? 1.0 : 0.0;
            A[i][j] = v;
            A[j][i] = v;
            p++;
        }
    // A = L L^T, L in the lower triangle of A
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; k++) d -= A[j][k] * A[j][k];
        ok = ok && d > 0.0;
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        A[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            double v = A[i][j];
#pragma unroll
            for (int k = 0; k < j; k++) v -= A[i][k] * A[j][k];
            A[i][j] = v / ljj;
        }
    }
    // columns of the inverse: L y = e_c, L^T x = y
#pragma unroll
    for (int c = 0; c < 6; c++) {
        double y[6], x[6];
#pragma unroll
        for (int i = 0; i < 6; i++) {
            double v = i == c ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; k++) v -= A[i][k] * y[k];
            y[i] = v / A[i][i];
        }
#pragma unroll
        for (int i = 5; i >= 0; i--) {
            double v = y[i];
#pragma unroll
            for (int k = i + 1; k < 6; k++) v -= A[k][i] * x[k];
            x[i] = v / A[i][i];
        }
#pragma unroll
        for (int i = 0; i < 6; i++) {
            double v = x[i];
            if (!ok) {
                const double dg = i == c ? cK * blk[(int64_t)(i * 6 - i * (i - 1) / 2) * N + I] + cM * M[i * N + I]
                                         : 0.0;
                v = (i == c && dg > 0.0) ? 1.0 / dg : 0.0;
            }
            binv[(int64_t)(6 * i + c) * N + I] = (fr[i] && fr[c]) ? v : 0.0;
        }
    }
}

// a_0 = (g_0 + f_0) / M on free DoFs, 0 on prescribed ones; g_n = g_0;
// fext = f_0 on free DoFs, 0 on prescribed ones
__global__ __launch_bounds__(256) void k_im_init_acc(ImArgs ia, const double* __restrict__ g, double* __restrict__ an,
                                                     double* __restrict__ gn, double* __restrict__ fext)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 6 * ia.N) return;
    const bool fr = ia.mode[i] == 0;
    an[i] = fr ? (g[i] + ia.fn[i]) / ia.M[i] : 0.0;
    gn[i] = g[i];
    fext[i] = fr ? ia.fn[i] : 0.0;
}
