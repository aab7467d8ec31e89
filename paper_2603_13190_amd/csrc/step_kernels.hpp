// Device side of the explicit LDPM step: argument blocks, the facet kernel
// (strains, law, forces, per-tet-node sums), the particle kernel (gather and
// leapfrog update), the persistent multi-step kernel and the deterministic
// reductions.  Included once, by ldpm.hip, after `using namespace ldpm`.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "law.hpp"
#include "mlp.hpp"

// ---------------------------------------------------------------------------
// device argument blocks
// ---------------------------------------------------------------------------
// Four values of a facet in 16-byte chunks: [QC][F][QK], QK = 16 / sizeof(R)
// values per chunk and QC = 4 / QK chunks, so that one lane moves a facet's
// record with one (FP32) or two (FP64) 16-byte accesses.
template <typename R>
constexpr int QK = 16 / (int)sizeof(R);
template <typename R>
__host__ __device__ __forceinline__ int64_t quad_index(int64_t F, int64_t f, int j)
{
    return ((int64_t)(j / QK<R>) * F + f) * QK<R> + j % QK<R>;
}

template <typename R>
struct FacetArgs {
    const R* __restrict__ geo;     // quads c^I[3], area
    const int32_t* __restrict__ rec;  // [F]
    const R* __restrict__ frame;   // [E][8]: n[3], m[3], len, 1/len
    R* __restrict__ hist;          // quads t_N, t_M, t_L, e_max
    int64_t F, E;
};

struct NodeArgs {
    const int32_t* __restrict__ tet;  // [4][T]
    const double* __restrict__ node;  // [N][16]: q[6], v[6], x0[3], pad
    int64_t N, T;
};

// Piecewise-linear time programs (constant beyond their end points).  The
// facet kernel's first block evaluates every program at t_n and t_{n+1/2}
// into progv[2p], progv[2p+1]; the particle kernel of the same step reads them.
struct ProgArgs {
    const int64_t* __restrict__ off;  // [P+1]
    const double* __restrict__ t;
    const double* __restrict__ v;
    double* __restrict__ val;         // [2P]
    int64_t P;
};

__device__ __forceinline__ double prog_at(const ProgArgs& pr, int64_t p, double time)
{
    const int64_t a = pr.off[p], b = pr.off[p + 1];
    if (b <= a) return 0.0;
    if (time <= pr.t[a]) return pr.v[a];
    for (int64_t i = a; i + 1 < b; i++) {
        const double t1 = pr.t[i + 1];
        if (time <= t1) {
            const double t0 = pr.t[i];
            const double w = (time - t0) / (t1 - t0);
            return pr.v[i] + w * (pr.v[i + 1] - pr.v[i]);
        }
    }
    return pr.v[b - 1];
}

// Facet-kernel modes: plain step, plain step that also records surrogate
// training samples, step with the MLP surrogate in place of the law.
enum { MODE_PLAIN = 0, MODE_CAPTURE = 1, MODE_SURROGATE = 2 };

struct GateArgs {
    float kappa_t, kappa_c, damage_max;
};

struct SurrogateArgs {
    const float* __restrict__ params;  // [MLP_NPARAM] FP32
    uint8_t* __restrict__ flag;        // [F] sticky: 1 = handed back to the exact law
    // running counts of facet-updates: [0] by the network, [1] with damage
    // in (SG_DAMAGED, damage_max] whichever law produced them, [2] those of
    // [1] made by the network; facets handed back [3] by the strain
    // envelope, [4] by the feature box, [5] by the damage gate
    unsigned long long* __restrict__ stats;
    float xmean[MLP_IN], xscale[MLP_IN], yscale[MLP_OUT], ydead[MLP_OUT], lo[MLP_IN], hi[MLP_IN];
    float ytau;
    GateArgs gate;
};

// a facet-update counts as damaged above this damage (below it D is the
// rounding of an elastic update)
constexpr float SG_DAMAGED = 1e-3f;
constexpr int SG_NSTATS = 6;

struct CaptureArgs {
    float* __restrict__ rows;          // [cap][16]: x[9], residual[3], key (int64 bits)
    unsigned* __restrict__ count;
    int64_t cap;
    int32_t fstride, foff, sstride;
    GateArgs gate;
};

struct ParticleArgs {
    double* __restrict__ node;        // [N][16]: q[6], v[6], x0[3], pad
    const double* __restrict__ mass;  // [N]
    const double* __restrict__ inertia;  // [3][N]
    const uint8_t* __restrict__ mode;    // [6][N]
    const int32_t* __restrict__ prog;    // [6][N]
    const double* __restrict__ scale;    // [6][N]
    const double* __restrict__ body;     // [6][N] or nullptr
    double* __restrict__ fext;           // [6][N]
    double* __restrict__ wext;           // [N]
    double* __restrict__ wkin;           // [N]
    const int32_t* __restrict__ ptr;     // [N+1]
    const double* __restrict__ progv;    // [2P] program values of this step
    int32_t* __restrict__ flag;
    int64_t N;
    // full cell mass blocks, [N][72]: M (6 x 6 rows) then G (6 x 6 rows),
    // G = inverse of M over the free DoFs, zero rows/columns for prescribed
    // ones; nullptr with the lumped diagonal
    const double* __restrict__ mblk;
};

// ---------------------------------------------------------------------------
// facet kernel
// ---------------------------------------------------------------------------
// Facet records and the traction history are touched once per step, in facet
// order.  On systems larger than the last-level cache they are loaded and
// stored nontemporally (NT = 1), so that they do not evict what the step
// reuses (node records and edge frames, gathered by every tet around them,
// and the tet-node sums the particle kernel reads); on smaller ones plain
// accesses (NT = 0) let the whole step stay cache-resident across steps.
// NT is a template parameter: a run-time choice between the two forms of
// one load is merged by the compiler into a plain load.
template <typename T>
__device__ __forceinline__ T ld_once(const T* p)
{
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_once(T v, T* p)
{
    __builtin_nontemporal_store(v, p);
}

typedef double quad_d2 __attribute__((ext_vector_type(2)));
typedef float quad_f4 __attribute__((ext_vector_type(4)));

template <int NT, typename T>
__device__ __forceinline__ T ld_facet(const T* p)
{
    if constexpr (NT) return ld_once(p);
    else return *p;
}
template <int NT, typename T>
__device__ __forceinline__ void st_facet(T v, T* p)
{
    if constexpr (NT) st_once(v, p);
    else *p = v;
}

// the four values of facet f (quad layout)
template <int NT, typename R>
__device__ __forceinline__ void ld_quad(const R* base, int64_t F, int64_t f, R& a, R& b, R& c, R& e)
{
    if constexpr (sizeof(R) == 8) {
        const quad_d2 x = ld_facet<NT>((const quad_d2*)base + f), y = ld_facet<NT>((const quad_d2*)base + F + f);
        a = x.x; b = x.y; c = y.x; e = y.y;
    } else {
        const quad_f4 x = ld_facet<NT>((const quad_f4*)base + f);
        a = x.x; b = x.y; c = x.z; e = x.w;
    }
}
template <int NT, typename R>
__device__ __forceinline__ void st_quad(R* base, int64_t F, int64_t f, R a, R b, R c, R e)
{
    if constexpr (sizeof(R) == 8) {
        st_facet<NT>(quad_d2{a, b}, (quad_d2*)base + f);
        st_facet<NT>(quad_d2{c, e}, (quad_d2*)base + F + f);
    } else {
        st_facet<NT>(quad_f4{a, b, c, e}, (quad_f4*)base + f);
    }
}

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb, int remap)
{
    // Blocks are dispatched round-robin over the 8 XCDs (each with its own
    // L2); give every XCD a contiguous range of tet blocks instead, so that
    // neighbouring tets (which share nodes and edge frames) share an L2.
    if (!remap) return b;
    const int64_t x = b & 7, k = b >> 3;
    const int64_t qn = nb >> 3, r = nb & 7;
    return x * qn + (x < r ? x : r) + k;
}

// Is the facet inside the surrogate's envelope (the regime the network is
// trained on)?  Tension: the effective strain and e_max stay below kappa_t
// of the elastic limit e0(omega) at the current angle (kappa_t > 1 reaches
// past the peak into softening, where the damage gate hands the facet back);
// compression: -e_DV and -t_N stay below kappa_c of the onset of pore
// collapse (e_c0, sigma_c0).
template <typename R>
__device__ __forceinline__ bool in_envelope(const MatDev<R>& p, const R e[3], R eV, const R told[3], R emax,
                                            const GateArgs& g)
{
    if (e[0] > R(0)) {
        R sN, sT2, seff, seff2;
        int ex;
        scaled_norm(e[0], e[1], e[2], p.alpha, sN, sT2, seff, seff2, ex);
        const R eff = d_ldexp(seff, ex);
        const R inv = R(1) / seff;
        const R sn = sN * inv, cs2 = p.alpha * sT2 * (inv * inv);
        const R sigma0 = R(2) * p.sigma_t / (sn + d_sqrt(sn * sn + p.c4 * cs2));
        const R lim = (R)g.kappa_t * sigma0 * p.inv_E0;
        return eff < lim && emax < lim;
    }
    const R eD = e[0] - eV;
    const R eDV = eV + p.beta * eD;
    return (-eDV < (R)g.kappa_c * p.ec0) && (-told[0] < (R)g.kappa_c * p.sigma_c0);
}

// damage D = 1 - t/(E0 e) of a tensile facet; 0 in compression and while
// the effective strain is below 1 % of sigma_t/E0, where the ratio is a
// ratio of rounding errors (e.g. ahead of a stress wave) and the facet is
// far from any damage
template <typename R>
__device__ __forceinline__ float facet_damage(const MatDev<R>& p, const R e[3], const R t[3])
{
    if (!(e[0] > R(0))) return 0.f;
    R sN, sT2, seff, seff2;
    int ex;
    scaled_norm(e[0], e[1], e[2], p.alpha, sN, sT2, seff, seff2, ex);
    const R eff = d_ldexp(seff, ex);
    if (eff < R(0.01) * p.sigma_t * p.inv_E0) return 0.f;
    const R teff = d_sqrt(t[0] * t[0] + (t[1] * t[1] + t[2] * t[2]) * p.inv_alpha);
    return (float)(R(1) - teff / (p.E0 * eff));
}

// |t_old + E de|: magnitude of the elastic trial traction, the scale of a
// facet's surrogate residual
template <typename R>
__device__ __forceinline__ float trial_norm(const MatDev<R>& p, const R told[3], const R de[3])
{
    const R a = told[0] + p.E0 * de[0], b = told[1] + p.aE0 * de[1], c = told[2] + p.aE0 * de[2];
    return (float)d_sqrt(a * a + b * b + c * c);
}

// surrogate features (aligned with the trial shear traction) of a facet
template <typename R>
__device__ __forceinline__ AlignedFrame surrogate_features(const MatDev<R>& p, const R e[3], const R de[3],
                                                           const R told[3], float x[MLP_IN])
{
    const AlignedFrame fr =
        shear_frame((float)(told[1] + p.aE0 * de[1]), (float)(told[2] + p.aE0 * de[2]));
    x[0] = (float)de[0];
    to_frame(fr, (float)de[1], (float)de[2], x[1], x[2]);
    x[3] = (float)(e[0] - de[0]);
    to_frame(fr, (float)(e[1] - de[1]), (float)(e[2] - de[2]), x[4], x[5]);
    x[6] = (float)told[0];
    to_frame(fr, (float)told[1], (float)told[2], x[7], x[8]);
    return fr;
}

// LDS of the surrogate: the block's copy of the network's weights
__device__ __forceinline__ MlpFrag& mlp_smem()
{
    __shared__ MlpFrag sm;
    return sm;
}

// per-lane counts of the surrogate's facet-updates (SurrogateArgs::stats)
struct SgCount {
    unsigned nn = 0, dmg = 0, dmg_nn = 0;
    // facets handed back by the strain envelope, by the trained feature box
    // (inside the envelope), by the damage gate
    unsigned out_env = 0, out_box = 0, out_dmg = 0;
};

// One tile of TB tetrahedra (block-wide: every thread of a 12 TB block calls
// it together).  do_prog: this block also evaluates the time programs.
// cnt (surrogate mode): the lane's running counts.
template <typename R, int LAW, int TB, int MODE, int NT = 0>
__device__ __forceinline__ void facet_tile(int64_t blk, bool do_prog, const NodeArgs& na, const FacetArgs<R>& fa,
                                           const MatDev<R>& mat, const int32_t* __restrict__ pos,
                                           R* __restrict__ contrib, double* __restrict__ wint,
                                           const ProgArgs& pr, int64_t step, double dt,
                                           const SurrogateArgs& sg, const CaptureArgs& cp, SgCount* cnt = nullptr)
{
    const int first = step == 0;
    constexpr int NS = 4 * TB;   // node slots per block
    constexpr int NF = 12 * TB;  // facets per block
    __shared__ double s_x[3][NS];
    __shared__ double s_q[6][NS];
    __shared__ double s_v[6][NS];
    __shared__ double s_ev[NS];
    __shared__ R s_F[3][NF];
    __shared__ R s_MI[3][NF];
    __shared__ R s_MJ[3][NF];
    __shared__ double s_w[NF];
    __shared__ __align__(4) uint8_t s_code[NF];

    const int tid = threadIdx.x;
    const int64_t tet0 = blk * TB;
    const int64_t T = na.T, N = na.N;

    // ---- facet data for lane tid, issued before the node gather so that
    //      both latencies overlap ----
    const int ftl = tid / 12;
    const bool fvalid = (tid < NF) && (tet0 + ftl < T);
    const int64_t f = (tet0 + ftl) * 12 + (tid % 12);
    int32_t rc = 0;
    R n0 = 0, n1 = 0, n2 = 0, m0 = 0, m1 = 0, m2 = 0, len = 1, ilen = 1, cI0 = 0, cI1 = 0, cI2 = 0, A = 0;
    R tv[3] = {R(0), R(0), R(0)};
    R emx = R(0);
    if (fvalid) {
        const int64_t F = fa.F, E = fa.E;
        rc = ld_facet<NT>(&fa.rec[f]);
        const int64_t r = rc & 0x0fffffff;
        const R* fr = fa.frame + r * 8;
        n0 = fr[0]; n1 = fr[1]; n2 = fr[2];
        m0 = fr[3]; m1 = fr[4]; m2 = fr[5];
        len = fr[6];
        ilen = fr[7];
        ld_quad<NT>(fa.geo, F, f, cI0, cI1, cI2, A);
        ld_quad<NT>((const R*)fa.hist, F, f, tv[0], tv[1], tv[2], emx);
    }
    // output position (incidence order) of the tet-node sums of phase D, and
    // the tet's accumulated internal work
    int32_t opos = 0;
    double wacc = 0.0;
    if (tid < NS && tet0 + (tid >> 2) < T) {
        opos = pos[(tet0 + (tid >> 2)) * 4 + (tid & 3)];
        if ((tid & 3) == 0) wacc = wint[tet0 + (tid >> 2)];
    }
    if (do_prog) {
        const double tn = (double)step * dt, th = ((double)step + 0.5) * dt;
        for (int64_t p = tid; p < pr.P; p += blockDim.x) {
            pr.val[2 * p] = prog_at(pr, p, tn);
            pr.val[2 * p + 1] = prog_at(pr, p, th);
        }
    }

    // ---- A: stage the 4 nodes of each tet (slot a*TB + tl) ----
    if (tid < NS) {
        const int tl = tid % TB, a = tid / TB;
        const int64_t tt = tet0 + tl;
        if (tt < T) {
            const int64_t nd = na.tet[(int64_t)a * T + tt];
#pragma unroll
            for (int c = 0; c < 6; c++) s_q[c][tid] = na.node[nd * 16 + c];
#pragma unroll
            for (int c = 0; c < 6; c++) s_v[c][tid] = na.node[nd * 16 + 6 + c];
#pragma unroll
            for (int c = 0; c < 3; c++) s_x[c][tid] = na.node[nd * 16 + 12 + c];
        }
    }
    if constexpr (NS <= 64) {
        // staging and phase B are both done by wave 0, whose LDS accesses
        // complete in program order: a code-motion fence suffices
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }

    // ---- B: e_V contribution grad N_a . u_a of node a of tet tl ----
    if (tid < NS) {
        const int tl = tid % TB, a = tid / TB;
        if (tet0 + tl < T) {
            int o[3], k = 0;
#pragma unroll
            for (int b = 0; b < 4; b++)
                if (b != a) o[k++] = b * TB + tl;
            const int sa = tid;
            // N_a(x) = det[x_b - x, x_c - x, x_d - x] / det[x_b - x_a, x_c - x_a, x_d - x_a]
            // grad N_a = -((x_c - x_b) x (x_d - x_b)) / det[...]
            double cb[3], db[3], ba[3];
#pragma unroll
            for (int c = 0; c < 3; c++) {
                cb[c] = s_x[c][o[1]] - s_x[c][o[0]];
                db[c] = s_x[c][o[2]] - s_x[c][o[0]];
                ba[c] = s_x[c][o[0]] - s_x[c][sa];
            }
            const double g0 = cb[1] * db[2] - cb[2] * db[1];
            const double g1 = cb[2] * db[0] - cb[0] * db[2];
            const double g2 = cb[0] * db[1] - cb[1] * db[0];
            // det[x_b - x_a, x_c - x_a, x_d - x_a] = (x_b - x_a) . ((x_c - x_b) x (x_d - x_b))
            const double v6 = ba[0] * g0 + ba[1] * g1 + ba[2] * g2;
            s_ev[tid] = -(g0 * s_q[0][sa] + g1 * s_q[1][sa] + g2 * s_q[2][sa]) / v6;
        }
    }
    __syncthreads();

    // ---- C: one lane per facet (blockDim == NF: every lane takes part) ----
    {
        const int tl = ftl;
        double wk = 0.0;
        uint8_t code = 0xff;
        const int64_t F = fa.F;
        R e[3] = {R(0), R(0), R(0)}, de[3] = {R(0), R(0), R(0)}, eV = R(0);
        R l0 = 0, l1 = 0, l2 = 0, cJ0 = 0, cJ1 = 0, cJ2 = 0;
        const R told[3] = {tv[0], tv[1], tv[2]};
        if (fvalid) {
            const int aI = (rc >> 28) & 3, aJ = (rc >> 30) & 3;
            code = (uint8_t)(aI | (aJ << 2));
            const int sI = aI * TB + tl, sJ = aJ * TB + tl;
            l0 = n1 * m2 - n2 * m1;
            l1 = n2 * m0 - n0 * m2;
            l2 = n0 * m1 - n1 * m0;
            cJ0 = cI0 - len * n0;
            cJ1 = cI1 - len * n1;
            cJ2 = cI2 - len * n2;
            // displacement jump [[u]] = u_J + th_J x c^J - u_I - th_I x c^I
            // (translation difference in FP64, rotation terms in R)
            R d[3], dv[3];
            {
                const R du0 = (R)(s_q[0][sJ] - s_q[0][sI]);
                const R du1 = (R)(s_q[1][sJ] - s_q[1][sI]);
                const R du2 = (R)(s_q[2][sJ] - s_q[2][sI]);
                const R tI0 = (R)s_q[3][sI], tI1 = (R)s_q[4][sI], tI2 = (R)s_q[5][sI];
                const R tJ0 = (R)s_q[3][sJ], tJ1 = (R)s_q[4][sJ], tJ2 = (R)s_q[5][sJ];
                d[0] = du0 + (tJ1 * cJ2 - tJ2 * cJ1) - (tI1 * cI2 - tI2 * cI1);
                d[1] = du1 + (tJ2 * cJ0 - tJ0 * cJ2) - (tI2 * cI0 - tI0 * cI2);
                d[2] = du2 + (tJ0 * cJ1 - tJ1 * cJ0) - (tI0 * cI1 - tI1 * cI0);
                const R dv0 = (R)(s_v[0][sJ] - s_v[0][sI]);
                const R dv1 = (R)(s_v[1][sJ] - s_v[1][sI]);
                const R dv2 = (R)(s_v[2][sJ] - s_v[2][sI]);
                const R wI0 = (R)s_v[3][sI], wI1 = (R)s_v[4][sI], wI2 = (R)s_v[5][sI];
                const R wJ0 = (R)s_v[3][sJ], wJ1 = (R)s_v[4][sJ], wJ2 = (R)s_v[5][sJ];
                dv[0] = dv0 + (wJ1 * cJ2 - wJ2 * cJ1) - (wI1 * cI2 - wI2 * cI1);
                dv[1] = dv1 + (wJ2 * cJ0 - wJ0 * cJ2) - (wI2 * cI0 - wI0 * cI2);
                dv[2] = dv2 + (wJ0 * cJ1 - wJ1 * cJ0) - (wI0 * cI1 - wI1 * cI0);
            }
            const R il = ilen;
            e[0] = (n0 * d[0] + n1 * d[1] + n2 * d[2]) * il;
            e[1] = (m0 * d[0] + m1 * d[1] + m2 * d[2]) * il;
            e[2] = (l0 * d[0] + l1 * d[1] + l2 * d[2]) * il;
            if (first) {  // history starts from the undeformed state
                de[0] = e[0];
                de[1] = e[1];
                de[2] = e[2];
            } else {      // q^n - q^{n-1} = dt v^{n-1/2}
                const R sc = (R)dt * il;
                de[0] = (n0 * dv[0] + n1 * dv[1] + n2 * dv[2]) * sc;
                de[1] = (m0 * dv[0] + m1 * dv[1] + m2 * dv[2]) * sc;
                de[2] = (l0 * dv[0] + l1 * dv[1] + l2 * dv[2]) * sc;
            }
            eV = (R)((s_ev[tl] + s_ev[TB + tl] + s_ev[2 * TB + tl] + s_ev[3 * TB + tl]) / 3.0);
        }
        bool exact = fvalid;
        const R emx0 = emx;  // e_max before this step (capture gate)
        if constexpr (MODE == MODE_SURROGATE) {
            // gate: in-envelope facets not yet handed back go through the MLP
            uint8_t fl = 1;
            float x[MLP_IN];
            AlignedFrame fr{1.f, 0.f};
            if (fvalid) {
                fl = sg.flag[f];
                fr = surrogate_features(mat, e, de, told, x);
                if (!fl) {
                    const bool env = in_envelope(mat, e, eV, told, emx, sg.gate);
                    bool box = true;
#pragma unroll
                    for (int k = 0; k < MLP_IN; k++) box = box && x[k] >= sg.lo[k] && x[k] <= sg.hi[k];
                    if (!(env && box)) fl = 1;
                    if (cnt) {
                        cnt->out_env += !env;
                        cnt->out_box += env && !box;
                    }
                }
            }
            const bool use_nn = fvalid && !fl;
            if (__any(use_nn)) {  // wave-uniform: the whole wave runs the network
                float xin[MLP_IN], y[MLP_OUT];
#pragma unroll
                for (int k = 0; k < MLP_IN; k++) xin[k] = use_nn ? (x[k] - sg.xmean[k]) * sg.xscale[k] : 0.f;
                mlp_infer_wave(mlp_smem(), xin, y);
                if (use_nn) {
                    // traction = elastic predictor + residual, the residual
                    // relative to s = |t_old + E de| + tau; below the
                    // network's error floor a relative residual is zero
                    const float s_tr = trial_norm(mat, told, de) + sg.ytau;
                    float r0 = y[0] * sg.yscale[0];
                    float r1 = y[1] * sg.yscale[1];
                    float r2 = y[2] * sg.yscale[2];
                    r0 = (fabsf(r0) < sg.ydead[0] ? 0.f : r0) * s_tr;
                    r1 = (fabsf(r1) < sg.ydead[1] ? 0.f : r1) * s_tr;
                    r2 = (fabsf(r2) < sg.ydead[2] ? 0.f : r2) * s_tr;
                    float rM, rL;
                    from_frame(fr, r1, r2, rM, rL);
                    R tn[3];
                    tn[0] = told[0] + mat.E0 * de[0] + (R)r0;
                    tn[1] = told[1] + mat.aE0 * de[1] + (R)rM;
                    tn[2] = told[2] + mat.aE0 * de[2] + (R)rL;
                    if (facet_damage(mat, e, tn) > sg.gate.damage_max) {
                        fl = 1;  // leaves the envelope: exact law from now on
                        if (cnt) cnt->out_dmg += 1;
                    } else {
                        tv[0] = tn[0];
                        tv[1] = tn[1];
                        tv[2] = tn[2];
                        if (e[0] > R(0)) {  // keep e_max for a later hand-back
                            R sN, sT2, seff, seff2;
                            int ex;
                            scaled_norm(e[0], e[1], e[2], mat.alpha, sN, sT2, seff, seff2, ex);
                            const R eff = d_ldexp(seff, ex);
                            emx = emx > eff ? emx : eff;
                        }
                        exact = false;
                    }
                }
            }
            if (fvalid && fl && !sg.flag[f]) sg.flag[f] = 1;
        }
        if (exact) facet_law<R, LAW>(mat, len, e, de, eV, tv, emx);
        if constexpr (MODE == MODE_SURROGATE) {
            if (cnt && fvalid) {
                // damage of the new traction, whichever law produced it
                const float D = facet_damage(mat, e, tv);
                const bool dmg = D > SG_DAMAGED && D <= sg.gate.damage_max;
                cnt->nn += !exact;
                cnt->dmg += dmg;
                cnt->dmg_nn += dmg && !exact;
            }
        }
        if constexpr (MODE == MODE_CAPTURE) {
            if (fvalid && (f % cp.fstride) == cp.foff && (step % cp.sstride) == 0 &&
                in_envelope(mat, e, eV, told, emx0, cp.gate) &&
                facet_damage(mat, e, tv) <= cp.gate.damage_max) {
                float x[MLP_IN];
                const AlignedFrame fr = surrogate_features(mat, e, de, told, x);
                const R rN = tv[0] - (told[0] + mat.E0 * de[0]);
                const R rM = tv[1] - (told[1] + mat.aE0 * de[1]);
                const R rL = tv[2] - (told[2] + mat.aE0 * de[2]);
                float rp, rq;
                to_frame(fr, (float)rM, (float)rL, rp, rq);
                const unsigned slot = atomicAdd(cp.count, 1u);
                if (slot < (unsigned)cp.cap) {
                    float* row = cp.rows + (int64_t)slot * 16;
#pragma unroll
                    for (int k = 0; k < MLP_IN; k++) row[k] = x[k];
                    row[9] = (float)rN;
                    row[10] = rp;
                    row[11] = rq;
                    const int64_t key = step * 4294967296ll + f;
                    row[12] = __int_as_float((int)(key & 0xffffffff));
                    row[13] = __int_as_float((int)(key >> 32));
                    row[14] = trial_norm(mat, told, de);
                    row[15] = 0.f;
                }
            }
        }
        if (fvalid) {
            st_quad<NT>(fa.hist, F, f, tv[0], tv[1], tv[2], emx);
            // internal work A l (t_old + t)/2 . de
            wk = (double)(A * len * R(0.5) *
                          ((told[0] + tv[0]) * de[0] + (told[1] + tv[1]) * de[1] + (told[2] + tv[2]) * de[2]));
            // facet force A P t and its moments about I and J
            const R F0 = A * (tv[0] * n0 + tv[1] * m0 + tv[2] * l0);
            const R F1 = A * (tv[0] * n1 + tv[1] * m1 + tv[2] * l1);
            const R F2 = A * (tv[0] * n2 + tv[1] * m2 + tv[2] * l2);
            s_F[0][tid] = F0;
            s_F[1][tid] = F1;
            s_F[2][tid] = F2;
            s_MI[0][tid] = cI1 * F2 - cI2 * F1;
            s_MI[1][tid] = cI2 * F0 - cI0 * F2;
            s_MI[2][tid] = cI0 * F1 - cI1 * F0;
            s_MJ[0][tid] = cJ1 * F2 - cJ2 * F1;
            s_MJ[1][tid] = cJ2 * F0 - cJ0 * F2;
            s_MJ[2][tid] = cJ0 * F1 - cJ1 * F0;
        }
        s_w[tid] = wk;
        s_code[tid] = code;
    }
    __syncthreads();

    // ---- D: per tet node, sum its facets in ascending local order and
    //      write the sum at the node's incidence position ----
    if (tid < NS) {
        const int tl = tid >> 2, a = tid & 3;
        const int64_t tt = tet0 + tl;
        if (tt < T) {
            R acc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            // the tet's 12 codes in three words -> the facets on this node
            // (bit j) and those with the node on their J side
            const uint32_t* cw = reinterpret_cast<const uint32_t*>(s_code) + tl * 3;
            const uint32_t w0 = cw[0], w1 = cw[1], w2 = cw[2];
            uint32_t on = 0, onJ = 0;
#pragma unroll
            for (int j = 0; j < 12; j++) {
                const int cd = (int)(((j < 4 ? w0 : (j < 8 ? w1 : w2)) >> (8 * (j & 3))) & 0xff);
                const bool isI = (cd & 3) == a;
                const bool isJ = ((cd >> 2) & 3) == a;
                on |= (uint32_t)(isI || isJ) << j;
                onJ |= (uint32_t)isJ << j;
            }
            // facet j adds +-(F, M): fma(+-1, x, acc) rounds like acc +- x
            auto add = [&](int j) {
                const int fl = tl * 12 + j;
                const bool jside = (onJ >> j) & 1u;
                const R sg = jside ? R(-1) : R(1);
                const R* mrow = jside ? &s_MJ[0][fl] : &s_MI[0][fl];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c] = d_fma(sg, s_F[c][fl], acc[c]);
                    acc[3 + c] = d_fma(sg, mrow[c * NF], acc[3 + c]);
                }
            };
            // ascending j over the node's facets: six in every LDPM tet (two
            // per edge, three edges per node), any number otherwise
            if (__builtin_popcount(on) == 6) {
                int idx[6];
                uint32_t m = on;
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    idx[k] = __builtin_ctz(m);
                    m &= m - 1;
                }
#pragma unroll
                for (int k = 0; k < 6; k++) add(idx[k]);
            } else {
                for (uint32_t m = on; m; m &= m - 1) add(__builtin_ctz(m));
            }
            R* out = contrib + (int64_t)opos * 6;
#pragma unroll
            for (int c = 0; c < 6; c++) out[c] = acc[c];
            if (a == 0) {
                double w = 0.0;
#pragma unroll
                for (int j = 0; j < 12; j++) w += s_w[tl * 12 + j];
                wint[tt] = wacc + w;
            }
        }
    }
}

template <typename R, int LAW, int TB, int MODE, int NT = 0>
__global__ __launch_bounds__(12 * TB) void k_facet(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                                   const int32_t* __restrict__ pos,
                                                   R* __restrict__ contrib, double* __restrict__ wint,
                                                   ProgArgs pr, int64_t step, double dt, int remap,
                                                   SurrogateArgs sg, CaptureArgs cp)
{
    if constexpr (MODE == MODE_SURROGATE) mlp_load_frag(sg.params, mlp_smem(), threadIdx.x, 12 * TB);
    facet_tile<R, LAW, TB, MODE, NT>(xcd_block(blockIdx.x, gridDim.x, remap), blockIdx.x == 0, na, fa, mat, pos,
                                     contrib, wint, pr, step, dt, sg, cp);
}

// Grid-stride loop over tiles: blocks stay resident and load the surrogate's
// weights into LDS once instead of once per tile.  At least 3 waves per SIMD
// (at most 168 VGPRs): four 16-tet blocks per CU, as many as their LDS
// (weights and tile) allows.
template <typename R, int LAW, int TB, int MODE>
__global__ __launch_bounds__(12 * TB, 3) void k_facet_loop(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                                        const int32_t* __restrict__ pos,
                                                        R* __restrict__ contrib, double* __restrict__ wint,
                                                        ProgArgs pr, int64_t step, double dt,
                                                        SurrogateArgs sg, CaptureArgs cp)
{
    if constexpr (MODE == MODE_SURROGATE) mlp_load_frag(sg.params, mlp_smem(), threadIdx.x, 12 * TB);
    const int64_t nb = (na.T + TB - 1) / TB;
    SgCount c;
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x)
        facet_tile<R, LAW, TB, MODE>(blk, blk == 0, na, fa, mat, pos, contrib, wint, pr, step, dt, sg, cp, &c);
    if constexpr (MODE == MODE_SURROGATE) {
        // block totals (integer sums: exact in any order), then one atomic
        // per counter and block
        __shared__ unsigned s_cnt[SG_NSTATS];
        if (threadIdx.x < SG_NSTATS) s_cnt[threadIdx.x] = 0;
        __syncthreads();
        const unsigned v[SG_NSTATS] = {c.nn, c.dmg, c.dmg_nn, c.out_env, c.out_box, c.out_dmg};
#pragma unroll
        for (int k = 0; k < SG_NSTATS; k++)
            if (v[k]) atomicAdd(&s_cnt[k], v[k]);
        __syncthreads();
        if (threadIdx.x < SG_NSTATS && s_cnt[threadIdx.x])
            atomicAdd(&sg.stats[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// particle kernel
// ---------------------------------------------------------------------------
// PG lanes per particle: lane l sums incidences ptr[I] + l, + PG, ... of the
// contributions stored in incidence order; an xor butterfly (commutative, so
// every lane ends with the same bits) completes the sum; lane d < 6 then
// advances DoF d.  The grouping is fixed, so results do not depend on the
// block size.
constexpr int PG = 16;

// Particle I = gt / PG, lane gt % PG (gt: a global lane index; groups of PG
// lanes are aligned within a wave and take the branch together).
// FULLM: the particle's 6 x 6 cell mass block couples its DoFs (eq.
// balance): prescribed DoFs take their programmed velocity, whose
// acceleration a_P enters the free rows, a_F = G (f_net - M a_P); the
// reactions are (M a)_P - f_net,P and the kinetic energy 1/2 vb^T M vb.
template <typename R, int FULLM>
__device__ __forceinline__ void particle_group(int64_t gt, const ParticleArgs& pa, const R* __restrict__ contrib,
                                               int64_t n, double dt)
{
    const int64_t I = gt / PG;
    const int lane = (int)(gt % PG);
    const int64_t N = pa.N;
    if (I >= N) return;
    // per-DoF data of lane d < 6, loaded before the gather
    const int d = lane < 6 ? lane : 0;
    const int64_t id = d * N + I;
    const double M = FULLM ? 0.0 : (d < 3 ? pa.mass[I] : pa.inertia[(d - 3) * N + I]);
    const double bodyf = pa.body ? pa.body[id] : 0.0;
    const int32_t pg = pa.prog[id];
    const uint8_t md = pa.mode[id];
    const double scl = pa.scale[id];
    const double vold = pa.node[I * 16 + 6 + d];
    const double fold = pa.fext[id];
    const double qold = pa.node[I * 16 + d];
    double mrow[6], grow[6];
    if constexpr (FULLM) {
        const double* mb = pa.mblk + I * 72 + d * 6;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            mrow[k] = mb[k];
            grow[k] = mb[36 + k];
        }
    }
    double f[6] = {0, 0, 0, 0, 0, 0};
    const int32_t s0 = pa.ptr[I], s1 = pa.ptr[I + 1];
    for (int32_t s = s0 + lane; s < s1; s += PG) {
        const R* c = contrib + (int64_t)s * 6;
#pragma unroll
        for (int k = 0; k < 6; k++) f[k] += (double)c[k];
    }
#pragma unroll
    for (int off = PG / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 6; k++) f[k] += __shfl_xor(f[k], off, PG);
    }
    double wk = 0.0, dwe = 0.0;
    bool bad = false;
    const double h = (n == 0) ? 0.5 * dt : dt;
    if constexpr (FULLM) {
        double fd = f[0];
#pragma unroll
        for (int k = 1; k < 6; k++) fd = (d == k) ? f[k] : fd;
        double applied = bodyf;
        if (md == 0 && pg >= 0) applied += scl * pa.progv[2 * pg];
        const double fnet = fd + applied;
        double vnew = 0.0, acc = 0.0;
        if (md != 0) {
            vnew = (pg >= 0) ? scl * pa.progv[2 * pg + 1] : 0.0;
            acc = (vnew - vold) / h;
        }
        // z = f_net - M a_P (row d), then a_F = G z
        double z = fnet;
#pragma unroll
        for (int k = 0; k < 6; k++) z -= mrow[k] * __shfl(acc, k, PG);
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) a += grow[k] * __shfl(z, k, PG);
        if (md == 0) {
            acc = a;
            vnew = vold + h * a;
        }
        double ma = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) ma += mrow[k] * __shfl(acc, k, PG);
        const double Fd = (md == 0) ? applied : applied + (ma - fnet);  // reaction on prescribed DoFs
        const double vb = (n == 0) ? vold : 0.5 * (vold + vnew);
        double mvb = 0.0;
#pragma unroll
        for (int k = 0; k < 6; k++) mvb += mrow[k] * __shfl(vb, k, PG);
        if (lane < 6) {
            if (n > 0) dwe = 0.5 * (fold + Fd) * (dt * vold);
            wk = 0.5 * vb * mvb;
            pa.fext[id] = Fd;
            pa.node[I * 16 + 6 + d] = vnew;
            pa.node[I * 16 + d] = qold + dt * vnew;
            bad = !isfinite(vnew);
        }
    } else if (lane < 6) {
        double fd = f[0];
#pragma unroll
        for (int k = 1; k < 6; k++) fd = (d == k) ? f[k] : fd;
        double applied = bodyf;
        if (md == 0 && pg >= 0) applied += scl * pa.progv[2 * pg];
        const double fnet = fd + applied;
        double vnew, Fd;
        if (md == 0) {
            vnew = vold + h * fnet / M;
            Fd = applied;
        } else {
            vnew = (pg >= 0) ? scl * pa.progv[2 * pg + 1] : 0.0;
            const double R_ = M * (vnew - vold) / h - fnet;  // reaction
            Fd = applied + R_;
        }
        if (n > 0) dwe = 0.5 * (fold + Fd) * (dt * vold);
        const double vb = (n == 0) ? vold : 0.5 * (vold + vnew);
        wk = 0.5 * M * vb * vb;
        pa.fext[id] = Fd;
        pa.node[I * 16 + 6 + d] = vnew;
        pa.node[I * 16 + d] = qold + dt * vnew;
        bad = !isfinite(vnew);
    }
    // energies of the particle: DoFs summed in order 0..5 by lane 0
    double wks = 0.0, dws = 0.0;
#pragma unroll
    for (int d = 0; d < 6; d++) {
        wks += __shfl(wk, d, PG);
        dws += __shfl(dwe, d, PG);
    }
    if (lane == 0) {
        pa.wext[I] += dws;
        pa.wkin[I] = wks;
    }
    if (bad) pa.flag[0] = 1;
}

template <typename R, int FULLM>
__global__ __launch_bounds__(1024) void k_particle(ParticleArgs pa, const R* __restrict__ contrib,
                                                   int64_t n, double dt)
{
    particle_group<R, FULLM>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, pa, contrib, n, dt);
}

// ---------------------------------------------------------------------------
// persistent multi-step kernel: n steps in one cooperative launch, the facet
// and particle phases separated by grid barriers.  Co-residency of every
// block is guaranteed by the cooperative launch; the barrier still gives up
// after a bounded wait (flagging an error) so that no wave can spin forever.
// ---------------------------------------------------------------------------
struct GridSync {
    unsigned* count;  // arrivals at the current barrier
    unsigned* gen;    // barrier generation
    int32_t* flag;    // [1]: barrier timeout (error flag word 1)
};

__device__ __forceinline__ bool grid_barrier(const GridSync& g, unsigned nblocks)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        // release this block's writes to the device (one L2 write-back), read
        // the generation, and only then arrive (the wait keeps the read ahead
        // of the arrival, so the last arrival's increment cannot overtake it)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned gen0 = __hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
        const unsigned arrived = __hip_atomic_fetch_add(g.count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        int ok = 1;
        if (arrived == nblocks) {
            __hip_atomic_store(g.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(g.gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // poll with device-coherent relaxed loads (no cache maintenance per
            // poll); bounded so that no wave can spin forever
            long spins = 0;
            while (__hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1l << 24)) {  // ~seconds: never reached when co-resident
                    g.flag[1] = 1;
                    ok = 0;
                    break;
                }
            }
        }
        // acquire the other blocks' writes (one L2 invalidation)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

template <typename R, int LAW, int TB>
__global__ __launch_bounds__(12 * TB) void k_persist(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                                     const int32_t* __restrict__ pos, R* __restrict__ contrib,
                                                     double* __restrict__ wint, ProgArgs pr, ParticleArgs pa,
                                                     GridSync gs, int64_t step0, int64_t nsteps, double dt,
                                                     SurrogateArgs sg, CaptureArgs cp)
{
    const int64_t nb = (na.T + TB - 1) / TB;
    const unsigned G = gridDim.x;
    const int64_t lanes = pa.N * PG;
    for (int64_t i = 0; i < nsteps; i++) {
        const int64_t n = step0 + i;
        for (int64_t blk = blockIdx.x; blk < nb; blk += G)
            facet_tile<R, LAW, TB, MODE_PLAIN>(blk, blk == 0, na, fa, mat, pos, contrib, wint, pr, n, dt, sg, cp);
        if (!grid_barrier(gs, G)) return;
        for (int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gt < lanes; gt += (int64_t)G * blockDim.x)
            particle_group<R, 0>(gt, pa, contrib, n, dt);
        if (!grid_barrier(gs, G)) return;
    }
}

// ---------------------------------------------------------------------------
// deterministic reductions (fixed strided order + fixed LDS tree)
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

__device__ double block_sum_fixed(double x)
{
    __shared__ double s[RED_THREADS];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// Two stages with fixed grids: block b of G sums the elements
// lo + b*RED_THREADS + k*G*RED_THREADS (thread order, then the LDS tree)
// into partials [3][G]; one block then adds the G partials in order.  G
// depends only on the range's own length, so a specimen's energies do not
// depend on the other specimens of a batch.
constexpr int RED_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(RED_THREADS) void k_energy_part(const double* __restrict__ wint, int64_t t0,
                                                             int64_t t1, const double* __restrict__ wext,
                                                             const double* __restrict__ wkin, int64_t p0,
                                                             int64_t p1, double* __restrict__ part)
{
    const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
    const int64_t o = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = t0 + o; i < t1; i += stride) a += wint[i];
    for (int64_t i = p0 + o; i < p1; i += stride) {
        b += wext[i];
        c += wkin[i];
    }
    a = block_sum_fixed(a);
    b = block_sum_fixed(b);
    c = block_sum_fixed(c);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
        part[2 * gridDim.x + blockIdx.x] = c;
    }
}

// resultant of the generalised forces of DoFs driven by program p (partials)
__global__ __launch_bounds__(RED_THREADS) void k_reaction_part(const double* __restrict__ fext,
                                                               const int32_t* __restrict__ prog, int64_t n6,
                                                               int32_t p, double* __restrict__ part)
{
    const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < n6; i += stride)
        if (prog[i] == p) a += fext[i];
    a = block_sum_fixed(a);
    if (threadIdx.x == 0) part[blockIdx.x] = a;
}

// out[k] = sum of part[k*G .. k*G + G) in order, k < nk (one block)
__global__ __launch_bounds__(RED_THREADS) void k_sum_parts(const double* __restrict__ part, int G, int nk,
                                                           double* __restrict__ out)
{
    for (int k = 0; k < nk; k++) {
        double a = 0.0;
        for (int i = threadIdx.x; i < G; i += RED_THREADS) a += part[(int64_t)k * G + i];
        a = block_sum_fixed(a);
        if (threadIdx.x == 0) out[k] = a;
    }
}

