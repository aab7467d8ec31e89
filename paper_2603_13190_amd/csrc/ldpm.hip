// MI355X (gfx950) explicit LDPM step behind the C-ABI of include/ldpm.h.
//
// Data layout in HBM (structure of arrays):
//   particles  node records [N] of 16 doubles (q[6], v[6], x0[3], pad: one
//              128-byte line per node for the facet kernel's gather),
//              mass[N], inertia[3][N],
//              dof mode/program/scale [6][N], fext[6][N], w_ext[N], w_kin[N],
//              incidence CSR: ptr[N+1]; tet-node (t, a) sits at pos[4t+a]
//   tets       nodes[4][T], pos[4T], w_int[T],
//              contributions [4T][6] per tet-node, stored in incidence order
//   facets     cI[3][F], area[F], rec[F] (edge-frame id | local I,J code),
//              history t[3][F], e_max[F]                (FP64 or FP32)
//   edge frames records [E] of 8 R (n[3], m[3], len, pad): one 64-byte
//              (FP64) or 32-byte (FP32) record per deduplicated (n, m, len)
//
// One step = two kernels:
//   k_facet    one block per TB tetrahedra, one lane per facet (12 TB lanes).
//              Node states of the block's tets are staged in LDS; e_V per
//              tet (eq. for e_V in the appendix); per facet: displacement
//              jump and strain (eq. strain1), strain increment from the FP64
//              velocities, constitutive law (appendix), force A P t and
//              moments c x (A P t) (eq. balance), internal-work increment;
//              the 6 facets touching each tet node are summed in LDS in a
//              fixed order, so each tet writes 4 x 6 numbers instead of 12 x 9.
//   k_particle 16 lanes per particle: gathers its tet-node contributions,
//              stored contiguously in ascending tetrahedron order (no
//              atomics), adds applied and body forces, leapfrog update in
//              FP64 (one lane per DoF), reactions, energies.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ldpm.h"
#include "law.hpp"
#include "mlp.hpp"

using namespace ldpm;

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static ldpm_status fail(ldpm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

ldpm_status ldpm_fail(ldpm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess)                                                             \
            return fail(LDPM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

// ---------------------------------------------------------------------------
// device argument blocks
// ---------------------------------------------------------------------------
template <typename R>
struct FacetArgs {
    const R* __restrict__ cI;      // [3][F]
    const R* __restrict__ area;    // [F]
    const int32_t* __restrict__ rec;  // [F]
    const R* __restrict__ frame;   // [E][8]: n[3], m[3], len, pad
    R* __restrict__ ht;            // [3][F]
    R* __restrict__ hemax;         // [F]
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
    float xmean[MLP_IN], xscale[MLP_IN], yscale[MLP_OUT], ydead[MLP_OUT], lo[MLP_IN], hi[MLP_IN];
    float ytau;
    GateArgs gate;
};

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
};

// ---------------------------------------------------------------------------
// facet kernel
// ---------------------------------------------------------------------------
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

// Is the facet inside the surrogate's envelope (the pre-peak elastic and
// frictional regime the network is trained on)?  Tension: the effective
// strain and e_max stay below kappa_t of the elastic limit e0(omega) (and of
// sigma_t/E0 for e_max, whatever the angle); compression: -e_DV and -t_N stay
// below kappa_c of the onset of pore collapse (e_c0, sigma_c0).
template <typename R>
__device__ __forceinline__ bool in_envelope(const MatDev<R>& p, const R e[3], R eV, const R told[3], R emax,
                                            const GateArgs& g)
{
    const R emax_lim = (R)g.kappa_t * p.sigma_t * p.inv_E0;
    if (emax >= emax_lim) return false;
    if (e[0] > R(0)) {
        R sN, sT2, seff, seff2;
        int ex;
        scaled_norm(e[0], e[1], e[2], p.alpha, sN, sT2, seff, seff2, ex);
        const R eff = d_ldexp(seff, ex);
        const R inv = R(1) / seff;
        const R sn = sN * inv, cs2 = p.alpha * sT2 * (inv * inv);
        const R sigma0 = R(2) * p.sigma_t / (sn + d_sqrt(sn * sn + p.c4 * cs2));
        return eff < (R)g.kappa_t * sigma0 * p.inv_E0;
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

// LDS of the surrogate: weights of the block plus one activation tile per wave
template <int NW>
struct MlpSmem {
    MlpBf16 W;
    __bf16 buf[NW][64 * PA];
    float out[NW][64 * 4];
};
template <int NW>
__device__ __forceinline__ MlpSmem<NW>& mlp_smem()
{
    __shared__ MlpSmem<NW> sm;
    return sm;
}

// One tile of TB tetrahedra (block-wide: every thread of a 12 TB block calls
// it together).  do_prog: this block also evaluates the time programs.
template <typename R, int LAW, int TB, int MODE>
__device__ __forceinline__ void facet_tile(int64_t blk, bool do_prog, const NodeArgs& na, const FacetArgs<R>& fa,
                                           const MatDev<R>& mat, const int32_t* __restrict__ pos,
                                           R* __restrict__ contrib, double* __restrict__ wint,
                                           const ProgArgs& pr, int64_t step, double dt,
                                           const SurrogateArgs& sg, const CaptureArgs& cp)
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
        rc = fa.rec[f];
        const int64_t r = rc & 0x0fffffff;
        const R* fr = fa.frame + r * 8;
        n0 = fr[0]; n1 = fr[1]; n2 = fr[2];
        m0 = fr[3]; m1 = fr[4]; m2 = fr[5];
        len = fr[6];
        ilen = fr[7];
        cI0 = fa.cI[f]; cI1 = fa.cI[F + f]; cI2 = fa.cI[2 * F + f];
        A = fa.area[f];
        tv[0] = fa.ht[f]; tv[1] = fa.ht[F + f]; tv[2] = fa.ht[2 * F + f];
        if (LAW != 0) emx = fa.hemax[f];
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
        if constexpr (MODE == MODE_SURROGATE) {
            // gate: in-envelope facets not yet handed back go through the MLP
            uint8_t fl = 1;
            float x[MLP_IN];
            AlignedFrame fr{1.f, 0.f};
            if (fvalid) {
                fl = sg.flag[f];
                fr = surrogate_features(mat, e, de, told, x);
                if (!fl) {
                    bool ok = in_envelope(mat, e, eV, told, emx, sg.gate);
#pragma unroll
                    for (int k = 0; k < MLP_IN; k++) ok = ok && x[k] >= sg.lo[k] && x[k] <= sg.hi[k];
                    if (!ok) fl = 1;
                }
            }
            const bool use_nn = fvalid && !fl;
            auto& sm = mlp_smem<NF / 64>();
            const int w = tid >> 6, lane = tid & 63;
            if (__any(use_nn)) {  // wave-uniform: the whole wave runs the tiles
                __bf16* buf = sm.buf[w];
#pragma unroll
                for (int k = 0; k < K1; k++)
                    buf[lane * PA + k] =
                        to_bf16((use_nn && k < MLP_IN) ? (x[k] - sg.xmean[k]) * sg.xscale[k] : 0.f);
                __builtin_amdgcn_wave_barrier();
                mlp_forward_wave(sm.W, buf, sm.out[w]);
                if (use_nn) {
                    // traction = elastic predictor + residual, the residual
                    // relative to s = |t_old + E de| + tau; below the
                    // network's error floor a relative residual is zero
                    const float s_tr = trial_norm(mat, told, de) + sg.ytau;
                    float r0 = sm.out[w][lane * 4 + 0] * sg.yscale[0];
                    float r1 = sm.out[w][lane * 4 + 1] * sg.yscale[1];
                    float r2 = sm.out[w][lane * 4 + 2] * sg.yscale[2];
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
        if constexpr (MODE == MODE_CAPTURE) {
            if (fvalid && (f % cp.fstride) == cp.foff && (step % cp.sstride) == 0 &&
                in_envelope(mat, e, eV, told, (R)fa.hemax[f], cp.gate) &&
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
            fa.ht[f] = tv[0];
            fa.ht[F + f] = tv[1];
            fa.ht[2 * F + f] = tv[2];
            if (LAW != 0) fa.hemax[f] = emx;
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

    // ---- D: per tet node, sum its 6 facets in ascending local order and
    //      write the sum at the node's incidence position ----
    if (tid < NS) {
        const int tl = tid >> 2, a = tid & 3;
        const int64_t tt = tet0 + tl;
        if (tt < T) {
            R acc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            // the tet's 12 codes in three words; each facet adds sg * value
            // with sg = +1 (node on the I side), -1 (J side) or 0 (not on the
            // facet): fma(+-1, x, acc) rounds like acc +- x
            const uint32_t* cw = reinterpret_cast<const uint32_t*>(s_code) + tl * 3;
            const uint32_t w0 = cw[0], w1 = cw[1], w2 = cw[2];
#pragma unroll
            for (int j = 0; j < 12; j++) {
                const int fl = tl * 12 + j;
                const int cd = (int)(((j < 4 ? w0 : (j < 8 ? w1 : w2)) >> (8 * (j & 3))) & 0xff);
                const bool onI = (cd & 3) == a;
                const bool onJ = ((cd >> 2) & 3) == a;
                const R sg = onI ? R(1) : (onJ ? R(-1) : R(0));
                const R* mrow = onI ? &s_MI[0][fl] : &s_MJ[0][fl];
#pragma unroll
                for (int c = 0; c < 3; c++) {
                    acc[c] = d_fma(sg, s_F[c][fl], acc[c]);
                    acc[3 + c] = d_fma(sg, mrow[c * NF], acc[3 + c]);
                }
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

template <typename R, int LAW, int TB, int MODE>
__global__ __launch_bounds__(12 * TB) void k_facet(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                                   const int32_t* __restrict__ pos,
                                                   R* __restrict__ contrib, double* __restrict__ wint,
                                                   ProgArgs pr, int64_t step, double dt, int remap,
                                                   SurrogateArgs sg, CaptureArgs cp)
{
    if constexpr (MODE == MODE_SURROGATE) mlp_load_bf16(sg.params, mlp_smem<12 * TB / 64>().W, threadIdx.x, 12 * TB);
    facet_tile<R, LAW, TB, MODE>(xcd_block(blockIdx.x, gridDim.x, remap), blockIdx.x == 0, na, fa, mat, pos,
                                 contrib, wint, pr, step, dt, sg, cp);
}

// Grid-stride loop over tiles: blocks stay resident and load the surrogate's
// weights into LDS once instead of once per tile.
template <typename R, int LAW, int TB, int MODE>
__global__ __launch_bounds__(12 * TB) void k_facet_loop(NodeArgs na, FacetArgs<R> fa, MatDev<R> mat,
                                                        const int32_t* __restrict__ pos,
                                                        R* __restrict__ contrib, double* __restrict__ wint,
                                                        ProgArgs pr, int64_t step, double dt,
                                                        SurrogateArgs sg, CaptureArgs cp)
{
    if constexpr (MODE == MODE_SURROGATE) mlp_load_bf16(sg.params, mlp_smem<12 * TB / 64>().W, threadIdx.x, 12 * TB);
    const int64_t nb = (na.T + TB - 1) / TB;
    for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x)
        facet_tile<R, LAW, TB, MODE>(blk, blk == 0, na, fa, mat, pos, contrib, wint, pr, step, dt, sg, cp);
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
template <typename R>
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
    const double M = d < 3 ? pa.mass[I] : pa.inertia[(d - 3) * N + I];
    const double bodyf = pa.body ? pa.body[id] : 0.0;
    const int32_t pg = pa.prog[id];
    const uint8_t md = pa.mode[id];
    const double scl = pa.scale[id];
    const double vold = pa.node[I * 16 + 6 + d];
    const double fold = pa.fext[id];
    const double qold = pa.node[I * 16 + d];
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
    if (lane < 6) {
        double fd = f[0];
#pragma unroll
        for (int k = 1; k < 6; k++) fd = (d == k) ? f[k] : fd;
        const double h = (n == 0) ? 0.5 * dt : dt;
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

template <typename R>
__global__ __launch_bounds__(1024) void k_particle(ParticleArgs pa, const R* __restrict__ contrib,
                                                   int64_t n, double dt)
{
    particle_group<R>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, pa, contrib, n, dt);
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
        __threadfence();  // release this block's writes to the whole device
        const unsigned gen0 = __hip_atomic_load(g.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(g.count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        int ok = 1;
        if (arrived == nblocks) {
            __hip_atomic_store(g.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(g.gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long spins = 0;
            while (__hip_atomic_load(g.gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen0) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1l << 24)) {  // ~seconds: never reached when co-resident
                    g.flag[1] = 1;
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();  // acquire the other blocks' writes
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
            particle_group<R>(gt, pa, contrib, n, dt);
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

__global__ __launch_bounds__(RED_THREADS) void k_energy(const double* __restrict__ wint, int64_t t0,
                                                        int64_t t1, const double* __restrict__ wext,
                                                        const double* __restrict__ wkin, int64_t p0,
                                                        int64_t p1, double* __restrict__ out)
{
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = t0 + threadIdx.x; i < t1; i += RED_THREADS) a += wint[i];
    for (int64_t i = p0 + threadIdx.x; i < p1; i += RED_THREADS) {
        b += wext[i];
        c += wkin[i];
    }
    a = block_sum_fixed(a);
    b = block_sum_fixed(b);
    c = block_sum_fixed(c);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
        out[2] = c;
    }
}

__global__ __launch_bounds__(RED_THREADS) void k_reaction(const double* __restrict__ fext,
                                                          const int32_t* __restrict__ prog, int64_t n6,
                                                          int32_t p, double* __restrict__ out)
{
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n6; i += RED_THREADS)
        if (prog[i] == p) a += fext[i];
    a = block_sum_fixed(a);
    if (threadIdx.x == 0) out[0] = a;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct ldpm_system {
    int64_t N = 0, T = 0, F = 0, E = 0;
    int32_t nspec = 1, prec = 0, law = 1;
    std::vector<int64_t> poff, toff;
    std::vector<double> wkin0;
    double dt = 0;
    int64_t step = 0;
    hipStream_t stream = nullptr;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    void (*dev_free)(void*, void*) = nullptr;
    void* (*dev_alloc)(size_t, void*) = nullptr;
    void* alloc_ctx = nullptr;
    int device = 0;
    ldpm_launch launch{16, 256, 1, 0};
    int n_cu = 0;
    // device pointers
    double *node, *mass, *inertia, *scale, *body, *fext, *wext, *wkin, *wint;
    uint8_t* mode;
    int32_t *prog, *ptr, *pos, *tet, *rec, *flag;
    unsigned* bar;
    int64_t* prog_off;
    double *prog_t, *prog_v, *progv, *red;
    void *cI, *area, *frame, *ht, *hemax, *contrib;
    int64_t n_prog_pts = 0, n_prog = 0;
    MatDev<double> matd;
    MatDev<float> matf;
    // surrogate (mixed precision, full law) and training-sample capture (FP64)
    bool sg_on = false, cp_on = false;
    SurrogateArgs sg{};
    CaptureArgs cp{};
    void* sg_mem = nullptr;  // params + flags
    void* cp_mem = nullptr;  // rows + counter
};

namespace {

struct Carve {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        const size_t o = off;
        off += count * sizeof(T);
        return o;
    }
};

template <typename R>
MatDev<R> make_mat(const ldpm_material& m)
{
    MatDev<R> p;
    const double E0 = m.E0, al = m.alpha;
    p.E0 = (R)E0;
    p.alpha = (R)al;
    p.aE0 = (R)(al * E0);
    p.inv_alpha = (R)(1.0 / al);
    p.inv_E0 = (R)(1.0 / E0);
    p.sigma_t = (R)m.sigma_t;
    p.l_t = (R)m.l_t;
    p.c4 = (R)(4.0 * al / (m.r_st * m.r_st));
    p.n_t = (R)m.n_t;
    p.Hs_over_alpha = (R)(m.r_s * E0 / al);
    p.k_t = (R)m.k_t;
    p.sigma_c0 = (R)m.sigma_c0;
    p.Hc0 = (R)(m.Hc0_over_E0 * E0);
    p.Hc1 = (R)(m.Hc1_over_E0 * E0);
    p.kc1 = (R)m.kc1;
    p.kc2 = (R)m.kc2;
    p.eV0 = (R)(m.kc3 * m.sigma_c0 / E0);
    const double ec0 = m.sigma_c0 / E0;
    p.ec0 = (R)ec0;
    p.ec1 = (R)(m.kc0 * ec0);
    p.Ed = (R)(m.Ed_over_E0 * E0);
    p.beta = (R)m.beta;
    const double ss = m.r_st * m.sigma_t;
    p.sigma_s = (R)ss;
    p.sigma_s2 = (R)(ss * ss);
    p.dmu_sN0 = (R)((m.mu0 - m.mu_inf) * m.sigma_N0);
    p.mu_inf = (R)m.mu_inf;
    p.inv_sigma_N0 = (R)(1.0 / m.sigma_N0);
    p.two_over_pi = (R)(2.0 / M_PI);
    return p;
}

bool finite_all(const double* p, int64_t n)
{
    for (int64_t i = 0; i < n; i++)
        if (!std::isfinite(p[i])) return false;
    return true;
}

struct FrameKey {
    double v[7];
    bool operator==(const FrameKey& o) const { return memcmp(v, o.v, sizeof(v)) == 0; }
};
struct FrameHash {
    size_t operator()(const FrameKey& k) const
    {
        uint64_t h = 1469598103934665603ull;
        const unsigned char* p = (const unsigned char*)k.v;
        for (size_t i = 0; i < sizeof(k.v); i++) h = (h ^ p[i]) * 1099511628211ull;
        return (size_t)h;
    }
};

template <typename R>
void to_r(std::vector<unsigned char>& buf, const double* src, size_t n)
{
    buf.resize(n * sizeof(R));
    R* d = (R*)buf.data();
    for (size_t i = 0; i < n; i++) d[i] = (R)src[i];
}

size_t rbytes(int prec) { return prec == LDPM_PREC_MIXED ? 4 : 8; }

}  // namespace

// Kernel launches.  With events (ev0, ev1) the launch is made with
// hipExtLaunchKernelGGL, whose start/stop events are timestamped by the
// dispatch itself (the kernel's own duration, as a profiler reports it).
template <typename R, int LAW, int TB, int MODE>
static void launch_facet_m(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    NodeArgs na{s->tet, s->node, s->N, s->T};
    FacetArgs<R> fa{(const R*)s->cI, (const R*)s->area, s->rec, (const R*)s->frame, (R*)s->ht, (R*)s->hemax,
                    s->F, s->E};
    ProgArgs pr{s->prog_off, s->prog_t, s->prog_v, s->progv, s->n_prog};
    const MatDev<R>& mat = *(const MatDev<R>*)(sizeof(R) == 8 ? (const void*)&s->matd : (const void*)&s->matf);
    const int64_t nb = (s->T + TB - 1) / TB;
    if constexpr (MODE == MODE_SURROGATE) {
        int per_cu = 1;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_facet_loop<R, LAW, TB, MODE>, 12 * TB, 0);
        const int64_t G = std::min<int64_t>(nb, (int64_t)std::max(per_cu, 1) * std::max(s->n_cu, 1));
        if (ev0)
            hipExtLaunchKernelGGL((k_facet_loop<R, LAW, TB, MODE>), dim3((unsigned)G), dim3(12 * TB), 0, s->stream,
                                  ev0, ev1, 0, na, fa, mat, (const int32_t*)s->pos, (R*)s->contrib, s->wint, pr,
                                  s->step, s->dt, s->sg, s->cp);
        else
            hipLaunchKernelGGL((k_facet_loop<R, LAW, TB, MODE>), dim3((unsigned)G), dim3(12 * TB), 0, s->stream, na,
                               fa, mat, (const int32_t*)s->pos, (R*)s->contrib, s->wint, pr, s->step, s->dt, s->sg,
                               s->cp);
        return;
    }
    if (ev0)
        hipExtLaunchKernelGGL((k_facet<R, LAW, TB, MODE>), dim3((unsigned)nb), dim3(12 * TB), 0, s->stream, ev0, ev1,
                              0, na, fa, mat, (const int32_t*)s->pos, (R*)s->contrib, s->wint, pr, s->step, s->dt,
                              s->launch.xcd_remap, s->sg, s->cp);
    else
        hipLaunchKernelGGL((k_facet<R, LAW, TB, MODE>), dim3((unsigned)nb), dim3(12 * TB), 0, s->stream, na, fa, mat,
                           (const int32_t*)s->pos, (R*)s->contrib, s->wint, pr, s->step, s->dt, s->launch.xcd_remap,
                           s->sg, s->cp);
}

template <typename R, int LAW, int TB>
static void launch_facet_t(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    if constexpr (LAW == 1 && std::is_same<R, double>::value) {
        if (s->cp_on) return launch_facet_m<R, LAW, TB, MODE_CAPTURE>(s, ev0, ev1);
    }
    if constexpr (LAW == 1 && std::is_same<R, float>::value && TB >= 16 && TB <= 32) {
        if (s->sg_on) return launch_facet_m<R, LAW, TB, MODE_SURROGATE>(s, ev0, ev1);
    }
    if constexpr (LAW == 1 && std::is_same<R, float>::value && TB == 8) {
        // the surrogate's tiles need whole waves (8-tet tiles have 1.5)
        if (s->sg_on) return launch_facet_m<R, LAW, 16, MODE_SURROGATE>(s, ev0, ev1);
    }
    if constexpr (LAW == 1 && std::is_same<R, float>::value && TB == 64) {
        // the surrogate's weights and activation tiles do not fit next to a
        // 64-tet tile in LDS: it runs with 32-tet tiles
        if (s->sg_on) return launch_facet_m<R, LAW, 32, MODE_SURROGATE>(s, ev0, ev1);
    }
    launch_facet_m<R, LAW, TB, MODE_PLAIN>(s, ev0, ev1);
}

template <typename R, int LAW>
static void launch_facet_l(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (s->launch.tets_per_block) {
    case 8: launch_facet_t<R, LAW, 8>(s, ev0, ev1); break;
    case 32: launch_facet_t<R, LAW, 32>(s, ev0, ev1); break;
    case 64: launch_facet_t<R, LAW, 64>(s, ev0, ev1); break;
    default: launch_facet_t<R, LAW, 16>(s, ev0, ev1); break;
    }
}

static void launch_facet(ldpm_system* s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (s->prec == LDPM_PREC_MIXED) {
        if (s->law == 0) launch_facet_l<float, 0>(s, ev0, ev1);
        else launch_facet_l<float, 1>(s, ev0, ev1);
    } else {
        if (s->law == 0) launch_facet_l<double, 0>(s, ev0, ev1);
        else launch_facet_l<double, 1>(s, ev0, ev1);
    }
}

template <typename R>
static void launch_particle_t(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    ParticleArgs pa{s->node, s->mass, s->inertia, s->mode, s->prog, s->scale, s->body,
                    s->fext, s->wext, s->wkin, s->ptr,     s->progv, s->flag, s->N};
    const int th = s->launch.particle_threads;
    const unsigned nb = (unsigned)((s->N * PG + th - 1) / th);
    if (ev0)
        hipExtLaunchKernelGGL(k_particle<R>, dim3(nb), dim3(th), 0, s->stream, ev0, ev1, 0, pa,
                              (const R*)s->contrib, s->step, s->dt);
    else
        hipLaunchKernelGGL(k_particle<R>, dim3(nb), dim3(th), 0, s->stream, pa, (const R*)s->contrib, s->step,
                           s->dt);
}

static void launch_particle(ldpm_system* s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (s->prec == LDPM_PREC_MIXED) launch_particle_t<float>(s, ev0, ev1);
    else launch_particle_t<double>(s, ev0, ev1);
}

// Persistent launch: chunks of at most PERSIST_CHUNK steps per cooperative
// launch, grid = the number of blocks that fit on the chip at once.
constexpr int64_t PERSIST_CHUNK = 1024;

template <typename R, int LAW, int TB>
static hipError_t launch_persist_t(ldpm_system* s, int64_t nsteps)
{
    auto kern = k_persist<R, LAW, TB>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 12 * TB, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
    const int64_t nb = (s->T + TB - 1) / TB;
    const int64_t np = (s->N * PG + 12 * TB - 1) / (12 * TB);
    int64_t G = (int64_t)per_cu * s->n_cu;
    G = std::min<int64_t>(G, std::max<int64_t>(nb, np));
    NodeArgs na{s->tet, s->node, s->N, s->T};
    FacetArgs<R> fa{(const R*)s->cI, (const R*)s->area, s->rec, (const R*)s->frame, (R*)s->ht, (R*)s->hemax,
                    s->F, s->E};
    ProgArgs pr{s->prog_off, s->prog_t, s->prog_v, s->progv, s->n_prog};
    ParticleArgs pa{s->node, s->mass, s->inertia, s->mode, s->prog, s->scale, s->body,
                    s->fext, s->wext, s->wkin, s->ptr,     s->progv, s->flag, s->N};
    GridSync gs{s->bar, s->bar + 1, s->flag};
    MatDev<R> mat = *(const MatDev<R>*)(sizeof(R) == 8 ? (const void*)&s->matd : (const void*)&s->matf);
    const int32_t* pos = s->pos;
    R* contrib = (R*)s->contrib;
    double* wint = s->wint;
    double dt = s->dt;
    for (int64_t done = 0; done < nsteps;) {
        int64_t k = std::min<int64_t>(PERSIST_CHUNK, nsteps - done);
        int64_t step0 = s->step;
        SurrogateArgs sg = s->sg;
        CaptureArgs cp = s->cp;
        void* args[] = {&na, &fa, &mat, &pos, &contrib, &wint, &pr, &pa, &gs, &step0, &k, &dt, &sg, &cp};
        e = hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)G), dim3(12 * TB), args, 0, s->stream);
        if (e != hipSuccess) return e;
        s->step += k;
        done += k;
    }
    return hipSuccess;
}

template <typename R, int LAW>
static hipError_t launch_persist_l(ldpm_system* s, int64_t n)
{
    switch (s->launch.tets_per_block) {
    case 8: return launch_persist_t<R, LAW, 8>(s, n);
    case 32: return launch_persist_t<R, LAW, 32>(s, n);
    case 64: return launch_persist_t<R, LAW, 64>(s, n);
    default: return launch_persist_t<R, LAW, 16>(s, n);
    }
}

static hipError_t launch_persist(ldpm_system* s, int64_t n)
{
    if (s->prec == LDPM_PREC_MIXED)
        return s->law == 0 ? launch_persist_l<float, 0>(s, n) : launch_persist_l<float, 1>(s, n);
    return s->law == 0 ? launch_persist_l<double, 0>(s, n) : launch_persist_l<double, 1>(s, n);
}

// n steps in the configured launch shape
static hipError_t run_steps(ldpm_system* s, int64_t n)
{
    if (s->launch.persistent && !s->sg_on && !s->cp_on) return launch_persist(s, n);
    for (int64_t i = 0; i < n; i++) {
        launch_facet(s);
        launch_particle(s);
        s->step++;
    }
    return hipGetLastError();
}

extern "C" {

const char* ldpm_last_error(void) { return g_err.c_str(); }

ldpm_status ldpm_load_system(const ldpm_system_desc* d, ldpm_system** out)
{
    g_err.clear();
    if (!d || !out) return fail(LDPM_ERR_ARG, "null descriptor or output");
    *out = nullptr;
    const int64_t N = d->n_particles, T = d->n_tets, F = d->n_facets;
    if (N <= 0 || T <= 0) return fail(LDPM_ERR_ARG, "empty system (N=%lld, T=%lld)", (long long)N, (long long)T);
    if (F != 12 * T) return fail(LDPM_ERR_ARG, "n_facets (%lld) must be 12 * n_tets (%lld)", (long long)F, (long long)T);
    if (N >= (1ll << 31) || 4 * T >= (1ll << 31) || F >= (1ll << 40))
        return fail(LDPM_ERR_ARG, "system too large for 32-bit incidence indices");
    if (!d->x0 || !d->mass || !d->rot_inertia || !d->tet_nodes || !d->facet_I || !d->facet_J || !d->facet_cI ||
        !d->facet_n || !d->facet_m || !d->facet_area || !d->facet_len || !d->dof_mode || !d->dof_prog ||
        !d->dof_scale || !d->mat)
        return fail(LDPM_ERR_ARG, "missing required array");
    if (!(d->dt > 0) || !std::isfinite(d->dt)) return fail(LDPM_ERR_ARG, "dt must be positive and finite");
    if (d->precision != LDPM_PREC_FP64 && d->precision != LDPM_PREC_MIXED)
        return fail(LDPM_ERR_ARG, "unknown precision %d", d->precision);
    const ldpm_material& mat = *d->mat;
    if (mat.law != 0 && mat.law != 1) return fail(LDPM_ERR_ARG, "law must be 0 or 1");
    if (!(mat.E0 > 0) || !(mat.alpha > 0)) return fail(LDPM_ERR_ARG, "E0 and alpha must be positive");
    if (mat.law == 1) {
        if (mat.r_s != 0.0) return fail(LDPM_ERR_ARG, "r_s != 0 (shear softening of the cohesion) is not supported");
        if (!(mat.sigma_t > 0) || !(mat.r_st > 0) || !(mat.sigma_c0 > 0) || !(mat.sigma_N0 > 0) || !(mat.kc3 > 0))
            return fail(LDPM_ERR_ARG, "sigma_t, r_st, sigma_c0, sigma_N0 and kc3 must be positive");
    }
    const int nspec = d->n_specimens <= 0 ? 1 : d->n_specimens;
    std::vector<int64_t> poff(nspec + 1), toff(nspec + 1);
    if (nspec == 1 && (!d->particle_off || !d->tet_off)) {
        poff = {0, N};
        toff = {0, T};
    } else {
        if (!d->particle_off || !d->tet_off) return fail(LDPM_ERR_ARG, "batched system needs particle_off and tet_off");
        for (int i = 0; i <= nspec; i++) {
            poff[i] = d->particle_off[i];
            toff[i] = d->tet_off[i];
        }
        if (poff[0] != 0 || toff[0] != 0 || poff[nspec] != N || toff[nspec] != T)
            return fail(LDPM_ERR_ARG, "specimen offsets must start at 0 and end at N, T");
        for (int i = 0; i < nspec; i++)
            if (poff[i + 1] <= poff[i] || toff[i + 1] <= toff[i])
                return fail(LDPM_ERR_ARG, "specimen %d is empty", i);
    }
    // ---- validation of values and indices ----
    if (!finite_all(d->x0, 3 * N) || !finite_all(d->facet_cI, 3 * F) || !finite_all(d->facet_n, 3 * F) ||
        !finite_all(d->facet_m, 3 * F) || !finite_all(d->facet_area, F) || !finite_all(d->facet_len, F) ||
        !finite_all(d->dof_scale, 6 * N))
        return fail(LDPM_ERR_ARG, "non-finite geometry or loading input");
    for (int64_t i = 0; i < N; i++) {
        if (!(d->mass[i] > 0)) return fail(LDPM_ERR_ARG, "mass[%lld] must be positive", (long long)i);
        for (int c = 0; c < 3; c++)
            if (!(d->rot_inertia[c * N + i] > 0))
                return fail(LDPM_ERR_ARG, "rot_inertia of particle %lld must be positive", (long long)i);
    }
    // specimen of each particle (tets and facets must stay inside one specimen)
    std::vector<int32_t> spec_of(N);
    for (int s = 0; s < nspec; s++)
        for (int64_t i = poff[s]; i < poff[s + 1]; i++) spec_of[i] = s;
    for (int s = 0; s < nspec; s++)
        for (int64_t t = toff[s]; t < toff[s + 1]; t++)
            for (int a = 0; a < 4; a++) {
                const int64_t nd = d->tet_nodes[a * T + t];
                if (nd < 0 || nd >= N) return fail(LDPM_ERR_ARG, "tet %lld: node index out of range", (long long)t);
                if (spec_of[nd] != s) return fail(LDPM_ERR_ARG, "tet %lld crosses specimens", (long long)t);
            }
    const int64_t nP = d->n_programs;
    if (nP < 0 || (nP > 0 && (!d->prog_off || !d->prog_t || !d->prog_v)))
        return fail(LDPM_ERR_ARG, "programs: missing arrays");
    int64_t npts = 0;
    if (nP > 0) {
        if (d->prog_off[0] != 0) return fail(LDPM_ERR_ARG, "prog_off[0] must be 0");
        for (int64_t p = 0; p < nP; p++) {
            if (d->prog_off[p + 1] < d->prog_off[p]) return fail(LDPM_ERR_ARG, "prog_off must be non-decreasing");
            for (int64_t i = d->prog_off[p]; i + 1 < d->prog_off[p + 1]; i++)
                if (!(d->prog_t[i + 1] > d->prog_t[i])) return fail(LDPM_ERR_ARG, "program %lld: times must increase", (long long)p);
        }
        npts = d->prog_off[nP];
        if (!finite_all(d->prog_t, npts) || !finite_all(d->prog_v, npts)) return fail(LDPM_ERR_ARG, "non-finite program");
    }
    for (int64_t i = 0; i < 6 * N; i++) {
        if (d->dof_mode[i] > 1) return fail(LDPM_ERR_ARG, "dof_mode must be 0 or 1");
        if (d->dof_prog[i] < -1 || d->dof_prog[i] >= nP) return fail(LDPM_ERR_ARG, "dof_prog out of range");
    }
    // ---- facets: local codes and deduplicated edge frames ----
    std::vector<int32_t> rec(F);
    std::vector<double> en, em, el;
    std::unordered_map<FrameKey, int32_t, FrameHash> frames;
    frames.reserve((size_t)(F / 4 + 16));
    for (int64_t f = 0; f < F; f++) {
        const int64_t t = f / 12;
        const int32_t I = d->facet_I[f], J = d->facet_J[f];
        int aI = -1, aJ = -1;
        for (int a = 0; a < 4; a++) {
            if (d->tet_nodes[a * T + t] == I) aI = a;
            if (d->tet_nodes[a * T + t] == J) aJ = a;
        }
        if (aI < 0 || aJ < 0 || aI == aJ)
            return fail(LDPM_ERR_ARG, "facet %lld: I and J must be two distinct nodes of tet %lld", (long long)f, (long long)t);
        const double len = d->facet_len[f];
        if (!(len > 0)) return fail(LDPM_ERR_ARG, "facet %lld: non-positive length", (long long)f);
        if (mat.law == 1 && !(mat.l_t > len))
            return fail(LDPM_ERR_ARG, "facet %lld: l_t must exceed the edge length (H_t > 0)", (long long)f);
        FrameKey k;
        for (int c = 0; c < 3; c++) {
            k.v[c] = d->facet_n[c * F + f];
            k.v[3 + c] = d->facet_m[c * F + f];
        }
        k.v[6] = len;
        auto it = frames.find(k);
        int32_t r;
        if (it == frames.end()) {
            r = (int32_t)el.size();
            if (r >= (1 << 28)) return fail(LDPM_ERR_ARG, "too many distinct facet frames");
            frames.emplace(k, r);
            for (int c = 0; c < 3; c++) {
                en.push_back(k.v[c]);
                em.push_back(k.v[3 + c]);
            }
            el.push_back(len);
        } else {
            r = it->second;
        }
        rec[f] = (int32_t)((uint32_t)r | ((uint32_t)aI << 28) | ((uint32_t)aJ << 30));
    }
    const int64_t E = (int64_t)el.size();
    // ---- incidence CSR: slots 4t+a in ascending order ----
    std::vector<int32_t> ptr(N + 1, 0), slot(4 * T), pos(4 * T);
    for (int64_t t = 0; t < T; t++)
        for (int a = 0; a < 4; a++) ptr[d->tet_nodes[a * T + t] + 1]++;
    for (int64_t i = 0; i < N; i++) ptr[i + 1] += ptr[i];
    {
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t t = 0; t < T; t++)
            for (int a = 0; a < 4; a++) {
                const int32_t at = fill[d->tet_nodes[a * T + t]]++;
                slot[at] = (int32_t)(4 * t + a);
                pos[4 * t + a] = at;
            }
    }
    // ---- body force: constant generalised force V_I b, V_I r_I x b ----
    std::vector<double> body;
    if (d->body_force && (d->body_force[0] != 0 || d->body_force[1] != 0 || d->body_force[2] != 0)) {
        if (!d->cell_vol || !d->cell_r) return fail(LDPM_ERR_ARG, "body_force needs cell_vol and cell_r");
        const double* b = d->body_force;
        body.resize(6 * N);
        for (int64_t i = 0; i < N; i++) {
            const double V = d->cell_vol[i];
            const double r0 = d->cell_r[i], r1 = d->cell_r[N + i], r2 = d->cell_r[2 * N + i];
            body[0 * N + i] = V * b[0];
            body[1 * N + i] = V * b[1];
            body[2 * N + i] = V * b[2];
            body[3 * N + i] = V * (r1 * b[2] - r2 * b[1]);
            body[4 * N + i] = V * (r2 * b[0] - r0 * b[2]);
            body[5 * N + i] = V * (r0 * b[1] - r1 * b[0]);
        }
    }
    // ---- layout ----
    const int prec = d->precision;
    const size_t rb = rbytes(prec);
    Carve cv;
    const size_t o_node = cv.take<double>(16 * N);
    const size_t o_mass = cv.take<double>(N), o_in = cv.take<double>(3 * N), o_scale = cv.take<double>(6 * N);
    const size_t o_body = body.empty() ? 0 : cv.take<double>(6 * N);
    const size_t o_fext = cv.take<double>(6 * N), o_wext = cv.take<double>(N), o_wkin = cv.take<double>(N);
    const size_t o_wint = cv.take<double>(T), o_mode = cv.take<uint8_t>(6 * N), o_prog = cv.take<int32_t>(6 * N);
    const size_t o_ptr = cv.take<int32_t>(N + 1), o_tet = cv.take<int32_t>(4 * T);
    const size_t o_pos = cv.take<int32_t>(4 * T);
    const size_t o_rec = cv.take<int32_t>(F), o_flag = cv.take<int32_t>(4), o_bar = cv.take<unsigned>(4);
    const size_t o_poff = cv.take<int64_t>(nP + 1), o_pt = cv.take<double>(npts + 1), o_pv = cv.take<double>(npts + 1);
    const size_t o_red = cv.take<double>(8);
    const size_t o_progv = cv.take<double>(2 * nP + 2);
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_cI = cv.off; cv.off += 3 * F * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_area = cv.off; cv.off += F * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_frame = cv.off; cv.off += 8 * E * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_ht = cv.off; cv.off += 3 * F * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_hem = cv.off; cv.off += F * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_con = cv.off; cv.off += 4 * T * 6 * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t total = cv.off;

    ldpm_system* s = new ldpm_system();
    s->N = N; s->T = T; s->F = F; s->E = E; s->nspec = nspec; s->prec = prec; s->law = mat.law;
    s->poff = poff; s->toff = toff; s->dt = d->dt;
    s->stream = (hipStream_t)d->stream;
    s->dev_free = d->dev_alloc ? d->dev_free : nullptr;
    s->dev_alloc = d->dev_alloc;
    s->alloc_ctx = d->alloc_ctx;
    s->n_prog = nP; s->n_prog_pts = npts;
    s->matd = make_mat<double>(mat);
    s->matf = make_mat<float>(mat);
    (void)hipGetDevice(&s->device);
    (void)hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, s->device);
    void* base = nullptr;
    if (d->dev_alloc) {
        base = d->dev_alloc(total, d->alloc_ctx);
        if (!base) { delete s; return fail(LDPM_ERR_ALLOC, "device allocator returned NULL for %zu bytes", total); }
    } else {
        if (hipMalloc(&base, total) != hipSuccess) { delete s; return fail(LDPM_ERR_ALLOC, "hipMalloc(%zu) failed", total); }
    }
    s->arena = base;
    s->arena_bytes = total;
    char* B = (char*)base;
    s->node = (double*)(B + o_node);
    s->mass = (double*)(B + o_mass); s->inertia = (double*)(B + o_in); s->scale = (double*)(B + o_scale);
    s->body = body.empty() ? nullptr : (double*)(B + o_body);
    s->fext = (double*)(B + o_fext); s->wext = (double*)(B + o_wext); s->wkin = (double*)(B + o_wkin);
    s->wint = (double*)(B + o_wint); s->mode = (uint8_t*)(B + o_mode); s->prog = (int32_t*)(B + o_prog);
    s->ptr = (int32_t*)(B + o_ptr); s->tet = (int32_t*)(B + o_tet);
    s->pos = (int32_t*)(B + o_pos);
    s->rec = (int32_t*)(B + o_rec); s->flag = (int32_t*)(B + o_flag); s->bar = (unsigned*)(B + o_bar);
    s->prog_off = (int64_t*)(B + o_poff); s->prog_t = (double*)(B + o_pt); s->prog_v = (double*)(B + o_pv);
    s->red = (double*)(B + o_red);
    s->progv = (double*)(B + o_progv);
    s->cI = B + o_cI; s->area = B + o_area; s->frame = B + o_frame;
    s->ht = B + o_ht; s->hemax = B + o_hem; s->contrib = B + o_con;

    auto H2D = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s->stream);
    };
    std::vector<std::vector<unsigned char>> keep;  // host staging kept alive until sync
    auto put_r = [&](void* dst, const double* src, size_t n) -> hipError_t {
        keep.emplace_back();
        if (prec == LDPM_PREC_MIXED) to_r<float>(keep.back(), src, n);
        else to_r<double>(keep.back(), src, n);
        return H2D(dst, keep.back().data(), n * rb);
    };
    hipError_t e = hipSuccess;
    const ldpm_state* is = d->init_state;
    std::vector<double> zeros6(6 * N, 0.0);
    const double* q0 = (is && is->q) ? is->q : (d->q0 ? d->q0 : zeros6.data());
    const double* v0 = (is && is->v) ? is->v : (d->v0 ? d->v0 : zeros6.data());
    if (!finite_all(q0, 6 * N) || !finite_all(v0, 6 * N)) {
        ldpm_free(s);
        return fail(LDPM_ERR_ARG, "non-finite initial state");
    }
#define CK(x) do { e = (x); if (e != hipSuccess) { ldpm_free(s); return fail(LDPM_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e)); } } while (0)
    std::vector<double> nodes((size_t)16 * N, 0.0);
    for (int64_t i = 0; i < N; i++) {
        for (int c = 0; c < 6; c++) {
            nodes[16 * i + c] = q0[c * N + i];
            nodes[16 * i + 6 + c] = v0[c * N + i];
        }
        for (int c = 0; c < 3; c++) nodes[16 * i + 12 + c] = d->x0[c * N + i];
    }
    CK(H2D(s->node, nodes.data(), 16 * N * 8));
    CK(H2D(s->mass, d->mass, N * 8));
    CK(H2D(s->inertia, d->rot_inertia, 3 * N * 8));
    CK(H2D(s->scale, d->dof_scale, 6 * N * 8));
    if (s->body) CK(H2D(s->body, body.data(), 6 * N * 8));
    CK(H2D(s->mode, d->dof_mode, 6 * N));
    CK(H2D(s->prog, d->dof_prog, 6 * N * 4));
    CK(H2D(s->ptr, ptr.data(), (N + 1) * 4));
    CK(H2D(s->pos, pos.data(), 4 * T * 4));
    CK(H2D(s->tet, d->tet_nodes, 4 * T * 4));
    CK(H2D(s->rec, rec.data(), F * 4));
    std::vector<int64_t> po(nP + 1, 0);
    for (int64_t p = 0; p <= nP && nP > 0; p++) po[p] = d->prog_off[p];
    CK(H2D(s->prog_off, po.data(), (nP + 1) * 8));
    if (npts > 0) {
        CK(H2D(s->prog_t, d->prog_t, npts * 8));
        CK(H2D(s->prog_v, d->prog_v, npts * 8));
    }
    CK(put_r(s->cI, d->facet_cI, 3 * F));
    CK(put_r(s->area, d->facet_area, F));
    std::vector<double> frec((size_t)8 * E, 0.0);
    for (int64_t r = 0; r < E; r++) {
        for (int c = 0; c < 3; c++) {
            frec[8 * r + c] = en[3 * r + c];
            frec[8 * r + 3 + c] = em[3 * r + c];
        }
        frec[8 * r + 6] = el[r];
        frec[8 * r + 7] = 1.0 / el[r];
    }
    CK(put_r(s->frame, frec.data(), 8 * E));
    // history, accumulators
    std::vector<double> zF(3 * F, 0.0);
    CK(put_r(s->ht, (is && is->t) ? is->t : zF.data(), 3 * F));
    CK(put_r(s->hemax, (is && is->emax) ? is->emax : zF.data(), F));
    CK(H2D(s->fext, (is && is->fext) ? is->fext : zeros6.data(), 6 * N * 8));
    CK(H2D(s->wext, (is && is->w_ext) ? is->w_ext : zeros6.data(), N * 8));
    CK(H2D(s->wkin, (is && is->w_kin) ? is->w_kin : zeros6.data(), N * 8));
    std::vector<double> zT(T, 0.0);
    CK(H2D(s->wint, (is && is->w_int) ? is->w_int : zT.data(), T * 8));
    CK(hipMemsetAsync(s->flag, 0, 16, s->stream));
    CK(hipMemsetAsync(s->bar, 0, 16, s->stream));
    CK(hipMemsetAsync(s->contrib, 0, 4 * T * 6 * rb, s->stream));
#undef CK
    // initial kinetic energy per specimen, particle order then DoF order
    s->wkin0.assign(nspec, 0.0);
    if (is && is->w_kin0) {
        for (int i = 0; i < nspec; i++) s->wkin0[i] = is->w_kin0[i];
    } else {
        for (int sp = 0; sp < nspec; sp++) {
            double w = 0.0;
            for (int64_t i = poff[sp]; i < poff[sp + 1]; i++)
                for (int dd = 0; dd < 6; dd++) {
                    const double M = dd < 3 ? d->mass[i] : d->rot_inertia[(dd - 3) * N + i];
                    const double vv = v0[dd * N + i];
                    w += 0.5 * M * vv * vv;
                }
            s->wkin0[sp] = w;
        }
    }
    s->step = is ? is->step : 0;
    if (s->step < 0) { ldpm_free(s); return fail(LDPM_ERR_ARG, "negative step in init_state"); }
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { ldpm_free(s); return fail(LDPM_ERR_DEVICE, "upload sync failed: %s", hipGetErrorString(e)); }
    *out = s;
    return LDPM_OK;
}

ldpm_status ldpm_step(ldpm_system* s, int64_t n_steps)
{
    if (!s) return fail(LDPM_ERR_ARG, "null handle");
    if (n_steps < 0) return fail(LDPM_ERR_ARG, "negative step count");
    hipError_t e = run_steps(s, n_steps);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return LDPM_OK;
}

ldpm_status ldpm_step_profiled(ldpm_system* s, int64_t n_steps, double* facet_ms, double* particle_ms)
{
    if (!s || !facet_ms || !particle_ms) return fail(LDPM_ERR_ARG, "null argument");
    if (n_steps < 0) return fail(LDPM_ERR_ARG, "negative step count");
    constexpr int CH = 128;  // steps per chunk of events
    std::vector<hipEvent_t> ev(4 * CH);
    for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    double fsum = 0.0, psum = 0.0;
    hipError_t e = hipSuccess;
    for (int64_t done = 0; done < n_steps && e == hipSuccess;) {
        const int k = (int)std::min<int64_t>(CH, n_steps - done);
        for (int i = 0; i < k; i++) {
            launch_facet(s, ev[4 * i], ev[4 * i + 1]);
            launch_particle(s, ev[4 * i + 2], ev[4 * i + 3]);
            s->step++;
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(ev[4 * (k - 1) + 3]);
        for (int i = 0; i < k && e == hipSuccess; i++) {
            float a = 0.f, b = 0.f;
            e = hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[4 * i + 2], ev[4 * i + 3]);
            fsum += a;
            psum += b;
        }
        done += k;
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "profiled step failed: %s", hipGetErrorString(e));
    *facet_ms = fsum;
    *particle_ms = psum;
    return LDPM_OK;
}

ldpm_status ldpm_sync(ldpm_system* s)
{
    if (!s) return fail(LDPM_ERR_ARG, "null handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    int32_t flag[2] = {0, 0};
    HIP_TRY(hipMemcpy(flag, s->flag, 8, hipMemcpyDeviceToHost));
    if (flag[1]) return fail(LDPM_ERR_DEVICE, "persistent launch: a grid barrier timed out");
    if (flag[0]) return fail(LDPM_ERR_UNSTABLE, "non-finite velocity: the step is unstable");
    return LDPM_OK;
}

ldpm_status ldpm_read_state(ldpm_system* s, ldpm_state* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    ldpm_status st = ldpm_sync(s);
    if (st != LDPM_OK && st != LDPM_ERR_UNSTABLE) return st;
    const int64_t N = s->N, T = s->T, F = s->F;
    if (o->q || o->v) {
        std::vector<double> nodes((size_t)16 * N);
        HIP_TRY(hipMemcpy(nodes.data(), s->node, 16 * N * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < N; i++)
            for (int c = 0; c < 6; c++) {
                if (o->q) o->q[c * N + i] = nodes[16 * i + c];
                if (o->v) o->v[c * N + i] = nodes[16 * i + 6 + c];
            }
    }
    if (o->fext) HIP_TRY(hipMemcpy(o->fext, s->fext, 6 * N * 8, hipMemcpyDeviceToHost));
    if (o->w_int) HIP_TRY(hipMemcpy(o->w_int, s->wint, T * 8, hipMemcpyDeviceToHost));
    if (o->w_ext) HIP_TRY(hipMemcpy(o->w_ext, s->wext, N * 8, hipMemcpyDeviceToHost));
    if (o->w_kin) HIP_TRY(hipMemcpy(o->w_kin, s->wkin, N * 8, hipMemcpyDeviceToHost));
    if (o->w_kin0) for (int i = 0; i < s->nspec; i++) o->w_kin0[i] = s->wkin0[i];
    auto get_r = [&](double* dst, const void* src, size_t n) -> hipError_t {
        if (s->prec == LDPM_PREC_MIXED) {
            std::vector<float> tmp(n);
            hipError_t e = hipMemcpy(tmp.data(), src, n * 4, hipMemcpyDeviceToHost);
            for (size_t i = 0; i < n; i++) dst[i] = tmp[i];
            return e;
        }
        return hipMemcpy(dst, src, n * 8, hipMemcpyDeviceToHost);
    };
    if (o->t) HIP_TRY(get_r(o->t, s->ht, 3 * F));
    if (o->emax) HIP_TRY(get_r(o->emax, s->hemax, F));
    o->step = s->step;
    return st;
}

ldpm_status ldpm_energy(ldpm_system* s, int32_t sp, ldpm_energies* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    if (sp < 0 || sp >= s->nspec) return fail(LDPM_ERR_ARG, "specimen %d out of range", sp);
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(RED_THREADS), 0, s->stream, s->wint, s->toff[sp], s->toff[sp + 1],
                       s->wext, s->wkin, s->poff[sp], s->poff[sp + 1], s->red);
    HIP_TRY(hipGetLastError());
    ldpm_status st = ldpm_sync(s);
    if (st != LDPM_OK && st != LDPM_ERR_UNSTABLE) return st;
    double r[3];
    HIP_TRY(hipMemcpy(r, s->red, 24, hipMemcpyDeviceToHost));
    o->W_int = r[0];
    o->W_ext = r[1];
    o->W_kin = s->step > 0 ? r[2] : s->wkin0[sp];
    o->W_kin0 = s->wkin0[sp];
    const double den = std::max(std::fabs(o->W_ext + o->W_kin0), 1e-300);
    o->err = std::fabs(o->W_ext + o->W_kin0 - o->W_int - o->W_kin) / den;
    o->step = s->step;
    o->time = (double)(s->step > 0 ? s->step - 1 : 0) * s->dt;
    return st;
}

ldpm_status ldpm_reaction(ldpm_system* s, int32_t program, double* out)
{
    if (!s || !out) return fail(LDPM_ERR_ARG, "null argument");
    hipLaunchKernelGGL(k_reaction, dim3(1), dim3(RED_THREADS), 0, s->stream, s->fext, s->prog, 6 * s->N, program,
                       s->red + 4);
    HIP_TRY(hipGetLastError());
    ldpm_status st = ldpm_sync(s);
    if (st != LDPM_OK && st != LDPM_ERR_UNSTABLE) return st;
    HIP_TRY(hipMemcpy(out, s->red + 4, 8, hipMemcpyDeviceToHost));
    return st;
}

ldpm_status ldpm_get_info(ldpm_system* s, ldpm_info* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    const double rb = (double)rbytes(s->prec);
    o->n_particles = s->N;
    o->n_tets = s->T;
    o->n_facets = s->F;
    o->n_edges = s->E;
    o->n_specimens = s->nspec;
    o->step = s->step;
    o->precision = s->prec;
    o->law = s->law;
    const double N = (double)s->N, T = (double)s->T, F = (double)s->F, E = (double)s->E;
    // facet kernel: each array touched once per launch
    //   facets: rec 4 B + cI 3R + area R + history (t 3R + e_max R) read and written
    //   edge frames 8R per frame (n, m, l, 1/l); tets: nodes 16 B, pos 16 B,
    //   w_int 16 B (r+w), contributions written 24R; particles: x0, q, v read
    //   (15 doubles)
    const double hist = (s->law == 1 ? 4.0 : 3.0) * rb;
    o->facet_kernel_bytes = F * (4.0 + 4.0 * rb + 2.0 * hist) + E * 8.0 * rb + T * (16.0 + 16.0 + 16.0 + 24.0 * rb) +
                            N * 15.0 * 8.0;  // nodes: 15 of 16 words used
    // particle kernel: contributions 24R per tet read; per particle ptr 4 B,
    //   q, v, fext read + written (3 x 6 x 16 B), mass + inertia 32 B, scale 48 B,
    //   prog 24 B, mode 6 B, w_ext r+w 16 B, w_kin 8 B
    o->particle_kernel_bytes = T * 24.0 * rb + N * (4.0 + 288.0 + 32.0 + 48.0 + 24.0 + 6.0 + 16.0 + 8.0);
    o->device_bytes = s->arena_bytes;
    return LDPM_OK;
}

ldpm_status ldpm_set_launch(ldpm_system* s, const ldpm_launch* c)
{
    if (!s || !c) return fail(LDPM_ERR_ARG, "null argument");
    if (c->tets_per_block != 8 && c->tets_per_block != 16 && c->tets_per_block != 32 && c->tets_per_block != 64)
        return fail(LDPM_ERR_ARG, "tets_per_block must be 8, 16, 32 or 64");
    if (c->particle_threads < 64 || c->particle_threads > 1024 || c->particle_threads % 64)
        return fail(LDPM_ERR_ARG, "particle_threads must be a multiple of 64 in [64, 1024]");
    s->launch = *c;
    s->launch.xcd_remap = c->xcd_remap ? 1 : 0;
    s->launch.persistent = c->persistent ? 1 : 0;
    return LDPM_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times every launch shape on the live system and keeps the
// fastest.  The dynamic state is saved before the trials and restored after,
// and results do not depend on the launch shape, so tuning never changes the
// trajectory.  Choices are cached per (GPU architecture, system shape).
// ---------------------------------------------------------------------------
namespace {
struct TuneKey {
    std::string arch;
    int64_t N, T, F, E, nspec;
    int32_t prec, law;
    bool operator==(const TuneKey& o) const
    {
        return arch == o.arch && N == o.N && T == o.T && F == o.F && E == o.E && nspec == o.nspec &&
               prec == o.prec && law == o.law;
    }
};
struct TuneEntry {
    TuneKey key;
    ldpm_launch best;
    double us;
};
std::vector<TuneEntry> g_tune_cache;

struct Region {
    void* p;
    size_t bytes;
};

std::vector<Region> dynamic_regions(ldpm_system* s)
{
    const size_t rb = rbytes(s->prec);
    const size_t N = (size_t)s->N, T = (size_t)s->T, F = (size_t)s->F;
    return {{s->node, 16 * N * 8}, {s->fext, 6 * N * 8}, {s->wext, N * 8},
            {s->wkin, N * 8},  {s->wint, T * 8},    {s->ht, 3 * F * rb},  {s->hemax, F * rb}};
}
}  // namespace

ldpm_status ldpm_autotune(ldpm_system* s, int32_t steps_per_trial, ldpm_launch* best, double* best_us,
                          ldpm_tune_trial* trials, int32_t max_trials, int32_t* n_trials)
{
    if (!s) return fail(LDPM_ERR_ARG, "null handle");
    if (steps_per_trial <= 0) return fail(LDPM_ERR_ARG, "steps_per_trial must be positive");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, s->device));
    TuneKey key{prop.gcnArchName, s->N, s->T, s->F, s->E, s->nspec, s->prec, s->law};
    for (const auto& t : g_tune_cache)
        if (t.key == key) {
            s->launch = t.best;
            if (best) *best = t.best;
            if (best_us) *best_us = t.us;
            if (n_trials) *n_trials = 0;
            return LDPM_OK;
        }
    // save the dynamic state
    auto regs = dynamic_regions(s);
    size_t total = 0;
    for (auto& r : regs) total += (r.bytes + 255) & ~size_t(255);
    void* snap = nullptr;
    if (s->dev_alloc) snap = s->dev_alloc(total, s->alloc_ctx);
    else if (hipMalloc(&snap, total) != hipSuccess) snap = nullptr;
    if (!snap) return fail(LDPM_ERR_ALLOC, "autotune: cannot allocate %zu bytes for the state snapshot", total);
    auto copy_all = [&](bool save) -> hipError_t {
        size_t off = 0;
        for (auto& r : regs) {
            char* sp = (char*)snap + off;
            hipError_t e = save ? hipMemcpyAsync(sp, r.p, r.bytes, hipMemcpyDeviceToDevice, s->stream)
                                : hipMemcpyAsync(r.p, sp, r.bytes, hipMemcpyDeviceToDevice, s->stream);
            if (e != hipSuccess) return e;
            off += (r.bytes + 255) & ~size_t(255);
        }
        return hipSuccess;
    };
    const int64_t step0 = s->step;
    const ldpm_launch keep = s->launch;
    hipError_t e = copy_all(true);
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const int tbs[4] = {8, 16, 32, 64};
    const int pts[4] = {64, 128, 256, 512};
    std::vector<ldpm_launch> cands;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++)
            for (int rm = 0; rm < 2; rm++) cands.push_back(ldpm_launch{tbs[i], pts[j], rm, 0});
    for (int i = 0; i < 4; i++) cands.push_back(ldpm_launch{tbs[i], 256, 0, 1});
    double best_t = 1e300;
    ldpm_launch best_l = keep;
    int32_t nt = 0;
    for (size_t ci = 0; ci < cands.size() && e == hipSuccess; ci++) {
        s->launch = cands[ci];
        e = copy_all(false);
        s->step = step0;
        if (e == hipSuccess) e = run_steps(s, 5);  // warm-up: instruction caches, clocks
        if (e == hipSuccess) e = hipEventRecord(a, s->stream);
        if (e == hipSuccess) e = run_steps(s, steps_per_trial);
        if (e == hipSuccess) e = hipEventRecord(b, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        const double us = 1e3 * ms / steps_per_trial;
        if (trials && nt < max_trials) trials[nt] = ldpm_tune_trial{s->launch, us};
        nt++;
        if (us < best_t) {
            best_t = us;
            best_l = s->launch;
        }
    }
    // restore the state, keep the winner
    if (e == hipSuccess) e = copy_all(false);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    s->step = step0;
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (s->dev_alloc) s->dev_free(snap, s->alloc_ctx);
    else (void)hipFree(snap);
    if (e != hipSuccess) {
        s->launch = keep;
        return fail(LDPM_ERR_DEVICE, "autotune failed: %s", hipGetErrorString(e));
    }
    int32_t flag[2] = {0, 0};
    HIP_TRY(hipMemcpy(flag, s->flag, 8, hipMemcpyDeviceToHost));
    if (flag[1]) return fail(LDPM_ERR_DEVICE, "autotune: a persistent grid barrier timed out");
    if (flag[0]) {  // a trial went non-finite: the restored state is clean, clear the flag
        HIP_TRY(hipMemset(s->flag, 0, 4));
    }
    s->launch = best_l;
    g_tune_cache.push_back(TuneEntry{key, best_l, best_t});
    if (best) *best = best_l;
    if (best_us) *best_us = best_t;
    if (n_trials) *n_trials = nt;
    return LDPM_OK;
}

ldpm_status ldpm_set_surrogate(ldpm_system* s, const ldpm_surrogate* g)
{
    if (!s) return fail(LDPM_ERR_ARG, "null handle");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->sg_mem) (void)hipFree(s->sg_mem);
    s->sg_mem = nullptr;
    s->sg_on = false;
    s->sg = SurrogateArgs{};
    if (!g) return LDPM_OK;
    if (s->prec != LDPM_PREC_MIXED || s->law != 1)
        return fail(LDPM_ERR_STATE, "the surrogate replaces the FP32 facet law: needs precision MIXED and law 1");
    if (!g->params) return fail(LDPM_ERR_ARG, "surrogate: null parameters");
    for (int k = 0; k < MLP_NPARAM; k++)
        if (!std::isfinite(g->params[k])) return fail(LDPM_ERR_ARG, "surrogate: non-finite parameter %d", k);
    const size_t pbytes = ((size_t)MLP_NPARAM * 4 + 255) & ~size_t(255);
    if (hipMalloc(&s->sg_mem, pbytes + (size_t)s->F) != hipSuccess) {
        s->sg_mem = nullptr;
        return fail(LDPM_ERR_ALLOC, "surrogate: allocation failed");
    }
    SurrogateArgs a{};
    a.params = (const float*)s->sg_mem;
    a.flag = (uint8_t*)((char*)s->sg_mem + pbytes);
    for (int k = 0; k < MLP_IN; k++) {
        a.xmean[k] = g->x_mean[k];
        a.xscale[k] = g->x_scale[k];
        a.lo[k] = g->box_lo[k];
        a.hi[k] = g->box_hi[k];
    }
    for (int k = 0; k < MLP_OUT; k++) {
        if (!(std::isfinite(g->y_dead[k]) && g->y_dead[k] >= 0.f))
            return fail(LDPM_ERR_ARG, "surrogate: y_dead[%d] must be finite and >= 0", k);
        a.yscale[k] = g->y_scale[k];
        a.ydead[k] = g->y_dead[k];
    }
    if (!(std::isfinite(g->y_tau) && g->y_tau >= 0.f)) return fail(LDPM_ERR_ARG, "surrogate: y_tau must be finite and >= 0");
    a.ytau = g->y_tau;
    a.gate = GateArgs{g->kappa_t, g->kappa_c, g->damage_max};
    HIP_TRY(hipMemcpyAsync((void*)a.params, g->params, (size_t)MLP_NPARAM * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemsetAsync(a.flag, 0, (size_t)s->F, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->sg = a;
    s->sg_on = true;
    return LDPM_OK;
}

ldpm_status ldpm_surrogate_count(ldpm_system* s, int64_t* n_exact)
{
    if (!s || !n_exact) return fail(LDPM_ERR_ARG, "null argument");
    if (!s->sg_on) return fail(LDPM_ERR_STATE, "no surrogate installed");
    HIP_TRY(hipStreamSynchronize(s->stream));
    std::vector<uint8_t> f((size_t)s->F);
    HIP_TRY(hipMemcpy(f.data(), s->sg.flag, (size_t)s->F, hipMemcpyDeviceToHost));
    int64_t c = 0;
    for (uint8_t v : f) c += v != 0;
    *n_exact = c;
    return LDPM_OK;
}

ldpm_status ldpm_capture_begin(ldpm_system* s, const ldpm_capture_opts* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    if (s->prec != LDPM_PREC_FP64 || s->law != 1)
        return fail(LDPM_ERR_STATE, "capture records the FP64 full law: needs precision FP64 and law 1");
    if (o->capacity <= 0 || o->facet_stride <= 0 || o->step_stride <= 0 || o->facet_offset < 0 ||
        o->facet_offset >= o->facet_stride)
        return fail(LDPM_ERR_ARG, "capture: bad options");
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->cp_mem) (void)hipFree(s->cp_mem);
    s->cp_mem = nullptr;
    const size_t rows = (size_t)o->capacity * 16 * 4;
    if (hipMalloc(&s->cp_mem, rows + 256) != hipSuccess) {
        s->cp_mem = nullptr;
        return fail(LDPM_ERR_ALLOC, "capture: allocation of %zu bytes failed", rows);
    }
    CaptureArgs c{};
    c.rows = (float*)s->cp_mem;
    c.count = (unsigned*)((char*)s->cp_mem + rows);
    c.cap = o->capacity;
    c.fstride = o->facet_stride;
    c.foff = o->facet_offset;
    c.sstride = o->step_stride;
    c.gate = GateArgs{o->kappa_t, o->kappa_c, o->damage_max};
    HIP_TRY(hipMemsetAsync(c.count, 0, 4, s->stream));
    s->cp = c;
    s->cp_on = true;
    return LDPM_OK;
}

ldpm_status ldpm_capture_end(ldpm_system* s, float* rows, int64_t max_rows, int64_t* n_rows)
{
    if (!s || !n_rows) return fail(LDPM_ERR_ARG, "null argument");
    if (!s->cp_on) return fail(LDPM_ERR_STATE, "no capture in progress");
    HIP_TRY(hipStreamSynchronize(s->stream));
    unsigned cnt = 0;
    HIP_TRY(hipMemcpy(&cnt, s->cp.count, 4, hipMemcpyDeviceToHost));
    const int64_t n = std::min<int64_t>((int64_t)cnt, s->cp.cap);
    *n_rows = (int64_t)cnt;
    if (rows && max_rows > 0)
        HIP_TRY(hipMemcpy(rows, s->cp.rows, (size_t)std::min(n, max_rows) * 16 * 4, hipMemcpyDeviceToHost));
    (void)hipFree(s->cp_mem);
    s->cp_mem = nullptr;
    s->cp_on = false;
    s->cp = CaptureArgs{};
    return LDPM_OK;
}

ldpm_status ldpm_get_launch(ldpm_system* s, ldpm_launch* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    *o = s->launch;
    return LDPM_OK;
}

void ldpm_free(ldpm_system* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    if (s->sg_mem) (void)hipFree(s->sg_mem);
    if (s->cp_mem) (void)hipFree(s->cp_mem);
    if (s->arena) {
        (void)hipStreamSynchronize(s->stream);
        if (s->dev_free) s->dev_free(s->arena, s->alloc_ctx);
        else (void)hipFree(s->arena);
    }
    delete s;
}

}  // extern "C"
