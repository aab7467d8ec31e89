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
//   edge frames records [E] of 8 R (n[3], m[3], len, 1/len): one 64-byte
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
#include <mutex>
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

#include "step_kernels.hpp"
#include "fields.hpp"
#include "implicit.hpp"
#include "tessellate.hpp"
#include "bound.hpp"
#include "stream_ref.hpp"

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
    ldpm_launch launch{16, 256, 1, 0, 0};
    int n_cu = 0;
    // device pointers
    double *node, *mass, *inertia, *scale, *body, *fext, *wext, *wkin, *wint;
    uint8_t* mode;
    int32_t *prog, *ptr, *pos, *tet, *rec, *flag;
    unsigned* bar;
    int64_t* prog_off;
    double *prog_t, *prog_v, *progv, *red;
    double* mblk = nullptr;  // full cell mass blocks [N][72] (M rows, then G rows), or none
    void *geo, *frame, *hist, *contrib;  // geo, hist: quad layout (quad_index)
    int64_t n_prog_pts = 0, n_prog = 0;
    MatDev<double> matd;
    MatDev<float> matf;
    // surrogate (mixed precision, full law) and training-sample capture (FP64)
    bool sg_on = false, cp_on = false;
    SurrogateArgs sg{};
    CaptureArgs cp{};
    void* sg_mem = nullptr;  // params + flags
    void* cp_mem = nullptr;  // rows + counter
    // random perturbations: work per specimen, device staging (jump [6][N],
    // e_V [T], jump work [T], per-specimen sums)
    std::vector<double> wpert;
    void* pt_mem = nullptr;
    // implicit HHT-alpha integrator (device buffers allocated at its first call)
    bool imp_on = false;
    double imp_dt = 0.0, imp_am = 0.0, imp_af = 0.0;
    void* im_mem = nullptr;
    double *im_q, *im_qn, *im_vn, *im_an, *im_gn, *im_fn, *im_f1, *im_vp, *im_g, *im_R, *im_M, *im_binv;
    double *cg_x, *cg_r, *cg_z, *cg_p, *cg_Ap, *cg_sc, *cg_part, *im_red;
    double *im_node_p, *im_ht_scr, *im_wint_scr, *im_con_scr, *im_ht_c, *im_wint_c;  // histories: quads
    int cg_prev_its = 0;  // iterations of the last CG solve (schedules the host's convergence checks)
};

namespace {

// [3][F] values and one [F] value (NULL: zeros) in the quad layout of the
// given precision (quad_index), as doubles before the conversion to R
std::vector<double> to_quads(const double* v3, const double* v1, int64_t F, int prec)
{
    std::vector<double> q(4 * (size_t)F);
    const bool f32 = prec == LDPM_PREC_MIXED;
    for (int64_t f = 0; f < F; f++)
        for (int j = 0; j < 4; j++)
            q[f32 ? quad_index<float>(F, f, j) : quad_index<double>(F, f, j)] =
                j < 3 ? (v3 ? v3[j * F + f] : 0.0) : (v1 ? v1[f] : 0.0);
    return q;
}

// the inverse: quads -> [3][F] and [F] (either may be NULL)
void from_quads(const std::vector<double>& q, double* v3, double* v1, int64_t F, int prec)
{
    const bool f32 = prec == LDPM_PREC_MIXED;
    for (int64_t f = 0; f < F; f++)
        for (int j = 0; j < 4; j++) {
            const double v = q[f32 ? quad_index<float>(F, f, j) : quad_index<double>(F, f, j)];
            if (j < 3 && v3) v3[j * F + f] = v;
            if (j == 3 && v1) v1[f] = v;
        }
}

// bytes the facet kernel moves per launch, each array touched once:
//   facets: rec 4 B + geometry quad (c^I 3R, area R) + history quad (t 3R,
//   e_max R) read and written; edge frames 8R per frame (n, m, l, 1/l);
//   tets: nodes 16 B, pos 16 B, w_int 16 B (r+w), contributions written 24R;
//   particles: x0, q, v read (15 of the record's 16 doubles)
double facet_kernel_bytes(int64_t N, int64_t T, int64_t F, int64_t E, size_t rb)
{
    return (double)F * (4.0 + 4.0 * rb + 2.0 * 4.0 * rb) + (double)E * 8.0 * rb +
           (double)T * (16.0 + 16.0 + 16.0 + 24.0 * rb) + (double)N * 15.0 * 8.0;
}

// above this many bytes per launch the facet streams bypass the caches by
// default (the MI355X's last-level Infinity Cache holds 256 MiB)
constexpr double STREAM_FACETS_BYTES = 256.0 * 1024 * 1024;

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

// Cholesky factor L (lower) of the sub-block of A on the index set idx (n
// entries; idx == nullptr: the leading n x n block); false unless positive
// definite
bool cholesky_sub(const double A[6][6], const int* idx, int n, double L[6][6])
{
    for (int r = 0; r < n; r++)
        for (int c = 0; c <= r; c++) {
            const int ir = idx ? idx[r] : r, ic = idx ? idx[c] : c;
            double acc = A[ir][ic];
            for (int k = 0; k < c; k++) acc -= L[r][k] * L[c][k];
            if (r == c) {
                if (!(acc > 0.0)) return false;
                L[r][r] = std::sqrt(acc);
            } else {
                L[r][c] = acc / L[c][c];
            }
        }
    return true;
}

bool spd_ok(const double A[6][6], const int* idx, int n)
{
    double L[6][6];
    return cholesky_sub(A, idx, n, L);
}

// G = inverse of A over the free index set fr (nf entries), embedded in
// 6 x 6 with zero rows and columns elsewhere
bool spd_inverse(const double A[6][6], const int* fr, int nf, double G[6][6])
{
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) G[r][c] = 0.0;
    if (nf == 0) return true;
    double L[6][6];
    if (!cholesky_sub(A, fr, nf, L)) return false;
    for (int j = 0; j < nf; j++) {  // column j of the inverse: L L^T x = e_j
        double y[6], x[6];
        for (int r = 0; r < nf; r++) {
            double acc = (r == j) ? 1.0 : 0.0;
            for (int k = 0; k < r; k++) acc -= L[r][k] * y[k];
            y[r] = acc / L[r][r];
        }
        for (int r = nf - 1; r >= 0; r--) {
            double acc = y[r];
            for (int k = r + 1; k < nf; k++) acc -= L[k][r] * x[k];
            x[r] = acc / L[r][r];
        }
        for (int r = 0; r < nf; r++) G[fr[r]][fr[j]] = x[r];
    }
    return true;
}

}  // namespace

// Kernel launches.  With events (ev0, ev1) the launch is made with
// hipExtLaunchKernelGGL, whose start/stop events are timestamped by the
// dispatch itself (the kernel's own duration, as a profiler reports it).
template <typename R, int LAW, int TB, int MODE>
static void launch_facet_m(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    NodeArgs na{s->tet, s->node, s->N, s->T};
    FacetArgs<R> fa{(const R*)s->geo, s->rec, (const R*)s->frame, (R*)s->hist, s->F, s->E};
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
    // the two-kernel step's facet streams: nontemporal (NT = 1) or cached
    auto kern = k_facet<R, LAW, TB, MODE, 0>;
    if constexpr (MODE == MODE_PLAIN)
        if (s->launch.stream_facets) kern = k_facet<R, LAW, TB, MODE, 1>;
    if (ev0)
        hipExtLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(12 * TB), 0, s->stream, ev0, ev1, 0, na, fa, mat,
                              (const int32_t*)s->pos, (R*)s->contrib, s->wint, pr, s->step, s->dt,
                              s->launch.xcd_remap, s->sg, s->cp);
    else
        hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(12 * TB), 0, s->stream, na, fa, mat,
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

template <typename R, int FULLM>
static void launch_particle_t(ldpm_system* s, hipEvent_t ev0, hipEvent_t ev1)
{
    ParticleArgs pa{s->node, s->mass, s->inertia, s->mode, s->prog, s->scale, s->body,
                    s->fext, s->wext, s->wkin, s->ptr,     s->progv, s->flag, s->N, s->mblk};
    const int th = s->launch.particle_threads;
    const unsigned nb = (unsigned)((s->N * PG + th - 1) / th);
    if (ev0)
        hipExtLaunchKernelGGL((k_particle<R, FULLM>), dim3(nb), dim3(th), 0, s->stream, ev0, ev1, 0, pa,
                              (const R*)s->contrib, s->step, s->dt);
    else
        hipLaunchKernelGGL((k_particle<R, FULLM>), dim3(nb), dim3(th), 0, s->stream, pa, (const R*)s->contrib,
                           s->step, s->dt);
}

static void launch_particle(ldpm_system* s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    if (s->prec == LDPM_PREC_MIXED) {
        if (s->mblk) launch_particle_t<float, 1>(s, ev0, ev1);
        else launch_particle_t<float, 0>(s, ev0, ev1);
    } else {
        if (s->mblk) launch_particle_t<double, 1>(s, ev0, ev1);
        else launch_particle_t<double, 0>(s, ev0, ev1);
    }
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
    FacetArgs<R> fa{(const R*)s->geo, s->rec, (const R*)s->frame, (R*)s->hist, s->F, s->E};
    ProgArgs pr{s->prog_off, s->prog_t, s->prog_v, s->progv, s->n_prog};
    ParticleArgs pa{s->node, s->mass, s->inertia, s->mode, s->prog, s->scale, s->body,
                    s->fext, s->wext, s->wkin, s->ptr,     s->progv, s->flag, s->N, s->mblk};
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
    // full cell mass blocks: symmetric positive definite, and so is every
    // free-DoF sub-block (Cholesky); G = inverse over the free DoFs
    std::vector<double> mblk;
    if (d->mass_block) {
        if (!finite_all(d->mass_block, 21 * N)) return fail(LDPM_ERR_ARG, "non-finite mass_block");
        mblk.assign((size_t)72 * N, 0.0);
        for (int64_t i = 0; i < N; i++) {
            double Mb[6][6];
            for (int r = 0, k = 0; r < 6; r++)
                for (int c = r; c < 6; c++, k++) Mb[r][c] = Mb[c][r] = d->mass_block[k * N + i];
            int fr[6], nf = 0;
            for (int dd = 0; dd < 6; dd++)
                if (d->dof_mode[dd * N + i] == 0) fr[nf++] = dd;
            if (!spd_ok(Mb, nullptr, 6))
                return fail(LDPM_ERR_ARG, "mass_block of particle %lld is not positive definite", (long long)i);
            double G[6][6];
            if (!spd_inverse(Mb, fr, nf, G))
                return fail(LDPM_ERR_ARG, "mass_block of particle %lld: free-DoF block not positive definite",
                            (long long)i);
            for (int r = 0; r < 6; r++)
                for (int c = 0; c < 6; c++) {
                    mblk[(size_t)72 * i + 6 * r + c] = Mb[r][c];
                    mblk[(size_t)72 * i + 36 + 6 * r + c] = G[r][c];
                }
        }
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
    const size_t o_red = cv.take<double>(8 + 3 * RED_MAX_BLOCKS);  // results, then reduction partials
    const size_t o_mblk = mblk.empty() ? 0 : cv.take<double>(72 * N);
    const size_t o_progv = cv.take<double>(2 * nP + 2);
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_geo = cv.off; cv.off += 4 * F * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_frame = cv.off; cv.off += 8 * E * rb;
    cv.off = (cv.off + 255) & ~size_t(255);
    const size_t o_hist = cv.off; cv.off += 4 * F * rb;
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
    s->launch.stream_facets = facet_kernel_bytes(N, T, F, E, rb) > STREAM_FACETS_BYTES ? 1 : 0;
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
    s->mblk = mblk.empty() ? nullptr : (double*)(B + o_mblk);
    s->progv = (double*)(B + o_progv);
    s->geo = B + o_geo; s->frame = B + o_frame;
    s->hist = B + o_hist; s->contrib = B + o_con;

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
    if (s->mblk) CK(H2D(s->mblk, mblk.data(), 72 * N * 8));
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
    {
        const std::vector<double> q = to_quads(d->facet_cI, d->facet_area, F, prec);
        CK(put_r(s->geo, q.data(), 4 * F));
    }
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
    {
        const std::vector<double> q = to_quads(is ? is->t : nullptr, is ? is->emax : nullptr, F, prec);
        CK(put_r(s->hist, q.data(), 4 * F));
    }
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
                    const double vv = v0[dd * N + i];
                    if (!mblk.empty()) {
                        double mv = 0.0;
                        for (int k = 0; k < 6; k++) mv += mblk[(size_t)72 * i + 6 * dd + k] * v0[k * N + i];
                        w += 0.5 * vv * mv;
                    } else {
                        const double M = dd < 3 ? d->mass[i] : d->rot_inertia[(dd - 3) * N + i];
                        w += 0.5 * M * vv * vv;
                    }
                }
            s->wkin0[sp] = w;
        }
    }
    s->wpert.assign(nspec, 0.0);
    if (is && is->w_pert)
        for (int i = 0; i < nspec; i++) s->wpert[i] = is->w_pert[i];
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
    if (s->imp_on) return fail(LDPM_ERR_STATE, "the handle integrates implicitly (ldpm_implicit_step)");
    hipError_t e = run_steps(s, n_steps);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return LDPM_OK;
}

ldpm_status ldpm_step_profiled(ldpm_system* s, int64_t n_steps, double* facet_ms, double* particle_ms)
{
    if (!s || !facet_ms || !particle_ms) return fail(LDPM_ERR_ARG, "null argument");
    if (n_steps < 0) return fail(LDPM_ERR_ARG, "negative step count");
    if (s->imp_on) return fail(LDPM_ERR_STATE, "the handle integrates implicitly (ldpm_implicit_step)");
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
    if (o->w_pert) for (int i = 0; i < s->nspec; i++) o->w_pert[i] = s->wpert[i];
    auto get_r = [&](double* dst, const void* src, size_t n) -> hipError_t {
        if (s->prec == LDPM_PREC_MIXED) {
            std::vector<float> tmp(n);
            hipError_t e = hipMemcpy(tmp.data(), src, n * 4, hipMemcpyDeviceToHost);
            for (size_t i = 0; i < n; i++) dst[i] = tmp[i];
            return e;
        }
        return hipMemcpy(dst, src, n * 8, hipMemcpyDeviceToHost);
    };
    if (o->t || o->emax) {
        std::vector<double> q(4 * (size_t)F);
        HIP_TRY(get_r(q.data(), s->hist, 4 * F));
        from_quads(q, o->t, o->emax, F, s->prec);
    }
    o->step = s->step;
    return st;
}

// grid of the two-stage reductions: one block per RED_THREADS elements, at most RED_MAX_BLOCKS
static int red_blocks(int64_t n)
{
    return (int)std::max<int64_t>(1, std::min<int64_t>(RED_MAX_BLOCKS, (n + RED_THREADS - 1) / RED_THREADS));
}

ldpm_status ldpm_energy(ldpm_system* s, int32_t sp, ldpm_energies* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    if (sp < 0 || sp >= s->nspec) return fail(LDPM_ERR_ARG, "specimen %d out of range", sp);
    {
        const int64_t n = std::max(s->toff[sp + 1] - s->toff[sp], s->poff[sp + 1] - s->poff[sp]);
        const int G = red_blocks(n);
        hipLaunchKernelGGL(k_energy_part, dim3(G), dim3(RED_THREADS), 0, s->stream, s->wint, s->toff[sp],
                           s->toff[sp + 1], s->wext, s->wkin, s->poff[sp], s->poff[sp + 1], s->red + 8);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RED_THREADS), 0, s->stream, (const double*)(s->red + 8), G, 3,
                           s->red);
    }
    HIP_TRY(hipGetLastError());
    ldpm_status st = ldpm_sync(s);
    if (st != LDPM_OK && st != LDPM_ERR_UNSTABLE) return st;
    double r[3];
    HIP_TRY(hipMemcpy(r, s->red, 24, hipMemcpyDeviceToHost));
    o->W_int = r[0];
    o->W_ext = r[1];
    o->W_kin = s->step > 0 ? r[2] : s->wkin0[sp];
    o->W_kin0 = s->wkin0[sp];
    o->W_pert = s->wpert[sp];
    const double src = o->W_ext + o->W_pert + o->W_kin0;
    o->err = std::fabs(src - o->W_int - o->W_kin) / std::max(std::fabs(src), 1e-300);
    o->step = s->step;
    o->time = s->imp_on ? (double)s->step * s->imp_dt : (double)(s->step > 0 ? s->step - 1 : 0) * s->dt;
    return st;
}

ldpm_status ldpm_reaction(ldpm_system* s, int32_t program, double* out)
{
    if (!s || !out) return fail(LDPM_ERR_ARG, "null argument");
    {
        const int G = red_blocks(6 * s->N);
        hipLaunchKernelGGL(k_reaction_part, dim3(G), dim3(RED_THREADS), 0, s->stream, s->fext, s->prog, 6 * s->N,
                           program, s->red + 8);
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RED_THREADS), 0, s->stream, (const double*)(s->red + 8), G, 1,
                           s->red + 4);
    }
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
    o->facet_kernel_bytes = facet_kernel_bytes(s->N, s->T, s->F, s->E, (size_t)rb);
    // particle kernel: contributions 24R per tet read; per particle ptr 4 B,
    //   q, v, fext read + written (3 x 6 x 16 B), mass + inertia 32 B, scale 48 B,
    //   prog 24 B, mode 6 B, w_ext r+w 16 B, w_kin 8 B
    o->particle_kernel_bytes = T * 24.0 * rb + N * (4.0 + 288.0 + 32.0 + 48.0 + 24.0 + 6.0 + 16.0 + 8.0);
    if (s->mblk) o->particle_kernel_bytes += N * 576.0;  // mass block M and G
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
    if (c->persistent && s->mblk)
        return fail(LDPM_ERR_ARG, "the persistent launch supports the lumped diagonal mass only");
    s->launch = *c;
    s->launch.xcd_remap = c->xcd_remap ? 1 : 0;
    s->launch.persistent = c->persistent ? 1 : 0;
    s->launch.stream_facets = c->stream_facets ? 1 : 0;
    return LDPM_OK;
}

// ---------------------------------------------------------------------------
// autotuner: times every launch shape on the live system and keeps the
// fastest.  The dynamic state is saved before the trials and restored after,
// and results do not depend on the launch shape, so tuning never changes the
// trajectory.  Choices are cached per (GPU architecture, system shape).
// ---------------------------------------------------------------------------
extern "C++" {
namespace {
struct TuneKey {
    std::string arch;
    int64_t N, T, F, E, nspec;
    int32_t prec, law, fullm;
    bool operator==(const TuneKey& o) const
    {
        return arch == o.arch && N == o.N && T == o.T && F == o.F && E == o.E && nspec == o.nspec &&
               prec == o.prec && law == o.law && fullm == o.fullm;
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
            {s->wkin, N * 8},  {s->wint, T * 8},    {s->hist, 4 * F * rb}};
}
}  // namespace
}  // extern "C++"

ldpm_status ldpm_autotune(ldpm_system* s, int32_t steps_per_trial, ldpm_launch* best, double* best_us,
                          ldpm_tune_trial* trials, int32_t max_trials, int32_t* n_trials)
{
    if (!s) return fail(LDPM_ERR_ARG, "null handle");
    if (steps_per_trial <= 0) return fail(LDPM_ERR_ARG, "steps_per_trial must be positive");
    // the trial steps restore only the plain step's state: the surrogate's
    // sticky hand-back flags and a capture's rows would keep the trials'
    // traces, so tuning is refused while either is active
    if (s->sg_on) return fail(LDPM_ERR_STATE, "autotune: a surrogate is installed (tune before ldpm_set_surrogate)");
    if (s->cp_on) return fail(LDPM_ERR_STATE, "autotune: a sample capture is active");
    if (s->imp_on) return fail(LDPM_ERR_STATE, "autotune: the handle integrates implicitly");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, s->device));
    TuneKey key{prop.gcnArchName, s->N, s->T, s->F, s->E, s->nspec, s->prec, s->law, s->mblk ? 1 : 0};
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
            for (int rm = 0; rm < 2; rm++) cands.push_back(ldpm_launch{tbs[i], pts[j], rm, 0, keep.stream_facets});
    if (!s->mblk)
        for (int i = 0; i < 4; i++) cands.push_back(ldpm_launch{tbs[i], 256, 0, 1, keep.stream_facets});
    double best_t = 1e300;
    ldpm_launch best_l = keep;
    int32_t nt = 0;
    auto trial = [&](const ldpm_launch& l) {
        s->launch = l;
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
    };
    for (size_t ci = 0; ci < cands.size() && e == hipSuccess; ci++) trial(cands[ci]);
    // the facet streams' cache policy, at the best shape
    if (e == hipSuccess) {
        ldpm_launch l = best_l;
        l.stream_facets = !l.stream_facets;
        trial(l);
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
    const size_t cbytes = 256;  // counters
    if (hipMalloc(&s->sg_mem, pbytes + cbytes + (size_t)s->F) != hipSuccess) {
        s->sg_mem = nullptr;
        return fail(LDPM_ERR_ALLOC, "surrogate: allocation failed");
    }
    SurrogateArgs a{};
    a.params = (const float*)s->sg_mem;
    a.stats = (unsigned long long*)((char*)s->sg_mem + pbytes);
    a.flag = (uint8_t*)((char*)s->sg_mem + pbytes + cbytes);
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
    HIP_TRY(hipMemsetAsync(a.stats, 0, cbytes + (size_t)s->F, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->sg = a;
    s->sg_on = true;
    return LDPM_OK;
}

ldpm_status ldpm_surrogate_stats(ldpm_system* s, ldpm_surrogate_counts* o)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    if (!s->sg_on) return fail(LDPM_ERR_STATE, "no surrogate installed");
    int64_t n = 0;
    ldpm_status st = ldpm_surrogate_count(s, &n);
    if (st != LDPM_OK) return st;
    unsigned long long c[SG_NSTATS] = {};
    HIP_TRY(hipMemcpy(c, s->sg.stats, sizeof(c), hipMemcpyDeviceToHost));
    o->handed_back = n;
    o->network_updates = (int64_t)c[0];
    o->damaged_updates = (int64_t)c[1];
    o->damaged_network_updates = (int64_t)c[2];
    o->handed_back_envelope = (int64_t)c[3];
    o->handed_back_box = (int64_t)c[4];
    o->handed_back_damage = (int64_t)c[5];
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

// ---------------------------------------------------------------------------
// crack openings, volumetric strains, field comparison, random perturbation
// ---------------------------------------------------------------------------
extern "C++" {
namespace {
// is p device memory of the given device?  (clears the error a host pointer
// leaves behind)
bool on_device(const void* p, int device)
{
    hipPointerAttribute_t a;
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == device;
}

unsigned blocks_for(int64_t n, int th) { return (unsigned)((n + th - 1) / th); }

template <typename R>
FacetArgs<R> facet_args(ldpm_system* s)
{
    return FacetArgs<R>{(const R*)s->geo, s->rec, (const R*)s->frame, (R*)s->hist, s->F, s->E};
}
}  // namespace
}  // extern "C++"

ldpm_status ldpm_crack_opening(ldpm_system* s, double* w)
{
    if (!s || !w) return fail(LDPM_ERR_ARG, "null argument");
    if (!on_device(w, s->device)) return fail(LDPM_ERR_ARG, "crack_opening: w must be device memory of the handle's GPU");
    NodeArgs na{s->tet, s->node, s->N, s->T};
    const double E0 = s->matd.E0, aE0 = s->matd.aE0;
    const int first = s->step == 0;
    // explicit: the last law evaluation was at q^n - dt v^{n-1/2};
    // implicit: at the committed q_n itself
    const double dtl = s->imp_on ? 0.0 : s->dt;
    if (s->prec == LDPM_PREC_MIXED)
        hipLaunchKernelGGL((k_crack<float, 16>), dim3(blocks_for(s->T, 16)), dim3(192), 0, s->stream, na,
                           facet_args<float>(s), E0, aE0, dtl, first, w);
    else
        hipLaunchKernelGGL((k_crack<double, 16>), dim3(blocks_for(s->T, 16)), dim3(192), 0, s->stream, na,
                           facet_args<double>(s), E0, aE0, dtl, first, w);
    HIP_TRY(hipGetLastError());
    return LDPM_OK;
}

ldpm_status ldpm_volumetric_strain(ldpm_system* s, double* ev)
{
    if (!s || !ev) return fail(LDPM_ERR_ARG, "null argument");
    if (!on_device(ev, s->device))
        return fail(LDPM_ERR_ARG, "volumetric_strain: ev must be device memory of the handle's GPU");
    NodeArgs na{s->tet, s->node, s->N, s->T};
    hipLaunchKernelGGL(k_volstrain, dim3(blocks_for(s->T, 256)), dim3(256), 0, s->stream, na,
                       s->imp_on ? 0.0 : s->dt, (int)(s->step == 0), (const double*)nullptr, ev);
    HIP_TRY(hipGetLastError());
    return LDPM_OK;
}

}  // extern "C"

// Buffer of the field comparison: CMP_MAX_BLOCKS block partials, then the
// 7 results (and one spare double).
constexpr size_t CMP_BUF_BYTES = (size_t)CMP_MAX_BLOCKS * sizeof(Moments) + 8 * sizeof(double);

// The allocation-free entry point's copy of that buffer: one per GPU, held by
// the process.  On the host `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress (cmp_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[CMP_BUF_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mtx;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// device address of `scratch` on GPU dev (the current device), resolved on
// the first call per device and kept
ldpm_status cmp_scratch_ptr(int dev, void** out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(LDPM_ERR_DEVICE, "compare_fields_noalloc: device %d beyond the %d supported", dev,
                    SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mtx);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LDPM_ERR_DEVICE, "compare_fields_noalloc: hipGetSymbolAddress failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LDPM_OK;
}

ldpm_status cmp_check(const double* x, const double* ref, int64_t n, ldpm_field_stats* out, int* dev)
{
    if (!x || !ref || !out) return fail(LDPM_ERR_ARG, "null argument");
    if (n <= 0) return fail(LDPM_ERR_ARG, "compare_fields: n must be positive");
    HIP_TRY(hipGetDevice(dev));
    if (!on_device(x, *dev) || !on_device(ref, *dev))
        return fail(LDPM_ERR_ARG, "compare_fields: x and ref must be device memory of the current GPU");
    return LDPM_OK;
}

// the comparison proper, on a buffer of CMP_BUF_BYTES device bytes
ldpm_status cmp_run(const double* x, const double* ref, int64_t n, double cap, hipStream_t st, void* mem,
                    ldpm_field_stats* out)
{
    const int G = (int)std::min<int64_t>(CMP_MAX_BLOCKS, (n + CMP_THREADS - 1) / CMP_THREADS);
    Moments* part = (Moments*)mem;
    double* res = (double*)((char*)mem + (size_t)CMP_MAX_BLOCKS * sizeof(Moments));
    const int use_cap = (cap > 0.0 && std::isfinite(cap)) ? 1 : 0;
    hipLaunchKernelGGL(k_cmp_partial, dim3(G), dim3(CMP_THREADS), 0, st, x, ref, n, cap, use_cap, part);
    hipLaunchKernelGGL(k_cmp_final, dim3(1), dim3(CMP_THREADS), 0, st, (const Moments*)part, G, res);
    hipError_t e = hipGetLastError();
    double r[7] = {0, 0, 0, 0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "compare_fields failed: %s", hipGetErrorString(e));
    out->n = (int64_t)r[0];
    out->mean_x = r[1];
    out->mean_ref = r[2];
    out->pearson = r[3];
    out->rmse = r[4];
    out->ref_max = r[5];
    out->nrmse = r[6];
    return LDPM_OK;
}
}  // namespace

extern "C" {

ldpm_status ldpm_compare_fields(const double* x, const double* ref, int64_t n, double cap, void* stream,
                                ldpm_field_stats* out)
{
    int dev = 0;
    ldpm_status stc = cmp_check(x, ref, n, out, &dev);
    if (stc != LDPM_OK) return stc;
    // one buffer per device (partials and result), kept for the process;
    // calls are serialised (each waits for its stream before returning)
    static std::mutex mtx;
    static std::unordered_map<int, void*> bufs;
    std::lock_guard<std::mutex> lock(mtx);
    void*& mem = bufs[dev];
    if (!mem && hipMalloc(&mem, CMP_BUF_BYTES) != hipSuccess) {
        mem = nullptr;
        return fail(LDPM_ERR_ALLOC, "compare_fields: hipMalloc(%zu) failed", CMP_BUF_BYTES);
    }
    return cmp_run(x, ref, n, cap, (hipStream_t)stream, mem, out);
}

ldpm_status ldpm_stream_probe(int kind, const void* src, void* dst, int64_t bytes, void* stream)
{
    if (kind < LDPM_STREAM_COPY || kind > LDPM_STREAM_MIX)
        return fail(LDPM_ERR_ARG, "stream_probe: unknown kind %d", kind);
    // bytes moved per 16-byte element of each stream
    const int64_t unit = kind == LDPM_STREAM_MIX ? 80 : (kind == LDPM_STREAM_COPY ? 32 : 16);
    if (bytes <= 0 || bytes % unit != 0)
        return fail(LDPM_ERR_ARG, "stream_probe: bytes must be a positive multiple of %lld", (long long)unit);
    if ((kind != LDPM_STREAM_FILL && !src) || !dst)
        return fail(LDPM_ERR_ARG, "stream_probe: null buffer");
    if ((kind != LDPM_STREAM_FILL && ((uintptr_t)src & 15)) || ((uintptr_t)dst & 15))
        return fail(LDPM_ERR_ARG, "stream_probe: buffers must be 16-byte aligned");
    const int64_t n = bytes / unit;  // elements per stream
    const int64_t blocks = (n + STREAM_THREADS - 1) / STREAM_THREADS;
    if (blocks > 0x7fffffffll) return fail(LDPM_ERR_ARG, "stream_probe: bytes too large");
    hipStream_t st = (hipStream_t)stream;
    const auto* a = (const stream_d2*)src;
    auto* b = (stream_d2*)dst;
    switch (kind) {
    case LDPM_STREAM_COPY: k_stream_copy<<<(unsigned)blocks, STREAM_THREADS, 0, st>>>(a, b, n); break;
    case LDPM_STREAM_READ: k_stream_read<<<(unsigned)blocks, STREAM_THREADS, 0, st>>>(a, (double*)dst, n); break;
    case LDPM_STREAM_FILL: k_stream_fill<<<(unsigned)blocks, STREAM_THREADS, 0, st>>>(b, n); break;
    default: k_stream_mix<<<(unsigned)blocks, STREAM_THREADS, 0, st>>>(a, b, n); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "stream_probe: %s", hipGetErrorString(e));
    return LDPM_OK;
}

ldpm_status ldpm_compare_fields_noalloc(const double* x, const double* ref, int64_t n, double cap, void* stream,
                                        ldpm_field_stats* out)
{
    int dev = 0;
    ldpm_status stc = cmp_check(x, ref, n, out, &dev);
    if (stc != LDPM_OK) return stc;
    // the partials of any n fit: the grid is capped at CMP_MAX_BLOCKS blocks
    static_assert((size_t)CMP_MAX_BLOCKS * sizeof(Moments) + 7 * sizeof(double) <= sizeof(scratch),
                  "comparison scratch");
    void* mem = nullptr;
    stc = cmp_scratch_ptr(dev, &mem);
    if (stc != LDPM_OK) return stc;
    return cmp_run(x, ref, n, cap, (hipStream_t)stream, mem, out);
}

extern "C++" template <typename R, int LAW>
static void launch_jump(ldpm_system* s, const double* d, const double* evj, double* wj)
{
    NodeArgs na{s->tet, s->node, s->N, s->T};
    const MatDev<R>& mat = *(const MatDev<R>*)(sizeof(R) == 8 ? (const void*)&s->matd : (const void*)&s->matf);
    hipLaunchKernelGGL((k_jump<R, LAW>), dim3(blocks_for(s->T, 256)), dim3(256), 0, s->stream, na, facet_args<R>(s),
                       mat, d, evj, s->dt, s->wint, wj);
}

ldpm_status ldpm_perturb(ldpm_system* s, const double* delta, double* work)
{
    if (!s || !delta) return fail(LDPM_ERR_ARG, "null argument");
    if (s->imp_on) return fail(LDPM_ERR_STATE, "perturbations apply to explicit runs");
    const int64_t N = s->N, T = s->T;
    if (!finite_all(delta, 6 * N)) return fail(LDPM_ERR_ARG, "perturb: non-finite delta");
    Carve cv;
    const size_t o_d = cv.take<double>(6 * N), o_ev = cv.take<double>(T), o_wj = cv.take<double>(T);
    const size_t o_sum = cv.take<double>(s->nspec);
    const size_t bytes = (cv.off + 255) & ~size_t(255);
    if (!s->pt_mem && hipMalloc(&s->pt_mem, bytes) != hipSuccess) {
        s->pt_mem = nullptr;
        return fail(LDPM_ERR_ALLOC, "perturb: hipMalloc(%zu) failed", bytes);
    }
    char* B = (char*)s->pt_mem;
    double *d = (double*)(B + o_d), *evj = (double*)(B + o_ev), *wj = (double*)(B + o_wj);
    double* sums = (double*)(B + o_sum);
    HIP_TRY(hipMemcpyAsync(d, delta, 6 * N * 8, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(k_mask_free, dim3(blocks_for(6 * N, 256)), dim3(256), 0, s->stream, s->mode, 6 * N, d);
    std::vector<double> w(s->nspec, 0.0);
    if (s->step > 0) {
        NodeArgs na{s->tet, s->node, s->N, s->T};
        hipLaunchKernelGGL(k_volstrain, dim3(blocks_for(T, 256)), dim3(256), 0, s->stream, na, s->dt, 0,
                           (const double*)d, evj);
        if (s->prec == LDPM_PREC_MIXED) {
            if (s->law == 0) launch_jump<float, 0>(s, d, evj, wj);
            else launch_jump<float, 1>(s, d, evj, wj);
        } else {
            if (s->law == 0) launch_jump<double, 0>(s, d, evj, wj);
            else launch_jump<double, 1>(s, d, evj, wj);
        }
        for (int sp = 0; sp < s->nspec; sp++)
            hipLaunchKernelGGL(k_range_sum, dim3(1), dim3(RED_THREADS), 0, s->stream, (const double*)wj, s->toff[sp],
                               s->toff[sp + 1], sums + sp);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(w.data(), sums, s->nspec * 8, hipMemcpyDeviceToHost, s->stream));
    }
    hipLaunchKernelGGL(k_add_jump, dim3(blocks_for(6 * N, 256)), dim3(256), 0, s->stream, s->node, (const double*)d, N);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    double tot = 0.0;
    for (int sp = 0; sp < s->nspec; sp++) {
        s->wpert[sp] += w[sp];
        tot += w[sp];
    }
    if (work) *work = tot;
    return LDPM_OK;
}

// ---------------------------------------------------------------------------
// implicit generalised-alpha / HHT-alpha integration (modified Newton on the initial elastic
// stiffness, inner solves by Jacobi-preconditioned conjugate gradients with
// the stiffness applied matrix-free by the facet kernel of the elastic law)
// ---------------------------------------------------------------------------
extern "C++" {
namespace {
unsigned im_blocks(int64_t n) { return (unsigned)std::min<int64_t>(IM_MAX_BLOCKS, (n + IM_THREADS - 1) / IM_THREADS); }

template <int LAW, int TB>
void launch_facet_plain(ldpm_system* s, const NodeArgs& na, const FacetArgs<double>& fa, double* contrib,
                        double* wint, const ProgArgs& pr, int64_t step, double dt)
{
    const MatDev<double>& mat = s->matd;
    const int64_t nb = (s->T + TB - 1) / TB;
    hipLaunchKernelGGL((k_facet<double, LAW, TB, MODE_PLAIN>), dim3((unsigned)nb), dim3(12 * TB), 0, s->stream, na,
                       fa, mat, (const int32_t*)s->pos, contrib, wint, pr, step, dt, s->launch.xcd_remap,
                       SurrogateArgs{}, CaptureArgs{});
}

template <int LAW>
void launch_facet_plain_l(ldpm_system* s, const NodeArgs& na, const FacetArgs<double>& fa, double* contrib,
                          double* wint, const ProgArgs& pr, int64_t step, double dt)
{
    switch (s->launch.tets_per_block) {
    case 8: launch_facet_plain<LAW, 8>(s, na, fa, contrib, wint, pr, step, dt); break;
    case 32: launch_facet_plain<LAW, 32>(s, na, fa, contrib, wint, pr, step, dt); break;
    case 64: launch_facet_plain<LAW, 64>(s, na, fa, contrib, wint, pr, step, dt); break;
    default: launch_facet_plain<LAW, 16>(s, na, fa, contrib, wint, pr, step, dt); break;
    }
}

hipError_t im_alloc(ldpm_system* s)
{
    const int64_t N = s->N, T = s->T, F = s->F;
    Carve cv;
    const size_t n6 = 6 * N;
    size_t o[32];
    int k = 0;
    for (int i = 0; i < 11; i++) o[k++] = cv.take<double>(n6);     // im_* vectors
    o[k++] = cv.take<double>(36 * (size_t)N);                       // inverse particle blocks
    for (int i = 0; i < 5; i++) o[k++] = cv.take<double>(n6);      // cg x r z p Ap
    o[k++] = cv.take<double>(16);                                   // cg_sc
    o[k++] = cv.take<double>(3 * (size_t)IM_MAX_BLOCKS);            // cg_part (partials)
    o[k++] = cv.take<double>(8);                                    // im_red
    o[k++] = cv.take<double>(16 * N);                               // node_p
    o[k++] = cv.take<double>(4 * F);                                // history scratch (quads)
    o[k++] = cv.take<double>(T);                                    // wint scratch
    o[k++] = cv.take<double>(24 * T);                               // contrib scratch
    o[k++] = cv.take<double>(4 * F);                                // committed history (quads)
    o[k++] = cv.take<double>(T);                                    // committed w_int
    const size_t bytes = (cv.off + 255) & ~size_t(255);
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, bytes);
    if (e != hipSuccess) return e;
    s->im_mem = mem;
    char* B = (char*)mem;
    double** vec[12] = {&s->im_q, &s->im_qn, &s->im_vn, &s->im_an, &s->im_gn, &s->im_fn, &s->im_f1,
                        &s->im_vp, &s->im_g, &s->im_R, &s->im_M, &s->im_binv};
    k = 0;
    for (int i = 0; i < 12; i++) *vec[i] = (double*)(B + o[k++]);
    double** cgv[5] = {&s->cg_x, &s->cg_r, &s->cg_z, &s->cg_p, &s->cg_Ap};
    for (int i = 0; i < 5; i++) *cgv[i] = (double*)(B + o[k++]);
    s->cg_sc = (double*)(B + o[k++]);
    s->cg_part = (double*)(B + o[k++]);
    s->im_red = (double*)(B + o[k++]);
    s->im_node_p = (double*)(B + o[k++]);
    s->im_ht_scr = (double*)(B + o[k++]);
    s->im_wint_scr = (double*)(B + o[k++]);
    s->im_con_scr = (double*)(B + o[k++]);
    s->im_ht_c = (double*)(B + o[k++]);
    s->im_wint_c = (double*)(B + o[k++]);
    return hipSuccess;
}

ProgArgs prog_args(ldpm_system* s) { return ProgArgs{s->prog_off, s->prog_t, s->prog_v, s->progv, s->n_prog}; }

// g = -f_int(q) from the committed history: trial node records, history
// restored from the committed copies, facet kernel (dt = 1: the strain
// increment is e(q) - e(q_n); first: from the undeformed state), gather
hipError_t im_trial(ldpm_system* s, const double* q, int first)
{
    const int64_t N = s->N, T = s->T, F = s->F;
    hipLaunchKernelGGL(k_im_nodes, dim3(blocks_for(6 * N, 256)), dim3(256), 0, s->stream, s->node, q,
                       (const double*)s->im_qn, N);
    hipError_t e = hipMemcpyAsync(s->hist, s->im_ht_c, 4 * F * 8, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->wint, s->im_wint_c, T * 8, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return e;
    NodeArgs na{s->tet, s->node, N, T};
    const FacetArgs<double> fa = facet_args<double>(s);
    const ProgArgs pr = prog_args(s);
    if (s->law == 0) launch_facet_plain_l<0>(s, na, fa, (double*)s->contrib, s->wint, pr, first ? 0 : 1, 1.0);
    else launch_facet_plain_l<1>(s, na, fa, (double*)s->contrib, s->wint, pr, first ? 0 : 1, 1.0);
    hipLaunchKernelGGL(k_im_gather<double>, dim3(blocks_for(N * PG, 256)), dim3(256), 0, s->stream,
                       (const int32_t*)s->ptr, (const double*)s->contrib, N, s->im_g);
    return hipGetLastError();
}

// tet-node records of -K0 p for the p in the q slots of node_p (elastic law
// on scratch history); k_cg_gather_apply sums them per particle
void im_k0_facets(ldpm_system* s)
{
    NodeArgs na{s->tet, s->im_node_p, s->N, s->T};
    FacetArgs<double> fa = facet_args<double>(s);
    fa.hist = s->im_ht_scr;
    const ProgArgs pr{s->prog_off, s->prog_t, s->prog_v, s->progv, 0};
    launch_facet_plain_l<0>(s, na, fa, s->im_con_scr, s->im_wint_scr, pr, 1, 1.0);
}

// x = K_eff^{-1} R on the free DoFs; returns the iterations
hipError_t im_cg(ldpm_system* s, double cM, double cK, double tol, int max_it, int* its)
{
    const int64_t N = s->N;
    const int G = (int)im_blocks(6 * N);
    CgArgs cg{s->mode, s->im_M, s->im_binv, s->cg_x, s->cg_r, s->cg_z, s->cg_p, s->cg_Ap, s->cg_sc, s->cg_part,
              cM, cK, N};
    hipLaunchKernelGGL(k_cg_init, dim3(G), dim3(IM_THREADS), 0, s->stream, cg, (const double*)s->im_R, s->im_node_p);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(IM_THREADS), 0, s->stream, cg, G, 1);
    double sc[8];
    hipError_t e = hipMemcpyAsync(sc, s->cg_sc, 64, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return e;
    const double rr0 = sc[4];
    // partials: p.Ap of the gather-apply grid, then r.z and r.r of the update grid
    const int GA = (int)std::min<int64_t>(IM_MAX_BLOCKS, blocks_for(N * PG, 256));
    const int GU = (int)std::min<int64_t>(IM_MAX_BLOCKS, blocks_for(N * CG_LANES, IM_THREADS));
    double* partA = s->cg_part;
    double* partB = s->cg_part + IM_MAX_BLOCKS;
    // the host reads r.r (a stream synchronisation) every 8 iterations, and
    // every 2 from one iteration before the previous solve's count for the
    // next 8: successive solves need similar counts.  The schedule depends
    // only on the handle's own history, so runs stay reproducible.
    const int start = std::max(1, s->cg_prev_its - 1);
    auto check_due = [&](int k) {
        if (k == max_it) return true;
        if (k >= start && k <= start + 8) return (k - start) % 2 == 0;
        return k % 8 == 0;
    };
    int it = 0, par = 0;
    if (rr0 > 0.0) {
        while (it < max_it) {
            im_k0_facets(s);
            hipLaunchKernelGGL(k_cg_gather_apply<double>, dim3(GA), dim3(256), 0, s->stream, cg,
                               (const int32_t*)s->ptr, (const double*)s->im_con_scr, partA);
            hipLaunchKernelGGL(k_cg_update, dim3(GU), dim3(IM_THREADS), 0, s->stream, cg, (const double*)partA, GA,
                               partB, par);
            it++;
            if (check_due(it)) {
                hipLaunchKernelGGL(k_cg_rr, dim3(1), dim3(IM_THREADS), 0, s->stream, cg, (const double*)partB, GU);
                e = hipMemcpyAsync(sc, s->cg_sc, 64, hipMemcpyDeviceToHost, s->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
                if (e != hipSuccess) return e;
                if (!(sc[3] > tol * tol * rr0)) break;
            }
            hipLaunchKernelGGL(k_cg_newp, dim3(G), dim3(IM_THREADS), 0, s->stream, cg, (const double*)partB, GU,
                               s->im_node_p, par);
            par ^= 1;
        }
    }
    *its = it;
    s->cg_prev_its = it;
    return hipGetLastError();
}

// |R_F|, |(M a)_F| + |rhs_F| of the trial q
hipError_t im_residual(ldpm_system* s, const ImArgs& ia, double* res, double* ref)
{
    const int G = (int)im_blocks(6 * s->N);
    hipLaunchKernelGGL(k_im_residual, dim3(G), dim3(IM_THREADS), 0, s->stream, ia, (const double*)s->im_q,
                       (const double*)s->im_g, s->im_R, s->cg_part);
    hipLaunchKernelGGL(k_im_reduce3, dim3(1), dim3(IM_THREADS), 0, s->stream, (const double*)s->cg_part, G, s->im_red);
    double r[3];
    hipError_t e = hipMemcpyAsync(r, s->im_red, 24, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    *res = std::sqrt(r[0]);
    *ref = std::sqrt(r[1]) + std::sqrt(r[2]);
    return e;
}
}  // namespace
}  // extern "C++"

ldpm_status ldpm_implicit_step(ldpm_system* s, const ldpm_implicit_opts* o, int64_t n_steps,
                               ldpm_implicit_stats* stats)
{
    if (!s || !o) return fail(LDPM_ERR_ARG, "null argument");
    if (n_steps < 0) return fail(LDPM_ERR_ARG, "negative step count");
    if (s->prec != LDPM_PREC_FP64) return fail(LDPM_ERR_ARG, "the implicit integrator runs in FP64 only");
    if (s->mblk) return fail(LDPM_ERR_ARG, "the implicit integrator takes the lumped diagonal mass only");
    if (s->sg_on || s->cp_on) return fail(LDPM_ERR_STATE, "surrogate or capture active");
    if (!(o->dt > 0) || !std::isfinite(o->dt)) return fail(LDPM_ERR_ARG, "implicit dt must be positive");
    if (!(o->alpha_m >= -1.0 && o->alpha_m <= o->alpha_f + 1e-15 && o->alpha_f <= 0.5 + 1e-15))
        return fail(LDPM_ERR_ARG, "alpha_m <= alpha_f <= 1/2 and alpha_m >= -1 are required");
    if (!(o->tol > 0) || o->max_iter < 1 || !(o->cg_tol > 0) || o->cg_max_iter < 1)
        return fail(LDPM_ERR_ARG, "tolerances and iteration limits must be positive");
    if (!s->imp_on && s->step > 0) return fail(LDPM_ERR_STATE, "explicit steps were taken on this handle");
    if (s->imp_on && (o->dt != s->imp_dt || o->alpha_m != s->imp_am || o->alpha_f != s->imp_af))
        return fail(LDPM_ERR_ARG, "dt, alpha_m and alpha_f are fixed after the first implicit step");
    const int64_t N = s->N, T = s->T, F = s->F;
    const double dt = o->dt, am = o->alpha_m, af = o->alpha_f;
    const double be = (1.0 - am + af) * (1.0 - am + af) / 4.0, ga = 0.5 - am + af;
    const double cM = (1.0 - am) / (be * dt * dt), cK = 1.0 - af;
    hipError_t e = hipSuccess;
    if (!s->im_mem) {
        e = im_alloc(s);
        if (e != hipSuccess) return fail(LDPM_ERR_ALLOC, "implicit: device allocation failed: %s", hipGetErrorString(e));
    }
    const int64_t n6 = 6 * N;
    const unsigned b6 = blocks_for(n6, 256);
    ImArgs ia{s->mode, s->im_M, s->im_qn, s->im_vn, s->im_an, s->im_gn, s->im_fn, s->im_f1, dt, am, af, be, ga, N};
    if (!s->imp_on) {
        // committed state from the node records, lumped masses, and the
        // preconditioner: inverse 6 x 6 particle blocks of K_eff (the K0
        // blocks per tet node and their per-particle sums live in a
        // temporary buffer)
        hipLaunchKernelGGL(k_im_unpack, dim3(b6), dim3(256), 0, s->stream, (const double*)s->node, N, s->im_qn, s->im_vn);
        for (int d = 0; d < 3; d++) HIP_TRY(hipMemcpyAsync(s->im_M + d * N, s->mass, N * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync(s->im_M + 3 * N, s->inertia, 3 * N * 8, hipMemcpyDeviceToDevice, s->stream));
        {
            double* blk = nullptr;
            const size_t nb = (84 * (size_t)T + 21 * (size_t)N) * 8;
            if (hipMalloc((void**)&blk, nb) != hipSuccess)
                return fail(LDPM_ERR_ALLOC, "implicit: hipMalloc(%zu) for the preconditioner failed", nb);
            double* blk_p = blk + 84 * (size_t)T;
            hipLaunchKernelGGL(k_im_block_k0<double>, dim3(blocks_for(4 * T, 256)), dim3(256), 0, s->stream,
                               facet_args<double>(s), (const int32_t*)s->pos, T, s->matd.E0, s->matd.alpha, blk);
            hipLaunchKernelGGL((k_im_gather<double, 21>), dim3(blocks_for(N * PG, 256)), dim3(256), 0, s->stream,
                               (const int32_t*)s->ptr, (const double*)blk, N, blk_p);
            hipLaunchKernelGGL(k_im_block_inv, dim3(blocks_for(N, 256)), dim3(256), 0, s->stream,
                               (const double*)s->im_M, s->mode, (const double*)blk_p, cM, cK, N, s->im_binv);
            hipError_t eb = hipGetLastError();
            if (eb == hipSuccess) eb = hipStreamSynchronize(s->stream);
            (void)hipFree(blk);
            if (eb != hipSuccess) return fail(LDPM_ERR_DEVICE, "implicit: preconditioner: %s", hipGetErrorString(eb));
        }
        HIP_TRY(hipMemcpyAsync(s->im_node_p, s->node, 16 * N * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipMemsetAsync(s->cg_Ap, 0, n6 * 8, s->stream));
        hipLaunchKernelGGL(k_im_nodes, dim3(b6), dim3(256), 0, s->stream, s->im_node_p, (const double*)s->cg_Ap, nullptr, N);
        HIP_TRY(hipMemsetAsync(s->im_ht_scr, 0, 4 * F * 8, s->stream));
        HIP_TRY(hipMemsetAsync(s->im_wint_scr, 0, T * 8, s->stream));
        HIP_TRY(hipMemcpyAsync(s->im_ht_c, s->hist, 4 * F * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync(s->im_wint_c, s->wint, T * 8, hipMemcpyDeviceToDevice, s->stream));
        // a_0 from M a_0 = g(q_0) + f(0) on the free DoFs
        e = im_trial(s, s->im_qn, s->step == 0);
        if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "implicit: %s", hipGetErrorString(e));
        const ProgArgs pr = prog_args(s);
        const double t0 = (double)s->step * dt;
        hipLaunchKernelGGL(k_im_loads, dim3(b6), dim3(256), 0, s->stream, s->mode, s->prog, s->scale,
                           (const double*)s->body, pr, t0, t0, n6, s->im_fn, (double*)nullptr);
        hipLaunchKernelGGL(k_im_init_acc, dim3(b6), dim3(256), 0, s->stream, ia, (const double*)s->im_g, s->im_an,
                           s->im_gn, s->fext);
        HIP_TRY(hipGetLastError());
        // the trial left its history in place: back to the committed one
        HIP_TRY(hipMemcpyAsync(s->hist, s->im_ht_c, 4 * F * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync(s->wint, s->im_wint_c, T * 8, hipMemcpyDeviceToDevice, s->stream));
        hipLaunchKernelGGL(k_im_pack, dim3(b6), dim3(256), 0, s->stream, s->node, (const double*)s->im_qn,
                           (const double*)s->im_vn, N);
        s->imp_on = true;
        s->imp_dt = dt;
        s->imp_am = am;
        s->imp_af = af;
    }
    int64_t newton = 0, cgits = 0, notconv = 0;
    double maxres = 0.0;
    const ProgArgs pr = prog_args(s);
    for (int64_t it = 0; it < n_steps; it++) {
        const double tn = (double)s->step * dt;
        const int first = s->step == 0;
        hipLaunchKernelGGL(k_im_loads, dim3(b6), dim3(256), 0, s->stream, s->mode, s->prog, s->scale,
                           (const double*)s->body, pr, tn + dt, tn + 0.5 * dt, n6, s->im_f1, s->im_vp);
        hipLaunchKernelGGL(k_im_predict, dim3(b6), dim3(256), 0, s->stream, s->mode, (const double*)s->im_qn,
                           (const double*)s->im_vn, (const double*)s->im_an, (const double*)s->im_vp, dt, n6, s->im_q);
        int k = 0;
        double res = 0.0, ref = 0.0;
        while (true) {
            e = im_trial(s, s->im_q, first);
            if (e == hipSuccess) e = im_residual(s, ia, &res, &ref);
            if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "implicit: %s", hipGetErrorString(e));
            if (!std::isfinite(res)) return fail(LDPM_ERR_UNSTABLE, "implicit: non-finite residual");
            if (res <= o->tol * ref || k == o->max_iter) break;
            int its = 0;
            e = im_cg(s, cM, cK, o->cg_tol, o->cg_max_iter, &its);
            if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "implicit CG: %s", hipGetErrorString(e));
            cgits += its;
            hipLaunchKernelGGL(k_im_add, dim3(b6), dim3(256), 0, s->stream, s->mode, (const double*)s->cg_x, n6, s->im_q);
            k++;
        }
        newton += k;
        const double rel = ref > 0 ? res / ref : 0.0;
        if (!(res <= o->tol * ref)) notconv++;
        maxres = std::max(maxres, rel);
        hipLaunchKernelGGL(k_im_accept, dim3(blocks_for(N, 256)), dim3(256), 0, s->stream, ia, (const double*)s->im_q,
                           (const double*)s->im_g, s->fext, s->wext, s->wkin, s->node, s->im_qn, s->im_vn, s->im_an,
                           s->im_gn, s->im_fn, s->flag);
        HIP_TRY(hipMemcpyAsync(s->im_ht_c, s->hist, 4 * F * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipMemcpyAsync(s->im_wint_c, s->wint, T * 8, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipGetLastError());
        s->step++;
    }
    if (stats) {
        stats->steps = n_steps;
        stats->newton_iters = newton;
        stats->cg_iters = cgits;
        stats->not_converged = notconv;
        stats->max_residual = maxres;
    }
    return ldpm_sync(s);
}

// ---------------------------------------------------------------------------
// on-device tessellation
// ---------------------------------------------------------------------------
ldpm_status ldpm_tessellate(const ldpm_tess_desc* d, ldpm_tess_out* o, void* stream)
{
    if (!d || !o || !d->x || !d->diam || !d->tet_nodes) return fail(LDPM_ERR_ARG, "null argument");
    const int64_t N = d->n_particles, T = d->n_tets, F = 12 * T;
    if (N <= 0 || T <= 0) return fail(LDPM_ERR_ARG, "tessellate: empty input");
    if (N >= (1ll << 31) || 4 * T >= (1ll << 31)) return fail(LDPM_ERR_ARG, "tessellate: too large for 32-bit ids");
    if (!(d->rho > 0) || !std::isfinite(d->rho)) return fail(LDPM_ERR_ARG, "tessellate: rho must be positive");
    if (!finite_all(d->x, 3 * N)) return fail(LDPM_ERR_ARG, "tessellate: non-finite centres");
    for (int64_t i = 0; i < N; i++)
        if (!(d->diam[i] > 0) || !std::isfinite(d->diam[i])) return fail(LDPM_ERR_ARG, "tessellate: diameters must be positive");
    std::vector<int32_t> ptr(N + 1, 0), inc(4 * T);
    for (int64_t t = 0; t < T; t++)
        for (int a = 0; a < 4; a++) {
            const int64_t nd = d->tet_nodes[a * T + t];
            if (nd < 0 || nd >= N) return fail(LDPM_ERR_ARG, "tessellate: tet %lld: node out of range", (long long)t);
            for (int b = 0; b < a; b++)
                if (d->tet_nodes[b * T + t] == nd) return fail(LDPM_ERR_ARG, "tessellate: tet %lld repeats a node", (long long)t);
            ptr[nd + 1]++;
        }
    for (int64_t i = 0; i < N; i++) ptr[i + 1] += ptr[i];
    {
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t t = 0; t < T; t++)
            for (int a = 0; a < 4; a++) inc[fill[d->tet_nodes[a * T + t]]++] = (int32_t)(4 * t + a);
    }
    Carve cv;
    const size_t o_x = cv.take<double>(3 * N), o_dm = cv.take<double>(N), o_tet = cv.take<int32_t>(4 * T);
    const size_t o_inc = cv.take<int32_t>(4 * T), o_ptr = cv.take<int32_t>(N + 1);
    const size_t o_I = cv.take<int32_t>(F), o_J = cv.take<int32_t>(F);
    const size_t o_cI = cv.take<double>(3 * F), o_n = cv.take<double>(3 * F), o_m = cv.take<double>(3 * F);
    const size_t o_A = cv.take<double>(F), o_A0 = cv.take<double>(F), o_len = cv.take<double>(F);
    const size_t o_cone = cv.take<double>(40 * T);
    const size_t o_mass = cv.take<double>(N), o_vol = cv.take<double>(N), o_r = cv.take<double>(3 * N);
    const size_t o_Jd = cv.take<double>(3 * N), o_J6 = cv.take<double>(6 * N);
    const size_t bytes = (cv.off + 255) & ~size_t(255);
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(LDPM_ERR_ALLOC, "tessellate: hipMalloc(%zu) failed", bytes);
    char* B = (char*)mem;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    auto up = [&](size_t off, const void* src, size_t n) {
        if (e == hipSuccess) e = hipMemcpyAsync(B + off, src, n, hipMemcpyHostToDevice, st);
    };
    up(o_x, d->x, 3 * N * 8);
    up(o_dm, d->diam, N * 8);
    up(o_tet, d->tet_nodes, 4 * T * 4);
    up(o_inc, inc.data(), 4 * T * 4);
    up(o_ptr, ptr.data(), (N + 1) * 4);
    TessIn ti{(const double*)(B + o_x), (const double*)(B + o_dm), (const int32_t*)(B + o_tet), N, T};
    TessOut to{(int32_t*)(B + o_I), (int32_t*)(B + o_J), (double*)(B + o_cI), (double*)(B + o_n), (double*)(B + o_m),
               (double*)(B + o_A), (double*)(B + o_A0), (double*)(B + o_len), (double*)(B + o_cone)};
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_tessellate, dim3(blocks_for(T, kTessTets)), dim3(256), 0, st, ti, to);
        hipLaunchKernelGGL(k_cells, dim3(blocks_for(N * kCellGroup, 256)), dim3(256), 0, st,
                           (const int32_t*)(B + o_ptr), (const int32_t*)(B + o_inc), (const double*)(B + o_cone), N,
                           d->rho, (double*)(B + o_mass), (double*)(B + o_vol), (double*)(B + o_r),
                           (double*)(B + o_Jd), (double*)(B + o_J6));
        e = hipGetLastError();
    }
    auto down = [&](void* dst, size_t off, size_t n) {
        if (dst && e == hipSuccess) e = hipMemcpyAsync(dst, B + off, n, hipMemcpyDeviceToHost, st);
    };
    down(o->facet_I, o_I, F * 4);
    down(o->facet_J, o_J, F * 4);
    down(o->facet_cI, o_cI, 3 * F * 8);
    down(o->facet_n, o_n, 3 * F * 8);
    down(o->facet_m, o_m, 3 * F * 8);
    down(o->facet_area, o_A, F * 8);
    down(o->facet_area0, o_A0, F * 8);
    down(o->facet_len, o_len, F * 8);
    down(o->mass, o_mass, N * 8);
    down(o->cell_vol, o_vol, N * 8);
    down(o->cell_r, o_r, 3 * N * 8);
    down(o->rot_inertia, o_Jd, 3 * N * 8);
    down(o->cell_inertia, o_J6, 6 * N * 8);
    down(o->tet_node_cones, o_cone, 40 * T * 8);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(mem);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "tessellate failed: %s", hipGetErrorString(e));
    return LDPM_OK;
}

ldpm_status ldpm_element_lambda(const ldpm_elem_desc* d, double* lam, void* stream)
{
    if (!d || !lam || !d->tet_nodes || !d->facet_I || !d->facet_J || !d->facet_cI || !d->facet_n ||
        !d->facet_area || !d->facet_len || !d->share)
        return fail(LDPM_ERR_ARG, "null argument");
    const int64_t N = d->n_particles, T = d->n_tets, F = 12 * T;
    if (N <= 0 || T <= 0) return fail(LDPM_ERR_ARG, "element bound: empty input");
    if (N >= (1ll << 31) || F >= (1ll << 31)) return fail(LDPM_ERR_ARG, "element bound: too large for 32-bit ids");
    if (!(d->E0 > 0) || !std::isfinite(d->E0) || !(d->alpha >= 0) || !std::isfinite(d->alpha))
        return fail(LDPM_ERR_ARG, "element bound: need E0 > 0 and alpha >= 0");
    if (!finite_all(d->facet_cI, 3 * F) || !finite_all(d->facet_n, 3 * F) || !finite_all(d->facet_area, F))
        return fail(LDPM_ERR_ARG, "element bound: non-finite facet data");
    for (int64_t f = 0; f < F; f++)
        if (!(d->facet_len[f] > 0) || !std::isfinite(d->facet_len[f]))
            return fail(LDPM_ERR_ARG, "element bound: facet %lld: length must be positive", (long long)f);
    for (int64_t i = 0; i < 24 * T; i++)
        if (!(d->share[i] > 0) || !std::isfinite(d->share[i]))
            return fail(LDPM_ERR_ARG, "element bound: mass shares must be positive");
    for (int64_t t = 0; t < T; t++) {
        int32_t id[4];
        for (int a = 0; a < 4; a++) {
            id[a] = d->tet_nodes[a * T + t];
            if (id[a] < 0 || id[a] >= N) return fail(LDPM_ERR_ARG, "element bound: tet %lld: node out of range", (long long)t);
        }
        for (int k = 0; k < 12; k++) {
            const int32_t I = d->facet_I[t * 12 + k], J = d->facet_J[t * 12 + k];
            bool hi = false, hj = false;
            for (int a = 0; a < 4; a++) {
                hi = hi || id[a] == I;
                hj = hj || id[a] == J;
            }
            if (!hi || !hj || I == J)
                return fail(LDPM_ERR_ARG, "element bound: facet %lld does not join two nodes of its tet",
                            (long long)(t * 12 + k));
        }
    }
    Carve cv;
    const size_t o_tet = cv.take<int32_t>(4 * T), o_I = cv.take<int32_t>(F), o_J = cv.take<int32_t>(F);
    const size_t o_cI = cv.take<double>(3 * F), o_n = cv.take<double>(3 * F), o_A = cv.take<double>(F);
    const size_t o_len = cv.take<double>(F), o_sh = cv.take<double>(24 * T), o_lam = cv.take<double>(T);
    const size_t bytes = (cv.off + 255) & ~size_t(255);
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(LDPM_ERR_ALLOC, "element bound: hipMalloc(%zu) failed", bytes);
    char* B = (char*)mem;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    auto up = [&](size_t off, const void* src, size_t nb) {
        if (e == hipSuccess) e = hipMemcpyAsync(B + off, src, nb, hipMemcpyHostToDevice, st);
    };
    up(o_tet, d->tet_nodes, 4 * T * 4);
    up(o_I, d->facet_I, F * 4);
    up(o_J, d->facet_J, F * 4);
    up(o_cI, d->facet_cI, 3 * F * 8);
    up(o_n, d->facet_n, 3 * F * 8);
    up(o_A, d->facet_area, F * 8);
    up(o_len, d->facet_len, F * 8);
    up(o_sh, d->share, 24 * T * 8);
    if (e == hipSuccess) {
        ElemIn in{(const int32_t*)(B + o_tet), (const int32_t*)(B + o_I), (const int32_t*)(B + o_J),
                  (const double*)(B + o_cI), (const double*)(B + o_n), (const double*)(B + o_A),
                  (const double*)(B + o_len), (const double*)(B + o_sh), d->E0, d->alpha, T};
        hipLaunchKernelGGL(k_elem_lambda, dim3(blocks_for(T, EB_WAVES)), dim3(256), 0, st, in, (double*)(B + o_lam));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(lam, B + o_lam, T * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(mem);
    if (e != hipSuccess) return fail(LDPM_ERR_DEVICE, "element bound failed: %s", hipGetErrorString(e));
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
    if (s->pt_mem) (void)hipFree(s->pt_mem);
    if (s->im_mem) (void)hipFree(s->im_mem);
    if (s->arena) {
        (void)hipStreamSynchronize(s->stream);
        if (s->dev_free) s->dev_free(s->arena, s->alloc_ctx);
        else (void)hipFree(s->arena);
    }
    delete s;
}

}  // extern "C"
