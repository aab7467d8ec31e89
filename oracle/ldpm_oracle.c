/*
 * Plain FP64 CPU oracle of the explicit (central-difference) LDPM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the solver library uses this code;
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header or helper with the GPU
 * library: the two meet only in the arrays produced by the input generator.
 *
 * It is deliberately slow and literal: every quantity is computed the way the
 * paper defines it, in the paper's order, in IEEE double precision (built with
 * -ffp-contract=off).  Loops over facets and over particles may run in
 * parallel (OpenMP); every sum whose order could change the rounding is done
 * serially in ascending index order, so results do not depend on the number
 * of threads.
 *
 * Paper: Lale, Elias, ..., Cusatis, "Lattice Discrete Particle Model (LDPM):
 * Comparison of Various Time Integration Solvers and Implementations".
 *
 * Readings of passages that are silent or ambiguous (each also documented
 * with the design notes of the project):
 *  - central difference = half-step leapfrog with constant dt; the first
 *    velocity update uses dt/2 from the initial velocity;
 *  - facet history starts from zero strain, zero traction, e_max = 0;
 *  - e_N = 0 takes the compressive branch;
 *  - sigma_0(omega) in its rationalised form (no 0/0 at omega = pi/2);
 *  - e_max is updated in tension only, before the boundary is evaluated;
 *  - the old effective traction / strain are rebuilt from the stored vectors
 *    of the previous step, whichever branch produced them;
 *  - friction: radial return of the elastic shear trial onto sigma_bs(t_N)
 *    evaluated at the updated normal traction;
 *  - e_V = (1/3) sum_a grad N_a . u_a (linearised volume change over 3V);
 *  - internal work: trapezoid per facet; external work: trapezoid with the
 *    applied forces plus the reactions of prescribed DoFs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* material parameters: paper, appendix table of parameters */
typedef struct {
    double E0, alpha, sigma_t, l_t, r_st, n_t, r_s, k_t;
    double sigma_c0, Hc0_over_E0, Hc1_over_E0, kc0, kc1, kc2, kc3, Ed_over_E0, beta;
    double mu0, mu_inf, sigma_N0;
    int32_t law; /* 0: linear elastic t = E e; 1: full inelastic law */
} ora_mat;

/* system: all arrays row-major, particle-major (AoS) */
typedef struct {
    int64_t N, T, F;
    const double *x0;        /* [N][3] particle centres */
    const double *mass;      /* [N] */
    const double *inertia;   /* [N][3] diagonal rotational inertia */
    const double *cell_vol;  /* [N] */
    const double *cell_r;    /* [N][3] centre -> cell centroid */
    const int32_t *tet;      /* [T][4] */
    const int32_t *fI, *fJ, *ftet; /* [F] */
    const double *cI;        /* [F][3] node I -> facet centroid */
    const double *n, *m;     /* [F][3] facet frame (l = n x m) */
    const double *A, *len;   /* [F] projected area, edge length */
    const uint8_t *dof_mode; /* [N][6] 0 free, 1 prescribed velocity */
    const int32_t *dof_prog; /* [N][6] program id or -1 */
    const double *dof_scale; /* [N][6] */
    int64_t n_prog;
    const int64_t *prog_off; /* [n_prog+1] */
    const double *prog_t, *prog_v;
    const double *body;      /* [3] body force per unit volume */
    double dt;
    ora_mat mat;
    /* [N][21] or NULL: full rigid-body mass block of each cell about its
     * particle centre (eq. balance: M_u, M_theta, I_u, I_theta), upper
     * triangle row-major over (u_x, u_y, u_z, th_x, th_y, th_z); NULL: the
     * lumped diagonal (mass, inertia) */
    const double *mass_block;
} ora_sys;

typedef struct {
    double *q, *v;       /* [N][6]: q^n, and v^{n-1/2} (v^0 before the first step) */
    double *t, *e;       /* [F][3]: traction and strain of the last step */
    double *emax;        /* [F] */
    double *fext;        /* [N][6]: applied + reaction generalised force of the last step */
    double W_int, W_ext, W_kin, W_kin0;
    double W_pert;       /* work of the random perturbations (ora_perturb) */
    int64_t step;        /* completed steps */
} ora_state;

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double macaulay(double x) { return x > 0.0 ? x : 0.0; }

/* ---------------------------------------------------------------------- */
/* Tetrahedron volumetric strain (appendix, compressive behaviour: e_V "from
 * the tetrahedron volume"), linearised: e_V = (1/3) sum_a grad N_a . u_a with
 * N_a the linear shape functions of the tetrahedron.                       */
double ora_tet_volstrain(const double x[4][3], const double u[4][3])
{
    double Jm[3][3], inv[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++)
            Jm[r][c] = x[c + 1][r] - x[0][r];   /* columns x_a - x_0 */
    double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1])
               - Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0])
               + Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
    inv[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / det;
    inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
    inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
    inv[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / det;
    inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
    inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
    inv[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / det;
    inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
    inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
    /* grad N_a (a = 1..3) is row a-1 of J^{-1}; grad N_0 = -sum */
    double g[4][3];
    for (int c = 0; c < 3; c++) {
        g[1][c] = inv[0][c];
        g[2][c] = inv[1][c];
        g[3][c] = inv[2][c];
        g[0][c] = -(inv[0][c] + inv[1][c] + inv[2][c]);
    }
    double s = 0.0;
    for (int a = 0; a < 4; a++) s += dot3(g[a], u[a]);
    return s / 3.0;
}

/* Facet strain, eq. (strain1): e = P^T [[u]] / l with
 * [[u]] = u_J + theta_J x c^J - u_I - theta_I x c^I, c^J = c^I - l n.      */
void ora_facet_strain(const double qI[6], const double qJ[6], const double cI[3],
                      const double n[3], const double m[3], double len, double e[3])
{
    double cJ[3], l[3], wI[3], wJ[3], d[3];
    for (int i = 0; i < 3; i++) cJ[i] = cI[i] - len * n[i];
    cross3(n, m, l);
    cross3(qI + 3, cI, wI);
    cross3(qJ + 3, cJ, wJ);
    for (int i = 0; i < 3; i++) d[i] = qJ[i] + wJ[i] - qI[i] - wI[i];
    e[0] = dot3(n, d) / len;
    e[1] = dot3(m, d) / len;
    e[2] = dot3(l, d) / len;
}

/* Facet constitutive update t = T(e, s, p) (appendix).  Inputs: current
 * strain e, previous strain e_old, previous traction t_old, previous e_max,
 * tetrahedron volumetric strain eV and edge length len.                    */
void ora_facet_law(const ora_mat *p, double len, const double e[3], const double e_old[3],
                   double eV, const double t_old[3], double emax_old,
                   double t[3], double *emax_out)
{
    const double E0 = p->E0, al = p->alpha;
    *emax_out = emax_old;
    if (p->law == 0) {
        /* elastic: t = E e with E = E0 diag(1, alpha, alpha) */
        t[0] = E0 * e[0];
        t[1] = al * E0 * e[1];
        t[2] = al * E0 * e[2];
        return;
    }
    const double eN = e[0], eM = e[1], eL = e[2];
    if (eN > 0.0) {
        /* ---- fracturing behaviour (e_N > 0) ---- */
        /* effective strain e = sqrt(e_N^2 + alpha (e_M^2 + e_L^2)), evaluated
         * with hypot so that tiny strains cannot underflow to e = 0 while
         * e_N > 0 (the definition gives e >= e_N > 0)                      */
        const double sa = sqrt(al);
        double eTs = sa * hypot(eM, eL);                                   /* sqrt(alpha) e_T */
        double eff = hypot(eN, eTs);                                       /* e */
        double eff_old = hypot(e_old[0], sa * hypot(e_old[1], e_old[2]));
        double t_eff_old = hypot(t_old[0], hypot(t_old[1], t_old[2]) / sa);
        /* coupling variable: tan(omega) = e_N / sqrt(alpha (e_M^2 + e_L^2)) */
        double omega = atan2(eN, eTs);
        double sn = eN / eff;
        double cw = eTs / eff;
        double cs2 = cw * cw;
        double rst2 = p->r_st * p->r_st;
        /* strength limit sigma_0(omega), rationalised */
        double sigma0 = 2.0 * p->sigma_t / (sn + sqrt(sn * sn + 4.0 * al * cs2 / rst2));
        double e0 = sigma0 / E0;
        /* softening modulus H_0(omega) */
        double Ht = 2.0 * E0 / (p->l_t / len - 1.0);
        double Hs = p->r_s * E0;
        double H0 = Hs / al + (Ht - Hs / al) * pow(2.0 * omega / M_PI, p->n_t);
        double emax = emax_old > eff ? emax_old : eff;
        /* boundary sigma_bt, exponential in the maximum effective strain */
        double sbt = sigma0 * exp(-H0 * macaulay(emax - e0) / sigma0);
        /* unloading / reloading */
        double etr = p->k_t * (emax - sbt / E0);
        double ttr;
        if (t_eff_old > 0.0) {
            ttr = t_eff_old + E0 * (eff - eff_old);
        } else if (eff > etr) {
            double base = etr > eff_old ? etr : eff_old;
            ttr = E0 * macaulay(eff - base);
        } else {
            ttr = 0.0;
        }
        /* 0 <= t <= sigma_bt (vertical return) */
        double te = ttr;
        if (te < 0.0) te = 0.0;
        if (te > sbt) te = sbt;
        t[0] = te / eff * eN;
        t[1] = al * te / eff * eM;
        t[2] = al * te / eff * eL;
        *emax_out = emax;
        return;
    }
    /* ---- compressive behaviour (e_N <= 0) ---- */
    double eD = eN - eV;
    double eDV = eV + p->beta * eD;
    double sc0 = p->sigma_c0;
    double eV0 = p->kc3 * sc0 / E0;
    double rDV = (eV <= 0.0) ? -fabs(eD) / (eV - eV0) : fabs(eD) / eV0;
    double Hc0 = p->Hc0_over_E0 * E0, Hc1 = p->Hc1_over_E0 * E0;
    double Hc = (Hc0 - Hc1) / (1.0 + p->kc2 * macaulay(rDV - p->kc1)) + Hc1;
    double ec0 = sc0 / E0;
    double ec1 = p->kc0 * ec0;
    double sc1 = sc0 + (ec1 - ec0) * Hc;
    double sbc;
    if (-eDV <= 0.0)
        sbc = sc0;
    else if (-eDV <= ec1)
        sbc = sc0 + macaulay(-eDV - ec0) * Hc;
    else
        sbc = sc1 * exp((-eDV - ec1) * Hc / sc1);
    double ENc = (-t_old[0] <= sc0) ? E0 : p->Ed_over_E0 * E0;
    double tN = t_old[0] + ENc * (eN - e_old[0]);
    if (tN < -sbc) tN = -sbc;
    if (tN > 0.0) tN = 0.0;
    /* frictional behaviour: elastic shear trial, radial return onto
     * sqrt(t_M^2 + t_L^2) = sigma_bs(t_N)                                  */
    double ss = p->r_st * p->sigma_t;
    double dmu = p->mu0 - p->mu_inf;
    double sbs = ss + dmu * p->sigma_N0 - p->mu_inf * tN - dmu * p->sigma_N0 * exp(tN / p->sigma_N0);
    double tM = t_old[1] + al * E0 * (eM - e_old[1]);
    double tL = t_old[2] + al * E0 * (eL - e_old[2]);
    double nrm = sqrt(tM * tM + tL * tL);
    if (nrm > sbs) {
        tM = tM * (sbs / nrm);
        tL = tL * (sbs / nrm);
    }
    t[0] = tN;
    t[1] = tM;
    t[2] = tL;
}

/* piecewise-linear time program, constant beyond its end points */
static double prog_eval(const ora_sys *s, int32_t p, double time)
{
    if (p < 0) return 0.0;
    int64_t a = s->prog_off[p], b = s->prog_off[p + 1];
    if (b <= a) return 0.0;
    if (time <= s->prog_t[a]) return s->prog_v[a];
    for (int64_t i = a; i + 1 < b; i++) {
        if (time <= s->prog_t[i + 1]) {
            double w = (time - s->prog_t[i]) / (s->prog_t[i + 1] - s->prog_t[i]);
            return s->prog_v[i] + w * (s->prog_v[i + 1] - s->prog_v[i]);
        }
    }
    return s->prog_v[b - 1];
}

/* Facet contribution to particle I: A P t (force) and c^I x (A P t); to J:
 * the negatives with c^J (eq. balance).                                    */
static void facet_force(const ora_sys *s, int64_t k, const double t[3], double F[3])
{
    const double *n = s->n + 3 * k, *m = s->m + 3 * k;
    double l[3];
    cross3(n, m, l);
    for (int i = 0; i < 3; i++) F[i] = s->A[k] * (t[0] * n[i] + t[1] * m[i] + t[2] * l[i]);
}

static void tet_volstrains(const ora_sys *s, const double *q, double *eV)
{
#pragma omp parallel for schedule(static)
    for (int64_t tt = 0; tt < s->T; tt++) {
        double x[4][3], u[4][3];
        for (int a = 0; a < 4; a++) {
            int32_t nd = s->tet[4 * tt + a];
            for (int i = 0; i < 3; i++) {
                x[a][i] = s->x0[3 * nd + i];
                u[a][i] = q[6 * nd + i];
            }
        }
        eV[tt] = ora_tet_volstrain(x, u);
    }
}

/* Solve A x = b for the n x n leading part of A (row stride 6) by Gaussian
 * elimination with partial pivoting; A and b are overwritten.             */
static void solve_small(double A[6][6], double *b, double *x, int n)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c) {
            for (int k = 0; k < n; k++) {
                double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t;
            }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < n; k++) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        double acc = b[r];
        for (int k = r + 1; k < n; k++) acc -= A[r][k] * x[k];
        x[r] = acc / A[r][r];
    }
}

/* Velocity update of one particle with a full 6 x 6 mass block Mb (eq. of
 * motion M q'' = f_ext - f_int restricted to the particle): prescribed DoFs
 * take their programmed velocity, whose acceleration a_P = (v+ - v-)/h
 * enters the free rows: M_FF a_F = fnet_F - M_FP a_P; the reactions are
 * R_P = M_PF a_F + M_PP a_P - fnet_P.                                      */
static void block_update(const double Mb[6][6], const int pres[6], const double fnet[6], const double vold[6],
                         const double vpres[6], double h, double vnew[6], double react[6])
{
    double a[6], A[6][6], r[6], x[6];
    int fi[6], nf = 0;
    for (int d = 0; d < 6; d++) {
        if (pres[d]) {
            vnew[d] = vpres[d];
            a[d] = (vnew[d] - vold[d]) / h;
        } else {
            fi[nf++] = d;
        }
    }
    for (int i = 0; i < nf; i++) {
        r[i] = fnet[fi[i]];
        for (int k = 0; k < 6; k++)
            if (pres[k]) r[i] -= Mb[fi[i]][k] * a[k];
        for (int j = 0; j < nf; j++) A[i][j] = Mb[fi[i]][fi[j]];
    }
    if (nf > 0) solve_small(A, r, x, nf);
    for (int i = 0; i < nf; i++) {
        a[fi[i]] = x[i];
        vnew[fi[i]] = vold[fi[i]] + h * x[i];
    }
    for (int d = 0; d < 6; d++) {
        react[d] = 0.0;
        if (pres[d]) {
            double ma = 0.0;
            for (int k = 0; k < 6; k++) ma += Mb[d][k] * a[k];
            react[d] = ma - fnet[d];
        }
    }
}

/* Explicit central-difference steps (eq. of motion M q'' + f_int = f_ext with
 * the lumped diagonal M, or the full per-cell blocks).  Returns 0, or 1 if a
 * non-finite value appeared.                                                */
int ora_step(const ora_sys *s, ora_state *st, int64_t nsteps, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const int64_t N = s->N, T = s->T, F = s->F;
    double *eV = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    double *Fk = (double *)malloc(sizeof(double) * 3 * (size_t)(F > 0 ? F : 1));
    double *dW = (double *)malloc(sizeof(double) * (size_t)(F > 0 ? F : 1));
    double *enew = (double *)malloc(sizeof(double) * 3 * (size_t)(F > 0 ? F : 1));
    double *tnew = (double *)malloc(sizeof(double) * 3 * (size_t)(F > 0 ? F : 1));
    double *emnew = (double *)malloc(sizeof(double) * (size_t)(F > 0 ? F : 1));
    double *f = (double *)malloc(sizeof(double) * 6 * (size_t)(N > 0 ? N : 1));
    int bad = 0;
    const double dt = s->dt;
    for (int64_t it = 0; it < nsteps; it++) {
        const int64_t n = st->step;
        const double time = (double)n * dt;
        /* 1. tetrahedron volumetric strains */
        tet_volstrains(s, st->q, eV);
        /* 2. facet strain, constitutive law, force, work increment */
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < F; k++) {
            const double *qI = st->q + 6 * (int64_t)s->fI[k];
            const double *qJ = st->q + 6 * (int64_t)s->fJ[k];
            double e[3], t[3], em;
            ora_facet_strain(qI, qJ, s->cI + 3 * k, s->n + 3 * k, s->m + 3 * k, s->len[k], e);
            ora_facet_law(&s->mat, s->len[k], e, st->e + 3 * k, eV[s->ftet[k]], st->t + 3 * k,
                          st->emax[k], t, &em);
            double w = 0.0;
            for (int i = 0; i < 3; i++)
                w += 0.5 * (st->t[3 * k + i] + t[i]) * (e[i] - st->e[3 * k + i]);
            dW[k] = s->A[k] * s->len[k] * w;
            facet_force(s, k, t, Fk + 3 * k);
            for (int i = 0; i < 3; i++) {
                enew[3 * k + i] = e[i];
                tnew[3 * k + i] = t[i];
            }
            emnew[k] = em;
        }
        /* 3. internal work, ascending facet order */
        for (int64_t k = 0; k < F; k++) st->W_int += dW[k];
        /* 4. gather onto particles, ascending facet order (eq. balance) */
        memset(f, 0, sizeof(double) * 6 * (size_t)N);
        for (int64_t k = 0; k < F; k++) {
            const double *Fv = Fk + 3 * k;
            const double *cI = s->cI + 3 * k;
            double cJ[3], MI[3], MJ[3];
            for (int i = 0; i < 3; i++) cJ[i] = cI[i] - s->len[k] * s->n[3 * k + i];
            cross3(cI, Fv, MI);
            cross3(cJ, Fv, MJ);
            double *fI = f + 6 * (int64_t)s->fI[k], *fJ = f + 6 * (int64_t)s->fJ[k];
            for (int i = 0; i < 3; i++) {
                fI[i] += Fv[i];
                fI[3 + i] += MI[i];
                fJ[i] -= Fv[i];
                fJ[3 + i] -= MJ[i];
            }
        }
        /* 5. external forces, leapfrog update, reactions, energies */
        const double h = (n == 0) ? 0.5 * dt : dt;
        const double t_half = ((double)n + 0.5) * dt;
        double Wk = 0.0, dWext = 0.0;
        for (int64_t I = 0; I < N; I++) {
            double Mv[6];
            Mv[0] = Mv[1] = Mv[2] = s->mass[I];
            for (int i = 0; i < 3; i++) Mv[3 + i] = s->inertia[3 * I + i];
            double body[6] = {0, 0, 0, 0, 0, 0};
            if (s->body) {
                double rxb[3];
                cross3(s->cell_r + 3 * I, s->body, rxb);
                for (int i = 0; i < 3; i++) {
                    body[i] = s->cell_vol[I] * s->body[i];
                    body[3 + i] = s->cell_vol[I] * rxb[i];
                }
            }
            if (s->mass_block) {
                double Mb[6][6], fnet[6], applied[6], vold[6], vpres[6], vnew[6], react[6];
                int pres[6];
                const double *ut = s->mass_block + 21 * I;
                for (int r = 0, k = 0; r < 6; r++)
                    for (int c = r; c < 6; c++, k++) Mb[r][c] = Mb[c][r] = ut[k];
                for (int d = 0; d < 6; d++) {
                    const int64_t id = 6 * I + d;
                    const int32_t pg = s->dof_prog[id];
                    applied[d] = body[d];
                    if (s->dof_mode[id] == 0 && pg >= 0) applied[d] += s->dof_scale[id] * prog_eval(s, pg, time);
                    fnet[d] = f[id] + applied[d];
                    vold[d] = st->v[id];
                    pres[d] = s->dof_mode[id] != 0;
                    vpres[d] = (pres[d] && pg >= 0) ? s->dof_scale[id] * prog_eval(s, pg, t_half) : 0.0;
                }
                block_update(Mb, pres, fnet, vold, vpres, h, vnew, react);
                double vbar[6];
                for (int d = 0; d < 6; d++) vbar[d] = (n == 0) ? vold[d] : 0.5 * (vold[d] + vnew[d]);
                for (int d = 0; d < 6; d++) {
                    const int64_t id = 6 * I + d;
                    const double Fd = applied[d] + react[d];
                    if (n > 0) dWext += 0.5 * (st->fext[id] + Fd) * (dt * vold[d]);
                    double Mvb = 0.0;
                    for (int k = 0; k < 6; k++) Mvb += Mb[d][k] * vbar[k];
                    Wk += 0.5 * vbar[d] * Mvb;
                    st->fext[id] = Fd;
                    st->v[id] = vnew[d];
                    st->q[id] += dt * vnew[d];
                    if (!isfinite(vnew[d])) bad = 1;
                }
                continue;
            }
            for (int d = 0; d < 6; d++) {
                const int64_t id = 6 * I + d;
                double applied = body[d];
                const int32_t pg = s->dof_prog[id];
                if (s->dof_mode[id] == 0 && pg >= 0) applied += s->dof_scale[id] * prog_eval(s, pg, time);
                const double fnet = f[id] + applied;          /* f_ext - f_int */
                const double vold = st->v[id];
                double vnew, Fd;
                if (s->dof_mode[id] == 0) {
                    vnew = vold + h * fnet / Mv[d];
                    Fd = applied;
                } else {
                    vnew = (pg >= 0) ? s->dof_scale[id] * prog_eval(s, pg, t_half) : 0.0;
                    double R = Mv[d] * (vnew - vold) / h - fnet;  /* reaction */
                    Fd = applied + R;
                }
                if (n > 0) dWext += 0.5 * (st->fext[id] + Fd) * (dt * vold);
                double vbar = (n == 0) ? vold : 0.5 * (vold + vnew);
                Wk += 0.5 * Mv[d] * vbar * vbar;
                st->fext[id] = Fd;
                st->v[id] = vnew;
                st->q[id] += dt * vnew;
                if (!isfinite(vnew)) bad = 1;
            }
        }
        st->W_ext += dWext;
        st->W_kin = Wk;
        if (n == 0) st->W_kin0 = Wk;
        memcpy(st->e, enew, sizeof(double) * 3 * (size_t)F);
        memcpy(st->t, tnew, sizeof(double) * 3 * (size_t)F);
        memcpy(st->emax, emnew, sizeof(double) * (size_t)F);
        st->step = n + 1;
        if (bad) break;
    }
    free(eV); free(Fk); free(dW); free(enew); free(tnew); free(emnew); free(f);
    return bad;
}

/* Elastic internal force f_int(q) (zero history, t = E e): the generalised
 * force such that M q'' = f_ext - f_int.                                   */
void ora_elastic_internal_force(const ora_sys *s, const double *q, double *fint)
{
    memset(fint, 0, sizeof(double) * 6 * (size_t)s->N);
    for (int64_t k = 0; k < s->F; k++) {
        double e[3], t[3], Fv[3], cJ[3], MI[3], MJ[3];
        ora_facet_strain(q + 6 * (int64_t)s->fI[k], q + 6 * (int64_t)s->fJ[k], s->cI + 3 * k,
                         s->n + 3 * k, s->m + 3 * k, s->len[k], e);
        t[0] = s->mat.E0 * e[0];
        t[1] = s->mat.alpha * s->mat.E0 * e[1];
        t[2] = s->mat.alpha * s->mat.E0 * e[2];
        facet_force(s, k, t, Fv);
        for (int i = 0; i < 3; i++) cJ[i] = s->cI[3 * k + i] - s->len[k] * s->n[3 * k + i];
        cross3(s->cI + 3 * k, Fv, MI);
        cross3(cJ, Fv, MJ);
        double *fI = fint + 6 * (int64_t)s->fI[k], *fJ = fint + 6 * (int64_t)s->fJ[k];
        for (int i = 0; i < 3; i++) {
            fI[i] -= Fv[i];
            fI[3 + i] -= MI[i];
            fJ[i] += Fv[i];
            fJ[3 + i] += MJ[i];
        }
    }
}

/* Random perturbation of the solution (section on the numerical study of
 * time step, convergence criteria and stability): delta [N][6] is added to
 * every free DoF (displacements and rotations) of every particle; prescribed
 * DoFs keep their values.
 * Reading (the paper does not say how the facet history sees the jump): the
 * jump is a strain increment of its own, taken by the facet law at once.
 * It starts from the configuration of the last law evaluation,
 * q^{n-1} = q^n - dt v^{n-1/2}, whose strain is the stored e, and ends at that
 * configuration plus the jump; so the next step starts from a history that
 * matches the perturbed positions.  The traction work of the jump
 * (trapezoid, as for a step) is added to W_int and, being done on the
 * specimen from outside, to W_pert.  Before the first step there is no
 * history yet: the jump only changes the initial displacement.
 * Returns the work of this jump.                                           */
double ora_perturb(const ora_sys *s, ora_state *st, const double *delta)
{
    const int64_t N = s->N, T = s->T, F = s->F;
    double *d = (double *)malloc(sizeof(double) * 6 * (size_t)(N > 0 ? N : 1));
    for (int64_t id = 0; id < 6 * N; id++) d[id] = s->dof_mode[id] == 0 ? delta[id] : 0.0;
    double W = 0.0;
    if (st->step > 0) {
        double *qj = (double *)malloc(sizeof(double) * 6 * (size_t)(N > 0 ? N : 1));
        double *eV = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
        double *dW = (double *)malloc(sizeof(double) * (size_t)(F > 0 ? F : 1));
        for (int64_t id = 0; id < 6 * N; id++) qj[id] = st->q[id] - s->dt * st->v[id] + d[id];
        tet_volstrains(s, qj, eV);
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < F; k++) {
            double de[3], e[3], t[3], em;
            ora_facet_strain(d + 6 * (int64_t)s->fI[k], d + 6 * (int64_t)s->fJ[k], s->cI + 3 * k,
                             s->n + 3 * k, s->m + 3 * k, s->len[k], de);
            for (int i = 0; i < 3; i++) e[i] = st->e[3 * k + i] + de[i];
            ora_facet_law(&s->mat, s->len[k], e, st->e + 3 * k, eV[s->ftet[k]], st->t + 3 * k,
                          st->emax[k], t, &em);
            double w = 0.0;
            for (int i = 0; i < 3; i++) w += 0.5 * (st->t[3 * k + i] + t[i]) * de[i];
            dW[k] = s->A[k] * s->len[k] * w;
            for (int i = 0; i < 3; i++) {
                st->e[3 * k + i] = e[i];
                st->t[3 * k + i] = t[i];
            }
            st->emax[k] = em;
        }
        for (int64_t k = 0; k < F; k++) W += dW[k];
        st->W_int += W;
        st->W_pert += W;
        free(qj); free(eV); free(dW);
    }
    for (int64_t id = 0; id < 6 * N; id++) st->q[id] += d[id];
    free(d);
    return W;
}

/* Trial internal force of an implicit iteration: every facet law is
 * evaluated at the trial configuration q from the committed history (strain
 * e, traction t, e_max of the state) without committing it.  g = -f_int(q)
 * (the contribution to M q'' as in the explicit step, ascending facet
 * order); t_out, e_out, emax_out: the trial history; dW: the trial
 * internal-work increment of each facet (trapezoid).                      */
void ora_trial_force(const ora_sys *s, const ora_state *st, const double *q, double *g, double *t_out,
                     double *e_out, double *emax_out, double *dW)
{
    const int64_t N = s->N, T = s->T, F = s->F;
    double *eV = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    double *Fk = (double *)malloc(sizeof(double) * 3 * (size_t)(F > 0 ? F : 1));
    tet_volstrains(s, q, eV);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < F; k++) {
        double e[3], t[3], em;
        ora_facet_strain(q + 6 * (int64_t)s->fI[k], q + 6 * (int64_t)s->fJ[k], s->cI + 3 * k, s->n + 3 * k,
                         s->m + 3 * k, s->len[k], e);
        ora_facet_law(&s->mat, s->len[k], e, st->e + 3 * k, eV[s->ftet[k]], st->t + 3 * k, st->emax[k], t, &em);
        double w = 0.0;
        for (int i = 0; i < 3; i++) w += 0.5 * (st->t[3 * k + i] + t[i]) * (e[i] - st->e[3 * k + i]);
        dW[k] = s->A[k] * s->len[k] * w;
        facet_force(s, k, t, Fk + 3 * k);
        for (int i = 0; i < 3; i++) {
            e_out[3 * k + i] = e[i];
            t_out[3 * k + i] = t[i];
        }
        emax_out[k] = em;
    }
    memset(g, 0, sizeof(double) * 6 * (size_t)N);
    for (int64_t k = 0; k < F; k++) {
        const double *Fv = Fk + 3 * k;
        const double *cI = s->cI + 3 * k;
        double cJ[3], MI[3], MJ[3];
        for (int i = 0; i < 3; i++) cJ[i] = cI[i] - s->len[k] * s->n[3 * k + i];
        cross3(cI, Fv, MI);
        cross3(cJ, Fv, MJ);
        double *gI = g + 6 * (int64_t)s->fI[k], *gJ = g + 6 * (int64_t)s->fJ[k];
        for (int i = 0; i < 3; i++) {
            gI[i] += Fv[i];
            gI[3 + i] += MI[i];
            gJ[i] -= Fv[i];
            gJ[3 + i] -= MJ[i];
        }
    }
    free(eV);
    free(Fk);
}

/* All facet strains for a given q (test helper). */
void ora_all_strains(const ora_sys *s, const double *q, double *e)
{
    for (int64_t k = 0; k < s->F; k++)
        ora_facet_strain(q + 6 * (int64_t)s->fI[k], q + 6 * (int64_t)s->fJ[k], s->cI + 3 * k,
                         s->n + 3 * k, s->m + 3 * k, s->len[k], e + 3 * k);
}

/* All tetrahedron volumetric strains for a given q (test helper). */
void ora_all_volstrains(const ora_sys *s, const double *q, double *eV)
{
    tet_volstrains(s, q, eV);
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
