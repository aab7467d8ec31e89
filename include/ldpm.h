/*
 * ldpm.h - C-ABI of the MI355X explicit LDPM solver library (libldpm.so).
 *
 * The library advances the Lattice Discrete Particle Model equations of
 * motion  M q'' + f_int(q) = f_ext  (paper: "Numerical Implementations",
 * equation of motion with the lumped, diagonal mass matrix) by the explicit
 * central-difference scheme used by the paper's explicit solvers.  Each step:
 *   - facet strains e = P^T [[u]] / l from the translations and rotations of
 *     the two particles of every facet (eq. strain1),
 *   - the tetrahedron volumetric strain e_V (appendix, compressive behaviour),
 *   - the history-dependent facet law t = T(e, s, p) (appendix: fracturing,
 *     compressive and frictional behaviour; or t = E e),
 *   - facet forces A P t and moments c x (A P t) gathered onto particles
 *     (eq. balance) in a fixed order, without floating-point atomics,
 *   - the leapfrog update of velocities and positions in FP64, with
 *     prescribed-velocity programs, applied-force programs and reactions,
 *   - the work of internal and external forces and the kinetic energy
 *     (numerical-examples section: energy-balance measure).
 *
 * Conventions
 *   - Units are the caller's; the workloads shipped with the project use mm,
 *     N, MPa, s, tonne.
 *   - Arrays are structure-of-arrays: "[3][N]" means three consecutive blocks
 *     of N values (x of all particles, then y, then z).
 *   - Particle DoF d = 0..5 is (u_x, u_y, u_z, theta_x, theta_y, theta_z).
 *   - Facets are tetrahedron-major: facet f belongs to tetrahedron f / 12 and
 *     connects two of its nodes; n_facets == 12 * n_tets.  The order of the
 *     12 facets inside a tetrahedron is free.
 *   - Facet k, from particle I to particle J: n_k along I->J, m_k an arbitrary
 *     unit tangent, l_k = n_k x m_k; c^I_k points from I to the facet
 *     centroid; c^J_k = c^I_k - len_k n_k (eq. strain1 and eq. balance).
 *   - Particle I receives +A P t and c^I x (A P t) from its facet k; J
 *     receives the negatives with c^J (eq. balance).
 *
 * Time stepping (central difference, constant dt): the state after n steps
 * is (q^n, v^{n-1/2}).  Step n evaluates the internal forces at q^n and the
 * applied forces at t_n = n dt, sets v^{n+1/2} = v^{n-1/2} + h M^{-1} f for
 * free DoFs (h = dt/2 for the first step from the initial velocity v^0, dt
 * afterwards), v^{n+1/2} = scale * program(t_{n+1/2}) for prescribed DoFs,
 * and q^{n+1} = q^n + dt v^{n+1/2}.
 *
 * Errors: every call returns an ldpm_status; nothing is thrown across the
 * ABI and nothing aborts.  ldpm_last_error() returns a thread-local message
 * for the last failing call.  ldpm_step only enqueues work: a non-finite
 * velocity raises a sticky device flag that the next synchronising call
 * (ldpm_read_state, ldpm_energy, ldpm_reaction, ldpm_sync) reports as
 * LDPM_ERR_UNSTABLE.
 *
 * Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef LDPM_H
#define LDPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldpm_system ldpm_system; /* opaque, owned by the library */

typedef enum {
    LDPM_OK = 0,
    LDPM_ERR_ARG = 1,      /* invalid argument or inconsistent system */
    LDPM_ERR_ALLOC = 2,    /* device or host allocation failed */
    LDPM_ERR_DEVICE = 3,   /* a HIP call failed */
    LDPM_ERR_UNSTABLE = 4, /* non-finite state (dt above the stability limit?) */
    LDPM_ERR_STATE = 5     /* call not valid in the handle's current state */
} ldpm_status;

/* Facet-law precision. */
enum {
    LDPM_PREC_FP64 = 0,  /* everything in FP64 */
    LDPM_PREC_MIXED = 1  /* facet geometry, history, kinematics and law in FP32;
                            particle state, gather, integration, energies FP64 */
};

/* Material parameters, appendix table of parameters (names follow it).
 * law = 0: elastic t = E0 diag(1, alpha, alpha) e (only E0 and alpha used).
 * law = 1: fracturing (e_N > 0), compressive (e_N <= 0) and frictional
 *          behaviour.  r_s must be 0 (the paper leaves the degradation of
 *          the cohesion with H_s != 0 unspecified): LDPM_ERR_ARG otherwise.
 * Requires l_t > len_k for every facet (H_t > 0) when law = 1.           */
typedef struct {
    double E0, alpha, sigma_t, l_t, r_st, n_t, r_s, k_t;
    double sigma_c0, Hc0_over_E0, Hc1_over_E0, kc0, kc1, kc2, kc3, Ed_over_E0, beta;
    double mu0, mu_inf, sigma_N0;
    int32_t law;
} ldpm_material;

/* Full dynamic state, used to read the state (ldpm_read_state) and to
 * resume from it (ldpm_system_desc.init_state).  All pointers are host
 * memory owned by the caller; a NULL field is skipped on read and means
 * "zero" (or v0/q0 of the descriptor) on resume.                          */
typedef struct {
    double *q;          /* [6][N] displacements and rotations q^n            */
    double *v;          /* [6][N] v^{n-1/2} (v^0 while step == 0)            */
    double *t;          /* [3][F] facet traction of the last step (t_N,t_M,t_L) */
    double *emax;       /* [F]    maximum effective strain reached           */
    double *fext;       /* [6][N] applied + reaction force of the last step  */
    double *w_int;      /* [T]    accumulated internal work per tetrahedron  */
    double *w_ext;      /* [N]    accumulated external work per particle     */
    double *w_kin;      /* [N]    kinetic energy per particle at the last step */
    double *w_kin0;     /* [n_specimens] initial kinetic energy              */
    double *w_pert;     /* [n_specimens] work of random perturbations (ldpm_perturb) */
    int64_t step;       /* completed steps n                                 */
} ldpm_state;

/* System description.  The library copies everything it needs during
 * ldpm_load_system; the caller may free its arrays afterwards.            */
typedef struct {
    int32_t n_specimens;              /* >= 1; independent specimens concatenated */
    const int64_t *particle_off;      /* [n_specimens+1] or NULL when n_specimens == 1 */
    const int64_t *tet_off;           /* [n_specimens+1] or NULL when n_specimens == 1 */
    int64_t n_particles, n_tets, n_facets;  /* N, T, F (F == 12 T) */
    const double *x0;                 /* [3][N] particle centres */
    const double *mass;               /* [N]    lumped translational mass (> 0) */
    const double *rot_inertia;        /* [3][N] lumped rotational inertia (> 0) */
    const double *cell_vol;           /* [N]    cell volume V_I (used with body_force) */
    const double *cell_r;             /* [3][N] centre -> cell centroid r_I (with body_force) */
    const int32_t *tet_nodes;         /* [4][T] node ids; positive orientation not required */
    const int32_t *facet_I;           /* [F] */
    const int32_t *facet_J;           /* [F] */
    const double *facet_cI;           /* [3][F] */
    const double *facet_n;            /* [3][F] unit, along I->J */
    const double *facet_m;            /* [3][F] unit, orthogonal to n */
    const double *facet_area;         /* [F] projected area A_k = A0 n.n0 */
    const double *facet_len;          /* [F] edge length l_k */
    const uint8_t *dof_mode;          /* [6][N] 0 free, 1 prescribed velocity */
    const int32_t *dof_prog;          /* [6][N] program id or -1 (free: applied force
                                         scale*prog(t); prescribed: velocity) */
    const double *dof_scale;          /* [6][N] */
    int32_t n_programs;               /* piecewise-linear programs, constant beyond ends */
    const int64_t *prog_off;          /* [n_programs+1] */
    const double *prog_t;             /* [prog_off[n_programs]] increasing times */
    const double *prog_v;             /* [prog_off[n_programs]] values */
    const double *body_force;         /* [3] per unit volume, or NULL */
    const double *q0;                 /* [6][N] or NULL (zero) */
    const double *v0;                 /* [6][N] or NULL (zero) */
    const ldpm_state *init_state;     /* resume from a read state, or NULL */
    const ldpm_material *mat;
    double dt;                        /* > 0 */
    int32_t precision;                /* LDPM_PREC_FP64 or LDPM_PREC_MIXED */
    void *stream;                     /* hipStream_t for all work, or NULL (null stream) */
    /* Optional device allocator (e.g. a framework's caching allocator);
     * NULL -> hipMalloc / hipFree.  The library makes one allocation.     */
    void *(*dev_alloc)(size_t bytes, void *ctx);
    void (*dev_free)(void *ptr, void *ctx);
    void *alloc_ctx;
    /* Mass representation (eq. balance: the cell's inertia tensors M_u,
     * M_theta, I_u, I_theta).  NULL: the lumped diagonal (mass,
     * rot_inertia), as the paper's explicit solvers use.  Otherwise the
     * full rigid-body mass block of every cell about its particle centre,
     * [21][N]: the upper triangle of the symmetric 6 x 6 block, row-major
     * over (u_x, u_y, u_z, theta_x, theta_y, theta_z), i.e. entries
     * (0,0) (0,1) .. (0,5) (1,1) .. (5,5); it must be positive definite
     * (LDPM_ERR_ARG otherwise).  The step then solves, per particle, the
     * free rows M_FF a_F = f_F - M_FP a_P with the prescribed DoFs'
     * accelerations a_P, reports reactions (M a - f)_P and the kinetic
     * energy 1/2 v^T M v.  mass and rot_inertia are still required
     * (validation) but not used by the step.  Not with persistent launches. */
    const double *mass_block;
} ldpm_system_desc;

/* Energies of one specimen after the last completed step n (all at time
 * t_{n-1}, the last configuration whose internal forces were evaluated).   */
typedef struct {
    double W_ext;   /* work of applied forces and reactions */
    double W_int;   /* work of the facet tractions (trapezoid per facet) */
    double W_kin;   /* kinetic energy at step n-1, mid-step velocities averaged */
    double W_kin0;  /* initial kinetic energy */
    double W_pert;  /* work of random perturbations (ldpm_perturb), done from outside */
    double err;     /* |W_src - W_int - W_kin| / max(|W_src|, tiny), W_src = W_ext + W_pert + W_kin0 */
    int64_t step;
    double time;    /* t_{n-1} */
} ldpm_energies;

/* Validate the description, build the internal layout (facet-sorted
 * particle incidence lists, deduplicated edge frames, SoA buffers), allocate
 * device memory and upload.  On success *out owns everything.             */
ldpm_status ldpm_load_system(const ldpm_system_desc *desc, ldpm_system **out);

/* Enqueue n_steps explicit steps on the handle's stream (asynchronous);
 * LDPM_ERR_STATE on a handle that integrates implicitly. */
ldpm_status ldpm_step(ldpm_system *s, int64_t n_steps);

/* Like ldpm_step, but brackets every facet-kernel and particle-kernel launch
 * with HIP events on the handle's stream, waits after each step, and returns
 * the summed kernel times in milliseconds (for roofline measurements).
 * LDPM_ERR_STATE on a handle that integrates implicitly.                   */
ldpm_status ldpm_step_profiled(ldpm_system *s, int64_t n_steps, double *facet_ms,
                               double *particle_ms);

/* Wait for the stream; report a sticky device error. */
ldpm_status ldpm_sync(ldpm_system *s);

/* Synchronise and copy the state into caller buffers (NULL fields skipped).
 * out->step receives the number of completed steps.                       */
ldpm_status ldpm_read_state(ldpm_system *s, ldpm_state *out);

/* Synchronise and reduce the energies of one specimen in a fixed order
 * (bitwise reproducible, independent of batching).                         */
ldpm_status ldpm_energy(ldpm_system *s, int32_t specimen, ldpm_energies *out);

/* Synchronise and sum fext over every DoF whose program id is `program`
 * (the resultant reaction of a loaded face: nominal stress = sum / area). */
ldpm_status ldpm_reaction(ldpm_system *s, int32_t program, double *out);

/* Counts and layout facts: N, T, F, number of deduplicated edge frames,
 * algorithmic bytes of one facet step and of one particle step.           */
typedef struct {
    int64_t n_particles, n_tets, n_facets, n_edges, n_specimens, step;
    int32_t precision, law;
    double facet_kernel_bytes;     /* compulsory HBM bytes per facet-kernel launch */
    double particle_kernel_bytes;  /* compulsory HBM bytes per particle-kernel launch */
    size_t device_bytes;           /* device memory held by the handle */
} ldpm_info;
ldpm_status ldpm_get_info(ldpm_system *s, ldpm_info *out);

/* Launch configuration of the step: tetrahedra per facet block (8, 16, 32
 * or 64), threads per particle block (64..1024, multiple of 64), whether the
 * facet kernel's tiles are remapped so that each XCD (own L2) works on a
 * contiguous range, and whether ldpm_step runs as one persistent
 * cooperative launch per chunk of steps (facet and particle phases separated
 * by grid barriers) instead of two kernels per step (lumped mass only), and
 * whether the two-kernel step's facet kernel streams the facet records and
 * traction history past the caches (nontemporal loads and stores: what the step reuses stays
 * cached when its data exceed the last-level cache) or through them (the
 * whole step can stay cache-resident on smaller systems).  stream_facets
 * defaults to 1 when the facet kernel moves more than 256 MiB per launch,
 * else 0.  Results do not depend on any of these (bitwise).               */
typedef struct {
    int32_t tets_per_block;
    int32_t particle_threads;
    int32_t xcd_remap;
    int32_t persistent;
    int32_t stream_facets;
} ldpm_launch;
ldpm_status ldpm_set_launch(ldpm_system *s, const ldpm_launch *cfg);
ldpm_status ldpm_get_launch(ldpm_system *s, ldpm_launch *out);

/* Autotuner: times every launch shape (tets_per_block x particle_threads x
 * xcd_remap for two kernels per step, and tets_per_block for the persistent
 * launch, at the handle's stream_facets; then the best two-kernel shape
 * with stream_facets flipped) for steps_per_trial steps on the live system, keeps the
 * fastest and returns it (best, best_us = microseconds per step).  The
 * dynamic state is saved before the trials and restored afterwards (a
 * temporary device buffer of the state's size is allocated), so the
 * trajectory is unchanged.  Choices are cached for the process per (GPU
 * architecture, system shape); a cache hit returns with *n_trials = 0.
 * trials (may be NULL) receives up to max_trials timings.
 * LDPM_ERR_STATE while a surrogate is installed or a sample capture is
 * active (their hand-back flags and rows are not part of the saved state:
 * tune first) and on a handle that integrates implicitly.                  */
typedef struct {
    ldpm_launch launch;
    double us_per_step;
} ldpm_tune_trial;
ldpm_status ldpm_autotune(ldpm_system *s, int32_t steps_per_trial, ldpm_launch *best,
                          double *best_us, ldpm_tune_trial *trials, int32_t max_trials,
                          int32_t *n_trials);

/* ---- Facet-law surrogate: a small MLP trained on the GPU ------------------
 * Network 9 -> 64 -> 64 -> 64 -> 3 with tanh, parameters as one flat FP32
 * vector of ldpm_mlp_num_params() = 9155 values, weights stored [out][in]:
 *   W1[64][9] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[3][64] b4[3].
 * Forward and backward run on BF16 matrix-core tiles with FP32
 * accumulation; the trainer keeps FP32 master weights and Adam moments.
 * Loss: mean over the batch of sum_j (y_j - target_j)^2.
 * For callers that bring their own (normalised) training data; the solver
 * uses the trained parameters through ldpm_set_surrogate.                 */
typedef struct ldpm_mlp ldpm_mlp;
int32_t ldpm_mlp_num_params(void);
/* init: host FP32 parameters (copied).  stream: hipStream_t or NULL. */
ldpm_status ldpm_mlp_create(const float *init, void *stream, ldpm_mlp **out);
/* Training data: host x[n][9], y[n][3] (copied; replaces previous data). */
ldpm_status ldpm_mlp_set_data(ldpm_mlp *m, const float *x, const float *y, int64_t n);
/* Gradient (host grad[9155]) and loss of the current parameters over the
 * batch of samples offset .. offset+batch-1 (indices modulo n; batch is
 * rounded up to a multiple of 64).  No update.                              */
ldpm_status ldpm_mlp_grad(ldpm_mlp *m, int32_t batch, int64_t offset, float *grad, float *loss);
/* steps Adam updates over consecutive batches of the data (wrapping);
 * *last_loss receives the loss of the last batch.                          */
ldpm_status ldpm_mlp_train(ldpm_mlp *m, int64_t steps, int32_t batch, float lr, float *last_loss);
/* Forward pass of host x[n][9] into host y[n][3] (the surrogate's path). */
ldpm_status ldpm_mlp_forward(ldpm_mlp *m, const float *x, int64_t n, float *y);
/* Current FP32 master parameters into host params[9155]. */
ldpm_status ldpm_mlp_get_params(ldpm_mlp *m, float *params);
void ldpm_mlp_free(ldpm_mlp *m);

/* ---- Surrogate of the facet law inside the step ----------------------------
 * With a surrogate installed (precision MIXED, law 1), every facet that is
 * inside the network's envelope and has not been handed back is updated by
 * t = t_old + E de + s * (y_scale * MLP(x_hat)) instead of the exact law,
 * where s = |t_old + E de| + y_tau is the magnitude of the elastic trial
 * traction (E = E0 diag(1, alpha, alpha)), x are the facet's features in
 * the frame aligned with its trial shear traction t_old,T + alpha E0 de_T:
 *   x = [de_N, de_par, de_perp, e_N, e_par, e_perp, t_N, t_par, t_perp]_old,
 * x_hat = (x - x_mean) * x_scale, and the output is the traction residual
 * over the elastic predictor in the same frame, relative to s.  Each
 * relative residual component whose magnitude is below y_dead (the
 * network's error floor on samples whose exact residual vanishes, e.g.
 * elastic facets) is taken as exactly zero, so that such facets follow the
 * elastic predictor without drift.
 * A facet is handed back to
 * the exact FP32 law for good (sticky flag) when
 *   - a feature leaves [box_lo, box_hi] (the trained range), or
 *   - tension: its effective strain or its e_max reaches kappa_t e0(omega),
 *     the elastic limit at the current angle (kappa_t > 1 keeps the facet
 *     on the network past the peak, into softening), or
 *   - compression: -e_DV reaches kappa_c e_c0 or -t_N reaches kappa_c sigma_c0
 *     (onset of pore collapse), or
 *   - the damage D = 1 - t / (E0 e) of the surrogate's traction exceeds
 *     damage_max (D is taken as 0 while e < 0.01 sigma_t / E0, where the
 *     ratio is rounding noise).
 * NULL removes the surrogate.  (For callers comparing a learned law with the
 * exact one; the exact law stays the reference.)                           */
typedef struct {
    const float *params;                    /* [ldpm_mlp_num_params()] FP32, copied */
    float x_mean[9], x_scale[9], y_scale[3];
    float y_dead[3];                        /* >= 0; 0 disables the dead zone */
    float y_tau;                            /* >= 0 (MPa): floor of the residual scale s */
    float box_lo[9], box_hi[9];
    float kappa_t, kappa_c, damage_max;
} ldpm_surrogate;
ldpm_status ldpm_set_surrogate(ldpm_system *s, const ldpm_surrogate *sg);
/* Number of facets handed back to the exact law so far. */
ldpm_status ldpm_surrogate_count(ldpm_system *s, int64_t *n_exact);
/* Running counts since ldpm_set_surrogate (synchronises): facets handed
 * back, facet-updates made by the network, facet-updates whose damage
 * D = 1 - t/(E0 e) of the new traction lies in (1e-3, damage_max] whichever
 * law made them (the softening range the network may carry; below 1e-3 D
 * is the rounding of an elastic update), and those of them the network
 * made; and the facets handed back by each gate: the strain envelope, the
 * trained feature box (facets inside the envelope), the damage limit.
 * Integer counts, exact in any order.                                      */
typedef struct {
    int64_t handed_back, network_updates, damaged_updates, damaged_network_updates;
    int64_t handed_back_envelope, handed_back_box, handed_back_damage;
} ldpm_surrogate_counts;
ldpm_status ldpm_surrogate_stats(ldpm_system *s, ldpm_surrogate_counts *out);

/* ---- Capture of surrogate training samples from the FP64 exact law -------
 * While a capture is active (precision FP64, law 1), every step n with
 * n % step_stride == 0 records, for the facets f with
 * f % facet_stride == facet_offset that are inside the envelope (same
 * criteria as above with kappa_t, kappa_c, damage_max), one row of 16 floats:
 * x[9] (features as above), the exact residual t - (t_old + E de) in the
 * aligned frame [3] (absolute, MPa), the key n * 2^32 + f as an int64 in
 * floats 12-13, and |t_old + E de| in float 14 (float 15 is 0).
 * Rows land in arrival order; sort by key for a reproducible order.        */
typedef struct {
    int64_t capacity;         /* rows */
    int32_t facet_stride, facet_offset, step_stride;
    float kappa_t, kappa_c, damage_max;
} ldpm_capture_opts;
ldpm_status ldpm_capture_begin(ldpm_system *s, const ldpm_capture_opts *opts);
/* Ends the capture; *n_rows = rows offered (may exceed the capacity);
 * copies min(n_rows, capacity, max_rows) rows into host rows[][16].      */
ldpm_status ldpm_capture_end(ldpm_system *s, float *rows, int64_t max_rows, int64_t *n_rows);

/* ---- Crack openings, volumetric strains, field comparison ----------------
 * The paper compares two solutions of a benchmark by their final crack
 * patterns (and, for confined compression, volumetric strains) through
 * Pearson's correlation coefficient and an NRMSE (numerical-examples
 * section).  The fields are written to DEVICE memory (on the handle's GPU),
 * enqueued on the handle's stream; a host pointer is rejected
 * (LDPM_ERR_ARG).                                                          */

/* Crack-opening vector of every facet after the last completed step n,
 * w [4][F] doubles: w_N, w_M, w_L, |w|, with w = len_k (e - E^{-1} t),
 * E = E0 diag(1, alpha, alpha), e and t the strain and traction of the last
 * law evaluation (configuration q^{n-1} = q^n - dt v^{n-1/2}; before the
 * first step the undeformed one), and only a positive normal inelastic
 * strain opening a crack: w_N = max(w_N, 0).  After implicit steps the last
 * law evaluation is at the committed q_n itself.                           */
ldpm_status ldpm_crack_opening(ldpm_system *s, double *w);

/* Volumetric strain e_V of every tetrahedron at the configuration of the
 * last law evaluation (zero before the first step), ev [T] doubles.        */
ldpm_status ldpm_volumetric_strain(ldpm_system *s, double *ev);

/* Comparison of a field x with a reference field ref (n doubles each, in
 * DEVICE memory of the current GPU): Pearson's correlation coefficient and
 * NRMSE = 100 / max(ref) * sqrt(mean (x - ref)^2), in percent.  cap > 0 and
 * finite: both fields are limited to cap first (the paper limits crack
 * openings to 4 mm where detached fragments would dominate); otherwise no
 * limit.  The reduction order depends on n only (bitwise reproducible).
 * IEEE results for degenerate fields: pearson is NaN when either field is
 * constant, nrmse is inf or NaN when max(ref) is 0.  Runs on `stream`
 * (hipStream_t or NULL) and synchronises it.  The first call on a device
 * allocates a 128 KiB buffer kept for the process; concurrent calls are
 * serialised.                                                              */
typedef struct {
    int64_t n;
    double mean_x, mean_ref;
    double pearson;
    double rmse;     /* sqrt(mean (x - ref)^2) */
    double ref_max;  /* max ref (after the cap): the normalisation */
    double nrmse;    /* percent */
} ldpm_field_stats;
ldpm_status ldpm_compare_fields(const double *x, const double *ref, int64_t n, double cap, void *stream,
                                ldpm_field_stats *out);

/* Allocation-free variant of ldpm_compare_fields, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, validation,
 * results (bitwise) and errors as ldpm_compare_fields; it calls no hipMalloc,
 * hipFree or other allocating routine.  Its block partials and results live
 * in a file-scope device array of the library (2048 partials of 64 bytes
 * plus the results, about 128 KiB), one per GPU, held until the process
 * ends; the first call on a device resolves that array's address there.
 * The scratch need does not grow with n (the grid is capped at 2048
 * blocks), so no n is refused for size.  Every call on a GPU uses the same
 * array: calls that overlap on one GPU (several host threads or streams at
 * once) race on it, and the caller must serialise them.  Each call writes
 * every partial it reads, so nothing is carried from the previous call.
 * Synchronises `stream` before returning.                                  */
ldpm_status ldpm_compare_fields_noalloc(const double *x, const double *ref, int64_t n, double cap,
                                        void *stream, ldpm_field_stats *out);

/* ---- Random perturbation of the solution ---------------------------------
 * The paper tests the stability of a strain-softening response by adding,
 * at regular intervals, a random vector uniform in [-eta/2, eta/2] to all
 * free displacements and rotations (section on the numerical study of time
 * step, convergence criteria and stability).  ldpm_perturb adds delta (HOST
 * memory [6][N], copied; the caller draws it) to every free DoF of q^n;
 * prescribed DoFs keep their values, velocities are unchanged.  The facet
 * law takes the jump as a strain increment of its own, at once: from the
 * configuration of the last law evaluation (q^{n-1} = q^n - dt v^{n-1/2}) to
 * that configuration plus the jump, so that the next step starts from a
 * history consistent with the perturbed positions (the paper does not say
 * how the history sees the jump; this is the reading taken).  The
 * traction work of the jump is added to the internal work and, as work done
 * from outside, to W_pert of each specimen.  Before the first step there is
 * no history: the jump only changes the initial displacement.  With a
 * surrogate installed the jump still goes through the exact law, and a
 * capture records nothing for it.  *work (may be NULL) receives the work of
 * this jump over all specimens.  Synchronises the stream.  The first call
 * allocates a device buffer of about 8 (6N + 2T) bytes, kept by the handle.
 * Explicit runs only (LDPM_ERR_STATE after implicit steps).               */
ldpm_status ldpm_perturb(ldpm_system *s, const double *delta, double *work);

/* ---- Implicit generalised-alpha / HHT-alpha integration ------------------
 * The paper's implicit solvers integrate the same equations with the HHT
 * (Hilber-Hughes-Taylor) alpha or generalised-alpha methods and Newton-type
 * iterations.  ldpm_implicit_step advances n_steps steps of the
 * generalised-alpha family with interpolated forces:
 *   (1 - a_m) M a_{n+1} + a_m M a_n
 *       = (1 - a_f)(g(q_{n+1}) + f_{n+1}) + a_f (g(q_n) + f_n) + R_{n+1},
 *   q_{n+1} = q_n + dt v_n + dt^2 ((1/2 - beta) a_n + beta a_{n+1}),
 *   v_{n+1} = v_n + dt ((1 - gamma) a_n + gamma a_{n+1}),
 *   gamma = 1/2 - a_m + a_f, beta = (1 - a_m + a_f)^2 / 4,
 * with a_m = alpha_m, a_f = alpha_f.  HHT-alpha is a_m = 0, a_f = -alpha
 * (alpha in [-1/3, 0]; 0: the trapezoidal rule); the generalised-alpha
 * method with high-frequency spectral radius rho in [0, 1] is
 * a_m = (2 rho - 1)/(rho + 1), a_f = rho/(rho + 1).
 * g = -f_int (the gathered facet forces), f the applied forces, R the
 * reactions of prescribed DoFs, which move by dt v_P(t_n + dt/2).  Each step
 * is solved by modified Newton on the free DoFs with the initial elastic
 * stiffness K0: K_eff = (1 - a_m) M / (beta dt^2) + (1 - a_f) K0, its systems
 * solved by conjugate gradients with K0 applied matrix-free (the facet
 * kernel of the elastic law), preconditioned by the inverse 6 x 6 blocks of
 * K_eff that couple each particle's DoFs with themselves.  Every Newton iteration
 * evaluates the facet law at the trial configuration from the committed
 * history; the last trial is committed when the step is accepted: when
 * |R_F|_2 <= tol (|((1 - a_m) M a)_F|_2 + |rhs_F|_2) or after max_iter
 * iterations (counted in not_converged).  The predictor keeps the
 * acceleration.  The state then holds q_n, v_n (not the explicit scheme's
 * mid-step velocities): a handle integrates either explicitly or implicitly
 * (LDPM_ERR_STATE otherwise), and dt, alpha_m, alpha_f stay fixed after the
 * first implicit step.  FP64, lumped mass, no surrogate or capture.
 * Energies as for the explicit step (W_int facet trapezoids of accepted
 * steps, W_ext the trapezoid of applied + reaction forces, W_kin =
 * 1/2 v^T M v) at t_n = n dt.  The first call allocates device buffers of
 * about 8 (120 N + 7 F + 26 T) bytes, kept by the handle.  Synchronises.   */
typedef struct {
    double dt;           /* implicit time step (> 0) */
    double alpha_m;      /* >= -1 (HHT: 0) */
    double alpha_f;      /* alpha_m <= alpha_f <= 1/2 (HHT: -alpha) */
    double tol;          /* relative Newton tolerance (> 0) */
    int32_t max_iter;    /* Newton iterations per step (>= 1) */
    double cg_tol;       /* relative residual of the CG solves (> 0) */
    int32_t cg_max_iter; /* CG iterations per solve (>= 1) */
} ldpm_implicit_opts;
typedef struct {
    int64_t steps, newton_iters, cg_iters, not_converged;
    double max_residual; /* largest relative Newton residual of an accepted step */
} ldpm_implicit_stats;
ldpm_status ldpm_implicit_step(ldpm_system *s, const ldpm_implicit_opts *opts, int64_t n_steps,
                               ldpm_implicit_stats *stats);

/* ---- On-device tessellation ------------------------------------------------
 * LDPM geometry from particle centres, diameters and a tetrahedralisation
 * (the paper's preprocessing: polyhedral cells around the particles and the
 * triangular facets between them; its own generator is not available, so
 * this is the construction documented with the project's input generator):
 * on every tetrahedron edge a point at mid-gap between the particle
 * surfaces, s = (l + r_a - r_b)/2 from x_a clamped to [0.05, 0.95] l; face
 * points at the centroids of their edge points; the tetrahedron point at the
 * centroid of the face points; two facets per edge, (edge point, point of
 * the face through the edge and the third node c, tetrahedron point),
 * ordered by edge (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) and then by c.  Facet
 * k joins I < J (particle ids), n = (x_J - x_I)/l, m = normalise(n x e_k)
 * with e_k the axis of the smallest |n_k|, A0 the triangle's area, A = A0
 * n.n0 its projection (eq. balance), c^I from x_I to the triangle centroid.
 * Cells: the exact cone integrals (centre, facet triangle) give volume,
 * mass = rho V, the inertia tensor J about the centre and the centroid
 * offset r.  All arrays are HOST memory owned by the caller; NULL outputs
 * are skipped.  Runs on `stream` (hipStream_t or NULL), allocates and frees
 * its device buffers, synchronises.  Errors: LDPM_ERR_ARG (no tetrahedra,
 * a node id out of range or repeated within a tetrahedron, a non-positive
 * or non-finite diameter or density, non-finite centres; checked on the
 * host before any device work), LDPM_ERR_ALLOC, LDPM_ERR_DEVICE.          */
typedef struct {
    int64_t n_particles, n_tets;
    const double *x;           /* [3][N] centres */
    const double *diam;        /* [N] particle diameters (> 0) */
    const int32_t *tet_nodes;  /* [4][T] four distinct node ids each */
    double rho;                /* density (> 0) */
} ldpm_tess_desc;
typedef struct {
    int32_t *facet_I, *facet_J;                     /* [F], F = 12 T */
    double *facet_cI, *facet_n, *facet_m;           /* [3][F] */
    double *facet_area, *facet_area0, *facet_len;   /* [F] */
    double *mass, *cell_vol;                        /* [N] */
    double *rot_inertia, *cell_r;                   /* [3][N]: diagonal of J; centroid offset */
    double *cell_inertia;                           /* [6][N]: J_xx J_yy J_zz J_xy J_yz J_xz */
    double *tet_node_cones;                         /* [T][4][10]: each tet's part of its nodes'
                                                       cells: V, first moment (3), second moment
                                                       (xx yy zz xy yz xz) about the node */
} ldpm_tess_out;
ldpm_status ldpm_tessellate(const ldpm_tess_desc *desc, ldpm_tess_out *out, void *stream);

/* ---- Element bound of the stable explicit step --------------------------
 * The paper sets the explicit step from an eigenvalue analysis of each
 * tetrahedron (section on free vibrations in the linear elastic regime):
 * lam[t] = largest eigenvalue of W K_e W for tetrahedron t, with K_e the
 * elastic stiffness of its 12 facets, sum (A/l) B^T D B, B = [-1, [c^I]x]
 * at the facet's I node and [1, -[c^J]x] at its J node (eq. strain1,
 * c^J = c^I - l n), D = E0 (alpha 1 + (1 - alpha) n n^T), and W =
 * diag(share)^(-1/2) from the tetrahedron's share of its four nodes' lumped
 * masses.  max_t lam[t] bounds the assembled system's largest eigenvalue;
 * dt = fraction * 2 / sqrt(max lam).  Facets tet-major (facet 12 t + k of
 * tetrahedron t), each joining two nodes of its tetrahedron.  DoF order per
 * node (u_x, u_y, u_z, th_x, th_y, th_z).  HOST arrays owned by the caller;
 * runs on `stream`, allocates and frees its device buffers, synchronises.
 * Errors: LDPM_ERR_ARG for inconsistent or non-finite input. */
typedef struct {
    int64_t n_particles, n_tets;
    const int32_t *tet_nodes;                 /* [4][T] */
    const int32_t *facet_I, *facet_J;         /* [F], F = 12 T */
    const double *facet_cI, *facet_n;         /* [3][F] */
    const double *facet_area, *facet_len;     /* [F] */
    const double *share;                      /* [T][4][6] (> 0) */
    double E0, alpha;
} ldpm_elem_desc;
ldpm_status ldpm_element_lambda(const ldpm_elem_desc *desc, double *lam, void *stream);

/* Reference streaming kernels, for measurement: the HBM bandwidth that
 * plain coalesced traffic reaches on the device, the practical ceiling that
 * the step's kernels are compared with beside the nominal peak.  Enqueues
 * ONE launch on `stream` (hipStream_t or NULL) and returns; the caller times
 * it (events on the same stream).  One 16-byte element per lane, one pass,
 * nontemporal loads and stores.  DEVICE buffers owned by the caller,
 * 16-byte aligned; `bytes` is the traffic the launch moves:
 *   LDPM_STREAM_COPY: reads bytes/2 from src, writes them to dst;
 *   LDPM_STREAM_READ: reads `bytes` from src, writes one double per 4 KiB
 *                     block of src to dst (dst holds bytes/512 bytes);
 *   LDPM_STREAM_FILL: writes `bytes` to dst (src unused, may be NULL);
 *   LDPM_STREAM_MIX:  three reads and two writes per element: reads 3/5 of
 *                     `bytes` from src, writes 2/5 to dst.
 * Errors: LDPM_ERR_ARG for an unknown kind, null or misaligned buffers, or
 * bytes not a positive multiple of 32 (COPY), 16 (READ, FILL) or 80 (MIX);
 * LDPM_ERR_DEVICE if the launch fails. */
enum { LDPM_STREAM_COPY = 0, LDPM_STREAM_READ = 1, LDPM_STREAM_FILL = 2, LDPM_STREAM_MIX = 3 };
ldpm_status ldpm_stream_probe(int kind, const void *src, void *dst, int64_t bytes, void *stream);

/* Release device memory and the handle (NULL is a no-op). */
void ldpm_free(ldpm_system *s);

/* Thread-local message of the last failing call ("" if none). */
const char *ldpm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LDPM_H */
