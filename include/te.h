/*
 * te.h -- C ABI of the MI355X (gfx950) thermoelastic PCG + smoothed-aggregation
 * AMG library.
 *
 * The library solves the linear thermoelastic problem of the paper's Sec. 3
 * (eqs. elasticity_bvp, u-dbc and the weak form wf_elastic, the boundary
 * pressure term included in fe_assemble_thermoelastic_materials):
 *   -div(C:(eps(u) - alpha (T - T_ref) I)) = f  on a tetrahedral
 * mesh with Lagrange P1 or P2 elements (Sec. 3.1), by conjugate gradients
 * preconditioned with smoothed-aggregation AMG using the rigid-body modes as
 * near-nullspace and a Chebyshev smoother (Sec. 2.1.2, 2.1.3 and 5.1).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller unless the
 *     comment says "host".  Arrays are dense, contiguous, row-major.
 *   - Vector unknowns are node-major: DOF 3*i + c is component c of node i.
 *   - All device work is enqueued on the caller's stream; calls return once
 *     the work is enqueued unless stated otherwise (setup and solve
 *     synchronise the stream because they need host-side decisions).
 *   - Return codes: 0 OK, >0 completed with a warning, <0 error (see below).
 *     te_last_error() gives a thread-local message for the last failure.
 *   - Handles are not safe for concurrent use from several threads.
 */
#ifndef TE_H
#define TE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define TE_OK          0
#define TE_ENOTCONV    1   /* maxit reached; result and report are valid     */
#define TE_EINVAL    (-1)  /* bad argument (null pointer, size, option)      */
#define TE_ENOMEM    (-2)  /* device or host allocation failed               */
#define TE_EHIP      (-3)  /* a HIP runtime call failed                      */
#define TE_EINDEF    (-4)  /* CG breakdown: (p,Ap) <= 0 or (r,z) <= 0         */
#define TE_ENAN      (-5)  /* NaN or Inf in a residual                       */
#define TE_ERANK     (-6)  /* aggregate near-nullspace block of rank < 6     */
#define TE_ECHOL     (-7)  /* coarsest-level pivot <= 0 (not SPD)            */

#define TE_PREC_FP64   0   /* everything in float64 (the reference method)   */
#define TE_PREC_MIXED  1   /* float32 V-cycle inside float64 flexible CG     */

/* Library version (major*10000 + minor*100 + patch). */
int te_version(void);
/* Thread-local text of the last error ("" if none). Host string, static. */
const char *te_last_error(void);

/* ---- inputs (Sec. 3.1: conforming Lagrange spaces on tetrahedra) ------- */
typedef struct {
    int64_t n_nodes;        /* N: vertices (P1) or vertices + edge nodes (P2) */
    int64_t n_cells;        /* C                                               */
    int32_t degree;         /* 1 or 2                                          */
    const double *coords;   /* device [N][3]                                   */
    const int32_t *cells;   /* device [C][4] (P1) or [C][10]: v0..v3 then the
                               edge nodes e01,e02,e03,e12,e13,e23 (P2); every
                               cell positively oriented, P2 edge nodes at the
                               straight-edge midpoints (affine cells)          */
} te_mesh;

typedef struct {            /* isotropic material: C from (E, nu)             */
    double E, nu;           /* Young's modulus, Poisson ratio                 */
    double alpha;           /* thermal expansion coefficient alpha_L          */
    double T_ref;           /* reference temperature of the thermal strain    */
} te_material;

/* 3x3-block compressed sparse rows (node-node coupling blocks). */
typedef struct {
    int64_t n_brows;        /* N                                              */
    int64_t nnzb;           /* number of stored 3x3 blocks                    */
    int64_t *row_ptr;       /* device [N+1]                                   */
    int32_t *col_idx;       /* device [nnzb], ascending within a row          */
    double *val;            /* device [nnzb][3][3], block row-major:
                               val[k][i][j] couples component i of the row
                               node with component j of the column node       */
} te_bsr;

/* ---- assembly (Sec. 2.3.3, weak form wf_elastic) ----------------------- */

/* Block sparsity of the stiffness matrix: node I couples with node J when
 * both belong to one cell (diagonal blocks included).
 *   row_ptr: device [N+1], written (row_ptr[0] = 0).
 *   nnzb_out: host, receives row_ptr[N].
 * Synchronises `stream`.  Errors: TE_EINVAL (bad mesh, node index out of
 * range, a node coupling to more than 192 nodes), TE_ENOMEM, TE_EHIP. */
int fe_assemble_pattern(const te_mesh *mesh, int64_t *row_ptr, int64_t *nnzb_out, hipStream_t stream);

/* Stiffness matrix and load vector of the thermoelastic weak form,
 *   K[(a,i),(b,j)] = int lam d_i phi_a d_j phi_b + mu d_j phi_a d_i phi_b
 *                        + mu delta_ij grad phi_a . grad phi_b
 *   b[(a,i)]       = (3 lam + 2 mu) alpha int (T_h - T_ref) d_i phi_a + int f_i phi_a
 * (T_h the nodal interpolant of T in the same space; exact integration),
 * followed by Dirichlet elimination that keeps every DOF: b -= A[:,D] u_D,
 * rows and columns of constrained DOFs zeroed, unit diagonal, b_D = u_D.
 *   T: device [N]; f: device [N][3] or NULL (no body force);
 *   dir_mask: device [N][3] uint8 (nonzero = constrained) or NULL;
 *   u_bc: device [N][3] prescribed values or NULL (= 0);
 *   A: row_ptr from fe_assemble_pattern, col_idx/val caller-allocated with
 *      A->nnzb entries; both are overwritten.  b: device [3N], overwritten.
 * Deterministic (gather-based, no atomics in the sums).  Errors: TE_EINVAL,
 * TE_ENOMEM, TE_EHIP. */
int fe_assemble_thermoelastic(const te_mesh *mesh, const te_material *mat, const double *T,
                              const double *f, const uint8_t *dir_mask, const double *u_bc,
                              te_bsr *A, double *b, hipStream_t stream);

/* Temperature-dependent isotropic materials (Sec. 3: C and alpha_L depend on
 * T; Sec. 4.2 shows such tables for several materials).  Material m gives E,
 * nu and alpha_L at n_points temperatures T[m][k] (strictly ascending); values
 * between samples are linear in T, beyond the first and last sample constant.
 * All arrays are host arrays [n_materials][n_points], read during the call. */
typedef struct {
    int32_t n_materials;
    int32_t n_points;
    const double *T;
    const double *E;        /* > 0                                            */
    const double *nu;       /* in (-1, 0.5)                                   */
    const double *alpha;
    double T_ref;           /* reference temperature of the thermal strain    */
} te_material_tables;

/* Boundary pressure of eq. wf_elastic: traction p_bc n on Gamma_N, p_bc
 * constant on each boundary triangle.  faces: device [n_faces][3] vertex
 * ids (P1) or [n_faces][6]: the three vertices, then the edge nodes 01, 02,
 * 12 of that vertex order (P2); n = (x1 - x0) x (x2 - x0) / |.| must point
 * out of the body.  p: device [n_faces]. */
typedef struct {
    int64_t n_faces;
    const int32_t *faces;
    const double *p;
} te_pressure;

/* fe_assemble_thermoelastic with per-cell coefficients and the boundary
 * pressure: cell c takes the values of material cell_material[c] (device
 * [C], 0..n_materials-1) at the mean of T_h over the cell, so lam, mu and
 * alpha_L are constant per cell; b gains int_F p_bc n . phi_a ds on every
 * pressure face (exact: |F|/3 per node for P1; 0 at the vertices and |F|/3
 * at the edge nodes for P2), before the Dirichlet elimination.  pressure may
 * be NULL (or hold no faces).  Other arguments, layouts and the elimination
 * as in fe_assemble_thermoelastic.  Deterministic.  Errors: TE_EINVAL (bad
 * tables, a material id or face node out of range), TE_ENOMEM, TE_EHIP. */
int fe_assemble_thermoelastic_materials(const te_mesh *mesh, const te_material_tables *mat,
                                        const int32_t *cell_material, const double *T,
                                        const double *f, const te_pressure *pressure,
                                        const uint8_t *dir_mask, const double *u_bc, te_bsr *A,
                                        double *b, hipStream_t stream);

/* Load vector only (same b as above with u_bc = 0), for many load cases on
 * one assembled matrix.  nrhs load cases: T device [nrhs][N], f device
 * [nrhs][N][3] or NULL; b device [N][3][nrhs] (right-hand sides fastest). */
int fe_assemble_load(const te_mesh *mesh, const te_material *mat, const double *T,
                     const double *f, const uint8_t *dir_mask, int32_t nrhs,
                     double *b, hipStream_t stream);

/* ---- smoothed-aggregation AMG (Sec. 2.1.3, 5.1) ------------------------- */
typedef struct amg_handle amg_handle;

/* Aggregation of each level (the rule is a reading: Sec. 5.1 names the
 * library the paper uses and its defaults, not the rule; that library
 * aggregates by maximal independent sets):
 *   TE_AGG_GREEDY  sequential greedy in node order on the host (phase 1: a
 *                  free node whose strong neighbours are all free roots an
 *                  aggregate of them; phase 2: the rest join the aggregate of
 *                  their strongest aggregated neighbour);
 *   TE_AGG_MIS2    on the device: the phase-1 roots are the maximal
 *                  distance-2 independent set of the (symmetrised) strong
 *                  graph chosen in parallel rounds by the fixed keys
 *                  (splitmix64((0xA66 + level) ^ node) >> 33, node), which is
 *                  the set the sequential phase 1 picks when it visits nodes
 *                  by descending key; aggregates numbered by ascending root;
 *                  phase 2 as above.  No strength values cross to the host
 *                  unless an aggregate is rank deficient. */
#define TE_AGG_GREEDY 0
#define TE_AGG_MIS2   1

typedef struct {
    double theta0;           /* strength threshold at level 0, halved per level (0.08) */
    int32_t coarse_max;      /* stop coarsening at <= this many DOF (3000)            */
    int32_t max_levels;      /* (10)                                                    */
    int32_t lanczos_steps;   /* steps of the largest-eigenvalue estimate (20)         */
    int32_t cheb_degree;     /* Chebyshev polynomial degree (2)                        */
    double cheb_ratio;       /* interval [b/ratio, b] (10)                              */
    double cheb_safety;      /* b = safety * lambda_hat (1.1)                           */
    double max_coarse_ratio; /* stop if a coarse level keeps more than this share (0.8) */
    int32_t build_fp32;      /* also keep float32 copies for TE_PREC_MIXED (1)         */
    int32_t host_threads;    /* host threads for the setup (0 = all)                    */
    int32_t max_nrhs;        /* largest nrhs a solve will use (1..64; 1)               */
    int32_t coarse_sym;      /* store the float64 coarse operators (6x6 blocks) by the
                                blocks on and above the diagonal, the others read
                                transposed from their mirror (symmetric pattern only;
                                float32 copies keep full storage) (1)                   */
    int32_t aggregation;     /* TE_AGG_MIS2 (default) or TE_AGG_GREEDY                   */
    int32_t smooth_filtered; /* 1: smooth the prolongator with the filtered operator:
                                per block row the strong blocks (s_IJ or s_JI >= theta_l)
                                and the diagonal block plus the dropped blocks; D and
                                lambda_hat stay those of A (0)                          */
} amg_options;

/* Fills the defaults listed above. */
void amg_options_default(amg_options *opt);

/* Builds the hierarchy for the Dirichlet-eliminated matrix A (3x3 blocks).
 *   coords: device [N][3] (rigid-body modes about the node centroid);
 *   dir_mask: device [N][3] or NULL: near-nullspace rows of constrained DOFs
 *             are zeroed;
 *   out: receives a library-owned handle (release with amg_destroy).
 * The rigid-body modes, strength of connection, the MIS-2 aggregation, the
 * per-aggregate QR of the tentative prolongator, prolongator smoothing, the
 * products A P and P^T (A P), the packing into the solver layouts and the
 * coarsest inverse run on the device.  On the host (host_threads threads):
 * the greedy aggregation when chosen, the merge of a rank-deficient
 * aggregate into a neighbour (the level's QR then runs on the host), the
 * storage orders and the aggregate ids of the MIS-2 roots.  Only the row
 * pointers, the coarse patterns and the aggregate maps cross to the host (the
 * mesh level's columns and strengths too under the greedy rule or a merge).
 * The matrix values are copied; A may be freed afterwards.  Synchronises
 * `stream`.  Errors: TE_EINVAL, TE_ENOMEM, TE_EHIP, TE_ERANK, TE_ECHOL. */
int amg_setup(const te_bsr *A, const double *coords, const uint8_t *dir_mask,
              const amg_options *opt, amg_handle **out, hipStream_t stream);

/* Test hook: as amg_setup, but the aggregate map of levels 0..n_levels_given-1
 * is imposed instead of computed (host arrays agg[l][n_l], -1 = isolated,
 * aggregate ids 0..n_agg-1 in creation order).  Used to drive the hierarchy
 * from an external aggregation for component-level comparisons. */
int amg_setup_with_aggregates(const te_bsr *A, const double *coords, const uint8_t *dir_mask,
                              const amg_options *opt, const int32_t *const *agg,
                              int32_t n_levels_given, amg_handle **out, hipStream_t stream);

typedef struct {
    int32_t n_levels;
    int64_t n_dof[16];       /* DOF per level                                   */
    int64_t nnzb[16];        /* stored blocks of A_l                            */
    int32_t bs[16];          /* block size of A_l                               */
    double lambda_hat[16];   /* largest-eigenvalue estimate of D^-1 A_l          */
    int64_t p_nnzb[16];      /* stored blocks of P_l                            */
    double setup_ms;         /* host wall time of the setup                      */
    int64_t bytes_device;    /* device memory held by the handle                 */
} amg_info;

int amg_get_info(const amg_handle *h, amg_info *info);

/* Host copy of the aggregate map of level l (n_l entries, natural order). */
int amg_get_aggregates(const amg_handle *h, int32_t level, int32_t *agg_host);

/* Host copy of A_l in natural (un-permuted) numbering:
 * row_ptr [n_l+1], col [nnzb], val [nnzb][bs][bs]; pass NULL arrays to query
 * sizes through *n_rows_out / *nnzb_out first. */
int amg_get_level_matrix(const amg_handle *h, int32_t level, int64_t *n_rows_out, int64_t *nnzb_out,
                         int64_t *row_ptr, int32_t *col, double *val);

/* Component access in natural numbering of level l (device vectors, float64),
 * for parity tests and diagnostics:
 *   TE_OP_A       y = A_l x
 *   TE_OP_P       y = P_l x        (x on level l+1)
 *   TE_OP_R       y = P_l^T x      (y on level l+1)
 *   TE_OP_SMOOTH  y = Chebyshev(A_l, g = x, x0 = y)   (y in: x0, out: result)
 *   TE_OP_VCYCLE  y = V-cycle from level l applied to x
 * `precision` selects the float64 or float32 operator copies. */
#define TE_OP_A       0
#define TE_OP_P       1
#define TE_OP_R       2
#define TE_OP_SMOOTH  3
#define TE_OP_VCYCLE  4
int amg_apply(amg_handle *h, int32_t level, int32_t op, int32_t precision,
              const double *x, double *y, hipStream_t stream);

/* ---- preconditioned conjugate gradients (Sec. 2.1.2) -------------------- */
typedef struct {
    double rtol;             /* stop at true |b - A u|_2 <= rtol |b|_2 (1e-8)           */
    int32_t maxit;           /* (500)                                                   */
    int32_t precision;       /* TE_PREC_FP64 or TE_PREC_MIXED                           */
    int32_t max_replace;     /* residual replacements after a failed true check (3)     */
    int32_t profile;         /* 1: time each kernel class with HIP events (0)           */
    int32_t block;           /* 1: block CG over the columns when nrhs > 1, float64
                                only (0; see amg_pcg_solve)                             */
} pcg_options;

/* Kernel classes timed when pcg_options.profile = 1 (level 0 = mesh level):   */
#define TE_K_AP        0   /* q = A_0 p with the (p,q) partial sums            */
#define TE_K_PRE       1   /* level-0 pre-smoothing Chebyshev step            */
#define TE_K_RESID     2   /* level-0 residual s = g - A_0 x                  */
#define TE_K_RESTRICT  3   /* R_0 s                                           */
#define TE_K_PROLONG   4   /* x += P_0 e                                      */
#define TE_K_POSTINIT  5   /* level-0 post-smoothing start r = g - A_0 x      */
#define TE_K_POST      6   /* level-0 post-smoothing Chebyshev step           */
#define TE_K_COARSE    7   /* all work on levels >= 1 (incl. the dense solve) */
#define TE_K_VECTOR    8   /* level-0 vector kernels (CG updates, dots)       */
#define TE_K_COUNT     9

void pcg_options_default(pcg_options *opt);

typedef struct {
    /* host arrays of nrhs entries each, filled if non-NULL */
    int32_t *iters;          /* iterations (A p products) per right-hand side          */
    int32_t *converged;      /* 1 if the true residual met rtol                         */
    double *relres_true;     /* final |b - A u| / |b|                                  */
    /* host array of (maxit + 1) * nrhs relative recurrence residuals, entry
       [k * nrhs + j] after iteration k of column j (NaN after it stopped), or NULL */
    double *history;
    /* outputs */
    int32_t max_iters;
    double time_ms;          /* elapsed device time of the solve (HIP events)           */
    double kernel_ms[TE_K_COUNT];       /* summed event time per class (profile = 1) */
    int32_t kernel_launches[TE_K_COUNT];
} pcg_report;

/* Solves A U = B for nrhs right-hand sides (1..max_nrhs of the setup).
 *   b: device [N][3][nrhs] (nrhs = 1: [3N]);
 *   u: device [N][3][nrhs]; in: initial guess, out: solution.
 *   rep: host, may be NULL.
 * Each column runs its own CG recurrence (the columns share every sparse
 * product); a converged column is frozen.  MIXED runs the V-cycle in float32
 * and uses the flexible beta.
 * With opt->block = 1 and nrhs > 1 the columns instead share one block
 * Krylov space (block CG, O'Leary 1980, with the search block orthonormalised
 * each step and numerically dependent directions dropped): every column takes
 * the same number of iterations, usually fewer than its own CG, and the stop
 * test waits for all of them; iters[j] is that common count, history is NaN,
 * the per-kernel profile is not kept, and the setup's solve workspace for
 * nrhs columns is used, plus Gram and update buffers that the first block
 * solve adds to the handle (kept for later calls).  Block CG
 * with MIXED is TE_EINVAL; a block P^T A P that is not positive definite is
 * TE_EINDEF.  Synchronises `stream`.
 * Returns TE_OK, TE_ENOTCONV (some column hit maxit), TE_EINDEF, TE_ENAN,
 * TE_EINVAL, TE_EHIP. */
int amg_pcg_solve(amg_handle *h, const double *b, double *u, int32_t nrhs,
                  const pcg_options *opt, pcg_report *rep, hipStream_t stream);

/* Solves n independent systems at once, system i with its own hierarchy
 * h[i] (from amg_setup; same Chebyshev degree), right-hand side b[i] and
 * guess/solution u[i] (device [3 N_i] each, float64 only).  Every phase of
 * the CG iteration is one persistent launch over a queue of (mesh, level,
 * row-tile) work, and one iteration is captured once as a HIP graph and
 * replayed; each system keeps its own CG recurrence and stop test, so system
 * i gets the standalone amg_pcg_solve of b[i] (up to the summation order of
 * reductions).  rep: host array of n reports (nrhs = 1 each) or NULL;
 * time_ms is the elapsed time of the whole batch.  The handles' solve
 * workspaces are used, so they must not be in use elsewhere meanwhile.
 * Returns TE_OK, TE_ENOTCONV, TE_EINDEF, TE_ENAN, TE_EINVAL, TE_EHIP. */
int amg_pcg_solve_multi(amg_handle **h, int32_t n, const double *const *b, double *const *u,
                        const pcg_options *opt, pcg_report *rep, hipStream_t stream);

/* Autotuner of amg_pcg_solve_multi for the set h[0..n-1]: times the grouped
 * launches (one V-cycle of every system plus the level-0 product, median of
 * 5 after a warm-up) for a persistent grid of 1, 2 or 4 times the workgroups
 * the device holds at once and for the work items in the order given or
 * largest system first, and keeps the fastest in every handle (later
 * amg_pcg_solve_multi calls on them use it).  report (host, may be NULL):
 * text of the choice.  Overwrites the handles' solve workspaces; synchronises.
 * Returns TE_OK, TE_EINVAL, TE_EHIP. */
int te_autotune_multi(amg_handle **h, int32_t n, char *report, int64_t report_len, hipStream_t stream);

/* Initial-guess scaling for CG: u0 <- gamma u0 with
 * gamma = (b, u0) / (u0, A u0), the multiple of the guess of least energy
 * (smallest A-norm error along u0); gamma = 0, i.e. the zero guess, when
 * (b, u0) <= 0 or (u0, A u0) <= 0.  b, u0: device [3N]; *gamma: host or NULL.
 * Synchronises `stream`. */
int amg_energy_scale(amg_handle *h, const double *b, double *u0, double *gamma, hipStream_t stream);

/* Autotuner: for every level operator (A_l, P_l, R_l; float64 and, if built,
 * float32) times the launch configurations (waves per workgroup 1/2/4/8,
 * slices or rows per wave 1/2/4, XCD-contiguous block order on/off,
 * non-temporal matrix loads on/off; for the operators stored one wave per
 * row (6-row blocks), each also with the x entries of a block column loaded
 * once per block slot and shared by lane permutes, the same values in the
 * same order; median of 5 launches) and keeps the fastest in the handle.  cache_path (host string, may be NULL): if
 * use_cache, choices already stored there for the same operator class
 * (layout, block shape, dtype, row-count octave, blocks per row) are applied
 * without timing; the merged choices are written back.  report (host, may be
 * NULL): a text summary, truncated to report_len bytes.  Synchronises. */
int te_autotune(amg_handle *h, const char *cache_path, int32_t use_cache, char *report, int64_t report_len,
                hipStream_t stream);

/* ---- transient runs (Sec. 3.3, Sec. 5.3) -------------------------------- */

/* Preconditioner reuse across time steps (Sec. 5.3: the elastic
 * preconditioner of the first step serves the later ones).  From this call
 * on, the CG products and residuals of amg_pcg_solve and amg_energy_scale use
 * A, while the V-cycle (level-0 smoother included) keeps the matrices the
 * hierarchy was built from.  A: device arrays as for amg_setup, with the same
 * block pattern as the setup matrix (checked: block rows, block count and a
 * 64-bit hash of row pointers and columns); its values are copied into
 * library storage, so A may be freed afterwards.  A = NULL goes back to the
 * setup matrix.  amg_pcg_solve_multi rejects a handle with such an operator.
 * Synchronises `stream`.  Returns TE_OK, TE_EINVAL (NULL handle, different
 * pattern), TE_ENOMEM, TE_EHIP. */
int amg_set_operator(amg_handle *h, const te_bsr *A, hipStream_t stream);

/* Time-step control of eq. dt_spec.  For a step of length dt that took the
 * temperature from T_old to T_new (device [n] each):
 *   dT = max_i |T_new[i] - T_old[i]|  (reduced on the device; exact);
 *   dT <= dT_max: *accept = 1, *dt_next = eps * dT_max / dT * dt
 *                 (2 dt when dT = 0, where the formula has no value);
 *   dT >  dT_max: *accept = 0, *dt_next = dt / 2 (repeat the step).
 * Outputs are host pointers; max_change may be NULL.  Needs dt > 0,
 * dT_max > 0, 0 < eps <= 1.  Synchronises `stream`.  Returns TE_OK,
 * TE_EINVAL, TE_ENAN (a NaN in either field), TE_EHIP. */
int te_timestep(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max, double eps,
                double *dt_next, int32_t *accept, double *max_change, hipStream_t stream);

/* te_timestep for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, checks, results and errors, but the partial maxima
 * live in a file-scope device array of the library (1088 doubles, 8.5 KB per
 * GPU, held until the process ends) instead of a buffer allocated per call,
 * and the call makes no device or host allocation.  Any n >= 0 fits: the
 * reduction folds n entries into at most 1024 partials.  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (several
 * threads or streams at once) race; the array is fully rewritten by each
 * call before it is read.  The first call on a device looks up the array's
 * device address on the current device. */
int te_timestep_noalloc(const double *T_new, const double *T_old, int64_t n, double dt, double dT_max,
                        double eps, double *dt_next, int32_t *accept, double *max_change, hipStream_t stream);

/* Releases everything the handle owns.  NULL is accepted. */
int amg_destroy(amg_handle *h);

/* ---- thermal solve (Sec. 3, eq. wf_thermal; Sec. 3.2; Sec. 5.1-5.3) ------
 * The temperature of a step solves F_T(T; s) = 0 for all s in V_h:
 *   F_T = int rho c_v (T - T_old)/dt s + int kappa grad T . grad s
 *         + int_Gamma h (T - T_bc) s ds
 * (backward Euler, theta = 1, Sec. 5.3; without the first term for a steady
 * solve, Sec. 5.2), kappa and c_v temperature dependent (so F_T is
 * nonlinear), by Newton's method (Sec. 3.2) with each correction solved by
 * CG preconditioned with classical AMG and an l1 hybrid Gauss-Seidel
 * smoother (Sec. 5.1).  The paper's Robin coefficient beta is -h here, h >= 0
 * the heat-transfer coefficient, so the boundary term draws T toward T_bc.
 * Coefficients: each material gives kappa and c_v as piecewise-linear tables
 * in T (constant beyond the ends) and a density; a cell takes its material's
 * values at the exact mean of T_h over the cell, so every integral is exact
 * (P1 and P2).  The Newton Jacobian includes the derivatives of the tables
 * (the slope of the segment [T_k, T_k+1) holding the cell mean), so it is not
 * symmetric. */

/* Scalar compressed sparse rows. */
typedef struct {
    int64_t n_rows;
    int64_t nnz;
    int64_t *row_ptr;       /* device [n_rows+1]                              */
    int32_t *col_idx;       /* device [nnz], ascending within a row, diagonal
                               present                                        */
    double *val;            /* device [nnz]                                   */
} te_csr;

/* Host arrays, read during the call: T, kappa, cv [n_materials][n_points]
 * (T strictly ascending, kappa and cv > 0), rho [n_materials] (> 0). */
typedef struct {
    int32_t n_materials;
    int32_t n_points;
    const double *T;
    const double *kappa;    /* thermal conductivity                           */
    const double *cv;       /* specific heat                                  */
    const double *rho;      /* density                                        */
} te_thermal_tables;

/* Heat-transfer boundary: faces device [n_faces][3] (P1) or [n_faces][6] (P2:
 * vertices, then the edge nodes 01, 02, 12), h and T_bc device [n_faces]
 * (h >= 0).  n_faces = 0: insulated everywhere. */
typedef struct {
    int64_t n_faces;
    const int32_t *faces;
    const double *h;
    const double *T_bc;
} te_robin;

/* Residual F (device [N]) and Jacobian J = dF/dT of F_T at T (device [N]),
 * all integrals exact.  T_old (device [N]) with dt > 0: one backward-Euler
 * step from T_old; T_old = NULL: steady.  cell_material: device [C].
 * J: row_ptr from fe_assemble_pattern (the node coupling), col_idx and val
 * caller-allocated with J->nnz entries, overwritten.  Deterministic (rows
 * gathered over their cells and faces in ascending order).  Errors:
 * TE_EINVAL (bad mesh, tables or faces, a material id out of range),
 * TE_ENOMEM, TE_EHIP. */
int fe_assemble_thermal(const te_mesh *mesh, const te_thermal_tables *tab, const int32_t *cell_material,
                        const te_robin *robin, const double *T, const double *T_old, double dt, te_csr *J,
                        double *F, hipStream_t stream);

/* Classical AMG (the paper's thermal preconditioner is a classical AMG with a
 * hybrid Gauss-Seidel smoother, Sec. 5.1): per level
 *   strength: row i strongly depends on j != i when
 *             -a_ij >= theta max_k (-a_ik) > 0;
 *   splitting: PMIS with the fixed keys (|S_i^T|, splitmix64((0xC1A5 + level)
 *             ^ i) >> 24, i), C points numbered ascending;
 *   interpolation: direct (negative and positive couplings scaled apart);
 *   A_c = P^T A P; stop at <= coarse_max rows, max_levels, or a coarse level
 *   keeping more than max_coarse_ratio of the rows; the coarsest level is
 *   applied as its explicit inverse;
 *   smoother: l1 hybrid Gauss-Seidel over blocks of `block` consecutive rows
 *   (Gauss-Seidel inside a block, Jacobi across, diagonal a_ii + the
 *   absolute entries outside the block): one forward sweep before the coarse
 *   correction (from zero), one backward sweep after it. */
typedef struct {
    double theta;            /* (0.25)                                          */
    int32_t coarse_max;      /* (500)                                           */
    int32_t max_levels;      /* (10)                                            */
    double max_coarse_ratio; /* (0.9)                                           */
    int32_t block;           /* rows per Gauss-Seidel block, 1..256 (128)       */
} camg_options;
void camg_options_default(camg_options *opt);

typedef struct camg_handle camg_handle;

/* Builds the hierarchy of A (square, scalar); the values are copied (the
 * hierarchy keeps them).  Synchronises `stream`.  Errors: TE_EINVAL,
 * TE_ENOMEM, TE_EHIP, TE_ECHOL (singular coarsest level). */
int camg_setup(const te_csr *A, const camg_options *opt, camg_handle **out, hipStream_t stream);
int camg_destroy(camg_handle *h);

typedef struct {
    int32_t n_levels;
    int64_t n_rows[16];
    int64_t nnz[16];
    int64_t p_nnz[16];
    double setup_ms;
} camg_info;
int camg_get_info(const camg_handle *h, camg_info *info);
/* Host copy of level l's C/F splitting: state[i] = 2 (C) or 0 (F). */
int camg_get_splitting(const camg_handle *h, int32_t level, int8_t *state_host);
/* Host copy of A_l (which = 0), P_l (1) or R_l = P_l^T (2); NULL arrays
 * query the sizes through *n_rows_out / *nnz_out. */
int camg_get_level_matrix(const camg_handle *h, int32_t level, int32_t which, int64_t *n_rows_out,
                          int64_t *nnz_out, int64_t *row_ptr, int32_t *col, double *val);

/* Component access (device vectors, level numbering = natural):
 *   TE_CAMG_A          y = A_l x
 *   TE_CAMG_P          y = P_l x       (x on level l+1)
 *   TE_CAMG_R          y = P_l^T x     (y on level l+1)
 *   TE_CAMG_VCYCLE     y = V-cycle from level l applied to x
 *   TE_CAMG_SWEEP_FWD  y <- one forward hybrid Gauss-Seidel sweep for
 *                      A_l z = x from z = y (y in: start, out: result)
 *   TE_CAMG_SWEEP_BWD  the same, backward */
#define TE_CAMG_A          0
#define TE_CAMG_P          1
#define TE_CAMG_R          2
#define TE_CAMG_VCYCLE     3
#define TE_CAMG_SWEEP_FWD  4
#define TE_CAMG_SWEEP_BWD  5
int camg_apply(camg_handle *h, int32_t level, int32_t op, const double *x, double *y, hipStream_t stream);

/* Preconditioned CG (Sec. 2.1.2) on A (any matrix with the level-0 size,
 * e.g. a newer Jacobian than the one the hierarchy was built from) with the
 * V-cycle as preconditioner, from the guess in x, stopping as amg_pcg_solve
 * (true |b - A x| <= rtol |b|, at most 3 residual replacements).  iters,
 * relres: host, may be NULL.  Returns TE_OK, TE_ENOTCONV, TE_EINDEF, TE_ENAN,
 * TE_EINVAL, TE_EHIP. */
int camg_pcg_solve(camg_handle *h, const te_csr *A, const double *b, double *x, double rtol, int32_t maxit,
                   int32_t *iters, double *relres, hipStream_t stream);

/* Newton's method for F_T = 0 (Sec. 3.2): T <- T + d with J(T) d = -F(T),
 * stopping at |F(T)|_2 <= max(rtol |F(T_0)|_2, atol) (rtol 1e-9 and T_0 =
 * 400 K in the paper's steady runs, Sec. 5.2; the absolute floor atol, in
 * the units of F, ends a time step that starts near a steady state).  The classical-AMG preconditioner is built
 * from the Jacobian of the first Newton step and kept across Newton steps
 * and calls (time steps); it is rebuilt before the next correction when a
 * correction needed more than rebuild_factor times the CG iterations of the
 * first correction after the last build (the paper rebuilds the thermal
 * preconditioner at the steps with rapid temperature change, Sec. 5.3). */
typedef struct {
    double rtol;             /* Newton stop (1e-9)                              */
    double atol;             /* absolute floor of the Newton stop (1e-8)        */
    double lin_rtol;         /* CG stop for each correction (1e-8)              */
    int32_t maxit;           /* Newton steps (25)                               */
    int32_t lin_maxit;       /* CG iterations per correction (500)              */
    double rebuild_factor;   /* (1.5)                                           */
    camg_options amg;
} newton_options;
void newton_options_default(newton_options *opt);

typedef struct {
    int32_t iters;           /* Newton corrections                              */
    int32_t converged;
    int32_t rebuilds;        /* preconditioner builds in this call              */
    int32_t lin_iters_total;
    double res0, res;        /* |F(T_0)|_2, |F(T)|_2 at the end                 */
    double res_hist[33];     /* |F| before each correction and at the end       */
    int32_t lin_iters[32];   /* CG iterations of each correction                */
    double time_ms;          /* host wall time of the call                      */
    double assembly_ms, setup_ms, solve_ms;  /* device event time per phase     */
} newton_report;

typedef struct thermal_solver thermal_solver;

/* A thermal solver for one mesh: copies the mesh, the tables, the cell
 * materials and the heat-transfer faces (device arrays may be freed
 * afterwards).  Synchronises.  Errors: TE_EINVAL, TE_ENOMEM, TE_EHIP. */
int thermal_create(const te_mesh *mesh, const te_thermal_tables *tab, const int32_t *cell_material,
                   const te_robin *robin, thermal_solver **out, hipStream_t stream);
/* New exterior temperatures of the faces (device [n_faces], copied), for
 * time-dependent boundary data. */
int thermal_set_exterior(thermal_solver *s, const double *T_bc, hipStream_t stream);
/* Newton solve of one step: T device [N] (in: initial guess, out: solution);
 * T_old device [N] with dt > 0 (backward Euler) or NULL (steady).  rep: host,
 * may be NULL.  Synchronises.  Returns TE_OK, TE_ENOTCONV (Newton or a CG
 * solve hit its limit; T holds the last iterate), TE_EINDEF, TE_ENAN,
 * TE_EINVAL, TE_EHIP, TE_ECHOL. */
int thermal_newton(thermal_solver *s, double *T, const double *T_old, double dt, const newton_options *opt,
                   newton_report *rep, hipStream_t stream);
/* Drops the kept preconditioner (the next correction builds a new one). */
int thermal_reset_preconditioner(thermal_solver *s);
int thermal_destroy(thermal_solver *s);

/* ---- learned initial guess (message-passing network, float32) ---------
 * The paper starts each transient elastic solve from the previous step's
 * displacement (Sec. 5.3).  This network maps the load instead:
 *   h0 = relu(X W_in + b_in);  4 layers of
 *   h  = h + relu(h W_s + mean_{N(v)} h W_n + mean_V h W_g
 *                 + sum_k (sum_{u in N(v)} w^k_vu h_u) W_dk + b),  k = x, y, z,
 *        w^k_vu = (x_u - x_v)_k / (deg_v l_v), l_v the mean edge length at v;
 *   y  = (h W_out + b_out) * (1 - mask),  u0 = 1e-3 * y.
 * Features X[v] = [(T-T_ref)/500, f/2e9 (3), mask (3), (x - centroid)/0.5 (3)].
 * Parameters: one float array of mpnn_param_count() entries in the order
 * W_in[10][64], b_in[64], per layer {W_s,W_n,W_g,W_dx,W_dy,W_dz}[64][64],
 * b[64], W_out[64][3], b_out[3] (weights [in][out]). */
typedef struct mpnn_handle mpnn_handle;

int64_t mpnn_param_count(void);

/* Graph and workspace for a mesh of N vertices.  row_ptr/col_idx: the P1
 * stiffness pattern (device, as produced by fe_assemble_pattern); its
 * diagonal is dropped.  coords: device [N][3].  Synchronises `stream`. */
int mpnn_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *coords,
                mpnn_handle **out, hipStream_t stream);
int mpnn_destroy(mpnn_handle *h);

/* X [N][10] float from T [N], f [N][3] or NULL, mask [N][3] (device). */
int mpnn_features(mpnn_handle *h, const double *T, double T_ref, const double *f, const uint8_t *mask,
                  float *X, hipStream_t stream);

/* y [N][3] = network output (may be NULL: kept inside the handle); the
 * activations are kept for mpnn_backward. */
int mpnn_forward(mpnn_handle *h, const float *params, const float *X, const uint8_t *mask, float *y,
                 hipStream_t stream);

/* Mean squared error of the last forward against target [N][3] (the
 * displacement divided by 1e-3) into *loss (host, may be NULL) and its
 * gradient with respect to every parameter into grad.  Synchronises. */
int mpnn_backward(mpnn_handle *h, const float *params, const float *target, float *grad, double *loss,
                  hipStream_t stream);

/* Gradients of any loss of the last forward given dL/dy (device float
 * [N][3]; entries of constrained DOFs are ignored) into grad. */
int mpnn_backward_from(mpnn_handle *h, const float *params, const float *gy, float *grad, hipStream_t stream);

/* Energy-norm loss of the last forward's guess taken at its energy-optimal
 * multiple (the guess the solve uses, amg_energy_scale):
 * loss = 1 - (u, A t)^2 / ((u, A u)(t, A t)) = ||g u - t||_A^2 / ||t||_A^2 at
 * the best g, with u = 1e-3 y (constrained DOFs zero), t = 1e-3 target and A
 * the level-0 operator of `amg` (same mesh); gy [N][3] = dloss/dy (device
 * float); a zero guess gives loss 1 and gy 0.  *loss host, may be NULL.  Uses
 * amg's solve workspace; synchronises. */
int mpnn_energy_grad(mpnn_handle *h, amg_handle *amg, const float *target, float *gy, double *loss,
                     hipStream_t stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on n entries. */
int mpnn_adam_step(int64_t n, float *params, const float *grad, float *m, float *v, int32_t step, float lr,
                   float beta1, float beta2, float eps, hipStream_t stream);

/* u0 [N][3] float64 = 1e-3 * y of the last forward. */
int mpnn_guess(mpnn_handle *h, double *u0, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* TE_H */
