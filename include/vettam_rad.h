/*
 * vettam_rad.h -- C ABI of the MI355X implicit VET radiation step library.
 *
 * The library advances the gray two-moment radiation equations (E, F) and the
 * gas temperature T by one fully implicit backward-Euler step, as the
 * implicit subsystem of Menon et al. 2022 (VETTAM), Sec. 2.3.2 eq.
 * implicit1-3 with the gas velocity set to zero:
 *
 *   (1 + sP) E - E_n - sP aR T^4 + (dt/h) sum_d (PhiE_{i+1/2} - PhiE_{i-1/2}) = 0
 *   (1 + sR) F - F_n             + (dt/h) sum_d (PhiF_{i+1/2} - PhiF_{i-1/2}) = 0
 *   alpha (T - T_n) + sP (aR T^4 - E)                                       = 0
 *
 * sP = c dt rho kappa_P, sR = c dt rho kappa_R, alpha = rho c_v.  The face
 * fluxes are first-order Godunov HLLE fluxes (Sec. 2.3.3) closed by the
 * per-cell variable Eddington tensor f_ij (eq. closure), with the
 * optical-depth wave-speed correction of eq. taucorrect and the same-level
 * interface rule of eq. wavespeedtau:
 *   PhiE   = (F_d,L + F_d,R)/2 - C (E_R - E_L)/2
 *   PhiF_j = c^2 (f_dj,L E_L + f_dj,R E_R)/2 - C (F_j,R - F_j,L)/2
 *   C = c sqrt(max(f_dd,L, f_dd,R)) sqrt((1 - exp(-tau))/tau),
 *   tau = (tau_L + tau_R)/2,  tau_cell = (10 h rho kappa_R)^2 / (2 f_dd).
 * The nonlinear system is solved by the Picard iteration of Sec. 2.3.4
 * (radiation solve at a guessed temperature, then a per-cell Newton solve of
 * eq. PicardTemp), with GMRES as the Krylov solver.
 *
 * Layout: structure of arrays, x fastest, index = i + nx*(j + ny*k).
 *   E, T_gas, rho, kappa_P, kappa_R: one plane of nx*ny*nz values each.
 *   F: three planes [Fx | Fy | Fz].   f_ij: six planes [xx|yy|zz|xy|xz|yz].
 * All data pointers are DEVICE pointers owned by the caller.  E, F, T_gas are
 * FP64 and are overwritten with the new state; rho, kappa_P, kappa_R and f_ij
 * have the element type params->coef_dtype (FP64 or FP32) and are read only.
 *
 * Errors are returned, never thrown.  Host-side argument checks happen before
 * any device work (RAD_EINVAL); rad_last_error() gives a thread-local message.
 * A step that does not reach params->tol returns RAD_NOT_CONVERGED and leaves
 * the last iterate in E, F, T_gas.  Invalid data found on the device
 * (negative or non-finite rho, kappa, f_dd) returns RAD_EDATA before the state
 * is touched.  `stream` is a hipStream_t; NULL means the default stream.
 */
#ifndef VETTAM_RAD_H
#define VETTAM_RAD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RAD_OK = 0,
    RAD_NOT_CONVERGED = 1,
    RAD_EINVAL = -1,   /* bad argument (checked on the host before any launch) */
    RAD_ENOMEM = -2,   /* workspace smaller than rad_workspace_bytes() */
    RAD_EHIP = -3,     /* a HIP runtime call failed */
    RAD_ENOTIMPL = -4,
    RAD_EDATA = -5     /* invalid coefficient data found on the device */
} rad_status;

/* Face kinds (see rad_step for what each does at a wall). */
typedef enum {
    RAD_BC_PERIODIC = 0,
    RAD_BC_OUTFLOW = 1,    /* zero-gradient outflow (Sec. 3.3): the ghost is the boundary cell */
    RAD_BC_DIRICHLET = 2,  /* fixed ghost data: params->ghost on the single grid, the blocks' ghost layers */
    RAD_BC_OPEN = 3,       /* characteristic outflow: incoming characteristic held at its old value */
    RAD_BC_MARSHAK = 4,    /* c E + 2 F_in = 4 F_inc at the wall (Sec. 3.4), F_inc in params->F_inc */
    RAD_BC_REFLECT = 5     /* mirror */
} rad_bc_kind;
typedef enum { RAD_FP64 = 0, RAD_MIXED = 1 } rad_precision;
typedef enum { RAD_PICARD_LAGGED = 0, RAD_PICARD_LINEARISED = 1 } rad_picard_mode;
typedef enum { RAD_F64 = 0, RAD_F32 = 1 } rad_dtype;

typedef struct {
    double c, a_R, c_v;   /* speed of light, radiation constant, gas heat capacity per mass */
    double tol;           /* target of the scaled nonlinear residual (see rad_stats_t) */
    double eps_R;         /* relative tolerance of each linear (Krylov) solve; the last solves of a
                             step are tightened to 0.1 tol / (current scaled residual) */
    double eps_P;         /* > 0: also stop when the relative change of [E,F,T] < eps_P (Sec. 2.3.4) */
    int max_picard;       /* Picard iterations per step */
    int max_krylov;       /* Krylov iterations per linear solve */
    int gmres_m;          /* GMRES restart length, 1..64 */
    int prec;             /* rad_precision: FP64, or FP32 Krylov with FP64 residual/refinement */
    int mode;             /* rad_picard_mode: paper's lagged emission, or emission linearised at T_* */
    int coef_dtype;       /* rad_dtype of rho, kappa_P, kappa_R, f_ij */
    int anderson_m;       /* 0: plain Picard; 1..5: Anderson acceleration of the Picard map
                             T_* -> T(E(T_*)) with this many past iterates (the acceleration the
                             paper names for its linearly convergent Picard iteration, Sec. 4.3).
                             Single-grid rad_step only; the batched plan requires 0. */
    int vel_implicit;     /* rad_step_moving only: 1 moves the O(v/c) part of the gas-radiation
                             energy exchange into the implicit gas energy row (the paper's runtime
                             switch, Sec. 2.3.2); 0 (default) leaves it to the explicit hydro update */
    int cv_cubic;         /* 0 (default): gas internal energy rho c_v T; 1: heat capacity rho c_v T^3,
                             internal energy rho c_v T^4 / 4 (the gas of the Marshak-wave test, Sec. 3.4).
                             rad_step, rad_step_moving, rad_residual and rad_exchange; the batched and
                             two-level paths require 0 */
    int krylov_poly;      /* Krylov operator, always right-multiplied onto the Jacobi-scaled operator B
                             so that GMRES minimises the residual of B itself:
                             1 (default): the first-order Neumann polynomial 2I - B (Arnoldi on
                             2B - B^2, two applies of B per iteration); every stepping entry point,
                             the batched plan included;
                             0: Jacobi scaling alone;
                             2: one multigrid V-cycle (levels halve the grid while every extent is
                             even and >= 8, at most 6 levels; coarse operators re-discretised on the
                             children's mean sR, tensor and E diagonal; one damped Jacobi sweep,
                             weight 0.4, before and after each coarse correction, two on the
                             coarsest level).  A GMRES cycle that gains less than 10% under the V-cycle
                             switches the rest of the step to the Neumann operator.  rad_step only,
                             on grids whose extents halve at least once (RAD_EINVAL otherwise); its
                             levels enlarge the workspace */
    double F_inc[6];      /* incident flux of each RAD_BC_MARSHAK face (-x,+x,-y,+y,-z,+z); ignored elsewhere */
    double eps_N;         /* relative tolerance of the per-cell Newton solve of eq. PicardTemp (Sec. 2.3.4);
                             0 (default): iterate to round-off */
    int energy_fix;       /* 0 (default): commit T as the last Newton root.  1: commit the gas energy
                             e(T_N) + dt dE of the energy correction of Sec. 2.3.4 (see rad_stats_t), so the
                             exchange terms of the radiation and gas equations cancel and the step conserves
                             energy for any eps_P.  rad_step only, with anderson_m = 0 */
    int max_refine;       /* most FP64 residual evaluations (GMRES restarts) per linear solve; 0: no limit
                             beyond max_krylov */
    const double *ghost[6]; /* each RAD_BC_DIRICHLET face (-x,+x,-y,+y,-z,+z) of a single grid: device
                             pointer (caller-owned, read only, FP64) to the ghost cells' fixed state, four
                             planes (E, F_x, F_y, F_z; F physical) over the face's cells in the order
                             x faces [nz][ny], y faces [nz][nx], z faces [ny][nx] (last index fastest);
                             one ghost layer, the one the first-order stencil reads.  NULL (default) for
                             other faces.  rad_step, rad_step_noalloc, rad_step_moving, rad_autotune_step
                             and rad_residual need it for every Dirichlet face (RAD_EINVAL otherwise);
                             rad_apply and rad_face_speeds never read it */
} rad_params_t;

typedef struct {
    int status;            /* rad_status of the step (per block in the batched call) */
    int picard_iters;
    int krylov_iters;      /* Krylov (Arnoldi) iterations summed over Picard iterations; with
                              krylov_poly = 1 each applies the scaled operator twice */
    int refine_sweeps;     /* FP64 residual evaluations (GMRES restarts) */
    int neg_cells;         /* cells whose exchange solve had no positive root (T set to 0) */
    int bad_cells;         /* cells with invalid coefficient data */
    double scaled_residual;/* max of the three parts below */
    double res_E;          /* || R_E / W_E || / ||E||,  W_E = 1 + sP + (dt/2h) sum_faces C */
    double res_F;          /* || R_F / W_F || / (||F|| + c ||E||),  W_F = 1 + sR + (dt/2h) sum C */
    double res_T;          /* || R_T / W_T || / ||T||,  W_T = alpha + 4 sP aR T^3 */
    double rel_change;     /* relative change of [E, F, T] over the last Picard iteration */
    double t_total_ms;     /* wall time of the call (host clock) */
    /* Energy correction of Sec. 2.3.4 in the last Picard iteration: the radiation solve took the
     * emission e_rad at the guess T_o (aR T_o^4 lagged, its linearisation about T_o linearised),
     * the gas solve at its root T_N, so per cell the exchange terms differ by
     * dt dE = sP (aR T_N^4 - e_rad).  Zero at the solution.  Single-grid steps only (0 elsewhere). */
    double energy_defect;  /* sum dt dE / sum (E_n + e(T_n)): the relative energy the mismatch creates */
    double dE_max;         /* max over cells of |dt dE| / (|E| + e(T_N)) */
    double bytes_moved;    /* algorithmic HBM bytes of the step's kernels (inputs and outputs once each) */
} rad_stats_t;

/* Fill *p with defaults: c = aR = cv = 1, tol 1e-10, eps_R 1e-2, eps_P 0,
 * max_picard 50, max_krylov 20000, gmres_m 12, FP64, linearised, FP64 coefficients,
 * anderson_m 0, vel_implicit 0, cv_cubic 0, krylov_poly 1, F_inc 0, eps_N 0,
 * energy_fix 0, max_refine 0. */
void rad_default_params(rad_params_t *p);

/* Device workspace (bytes) rad_step needs for an nx*ny*nz grid. */
size_t rad_workspace_bytes(int nx, int ny, int nz, const rad_params_t *p);

/* One implicit radiation step on a uniform grid (Sec. 2.3.1 steps iv-vi).
 * bc[6]: faces -x,+x,-y,+y,-z,+z, each RAD_BC_PERIODIC (in pairs) or one of
 * the walls, whose ghost cell (coefficients: the boundary cell's) holds
 *   RAD_BC_DIRICHLET the fixed state params->ghost[face] (the ghost data with which
 *                   the HLLE flux of Sec. 2.3.3 is taken across the face; the data
 *                   enter the right-hand side only);
 *   RAD_BC_OUTFLOW  the boundary cell's state (zero gradient, Sec. 3.3): uniform states
 *                   stay uniform, but where the corrected speed is below c sqrt(f_dd)
 *                   (optically thick boundary cells) the wall's block is indefinite, so
 *                   at tens of light-crossing times the step may not be well posed;
 *   RAD_BC_OPEN     the boundary cell's state with the amplitude of the incoming
 *                   characteristic of the normal flux, (E +- F_d / (c sqrt(f_dd))) / 2, held
 *                   at its value at the start of the step: well posed at any dt;
 *                   stationary states at the wall are kept, a streaming pulse leaves
 *                   without reflection;
 *   RAD_BC_MARSHAK  F = F_cell, E = 8 F_inc / c -+ 4 F_d,cell / c - E_cell, so that the
 *                   means of ghost and cell satisfy c E + 2 F_in = 4 F_inc (Sec. 3.4);
 *   RAD_BC_REFLECT  the mirror image (F_d and the tensor's f_dj, j != d, negated).
 * dt > 0, dx > 0.
 * workspace: device memory of at least rad_workspace_bytes(), 256-byte aligned.
 * stats: host pointer, may be NULL.  The call returns after the step completed. */
int rad_step(int nx, int ny, int nz, double *E, double *F, double *T_gas,
             const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
             double dt, double dx, const int bc[6], const rad_params_t *p,
             void *workspace, size_t ws_bytes, void *stream, rad_stats_t *stats);

/* ----------------------------------------------- allocation-free variant
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  rad_step
 * with the workspace taken from a static device array inside the library
 * (one copy per GPU, held until the process ends; rad_noalloc_max_bytes()
 * bytes, 64 MiB) instead of a caller buffer, and the reductions read back
 * through a thread-local pageable host buffer: the call makes no device or
 * pinned-host allocation.  Arguments, results and errors as rad_step; a step
 * whose rad_workspace_bytes() exceeds the array returns RAD_ENOMEM before any
 * device work.  Every call on one GPU uses that GPU's array: calls that
 * overlap on one GPU (other threads, other streams) race.  Profiling
 * (rad_profile_enable) must be off, since it creates HIP events. */
size_t rad_noalloc_max_bytes(void);
int rad_step_noalloc(int nx, int ny, int nz, double *E, double *F, double *T_gas,
                     const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
                     double dt, double dx, const int bc[6], const rad_params_t *p, void *stream,
                     rad_stats_t *stats);

/* ------------------------------------------------------- moving medium
 * rad_step with a gas velocity: the O(v/c) terms of the radiation four-force
 * (eq. G and G0, with kappa_E = kappa_P and kappa_F = kappa_R) enter the
 * implicit radiation rows -- with beta = v/c, sP = c dt rho kappa_P and
 * sR = c dt rho kappa_R, dt times
 *   energy row:  (sR - 2 sP) beta.F / c + (sP - sR) (beta.beta + beta.f.beta) E
 *   flux row:    -sR c E (beta + f beta)
 * -- and, with params->vel_implicit = 1, the first of them also into the gas
 * energy row (eq. G0explicit moved to the implicit subsystem).  beta: three
 * planes [bx|by|bz] of coef_dtype, device memory, the velocity held fixed
 * over the step (Sec. 2.3.2).  Other arguments as rad_step.  Errors as
 * rad_step; anderson_m must be 0 with vel_implicit = 1. */
size_t rad_workspace_bytes_moving(int nx, int ny, int nz, const rad_params_t *p);
int rad_step_moving(int nx, int ny, int nz, double *E, double *F, double *T_gas,
                    const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
                    const void *beta, double dt, double dx, const int bc[6], const rad_params_t *p,
                    void *workspace, size_t ws_bytes, void *stream, rad_stats_t *stats);

/* ---------------------------------------------------- two-level AMR grid
 * A coarse grid (nx, ny, nz) of cell width dx with one box [lo, hi) of its
 * cells (per axis x, y, z) refined by a factor 2 (Sec. 2.3.3, eq. wavespeedtau
 * and eq. interface_flux; App. A2).  Along each axis the box either spans the
 * whole extent (lo = 0, hi = n: no level jump there, the fine level takes the
 * domain's boundary condition) or stays at least one coarse cell inside it
 * (1 <= lo < hi <= n - 1).  The fine level has extents 2 (hi - lo).
 *
 * Every per-cell array holds the coarse level's cells, all nx ny nz of them
 * (covered ones included), followed by the fine level's: each level is a
 * complete single-grid array set of its own extents (x fastest), so F is
 * [Fx|Fy|Fz of the coarse level | Fx|Fy|Fz of the fine level] and f_ij the
 * six coarse planes followed by the six fine ones.
 *
 * The step solves the composite backward-Euler system: at a face where the
 * level changes the HLLE speeds take the upstream cell's optical depth (each
 * cell's with its own width), the fine cells' neighbour is the coarse cell,
 * and the coarse cell receives the mean of the four fine face fluxes, so E and
 * F are conserved by construction.  Covered coarse cells are no part of the
 * transport; on return they hold the mean of their eight children (E, F and
 * T).  Boundaries of the domain: periodic (in pairs) or outflow. */
typedef struct {
    int nx, ny, nz;     /* coarse extents */
    int lo[3], hi[3];   /* refined box in coarse cells, [lo, hi) per axis x, y, z */
} rad_amr2_t;

/* Workspace bytes of rad_step_amr2 (0 if the geometry or params are invalid). */
size_t rad_workspace_bytes_amr2(const rad_amr2_t *geom, const rad_params_t *p);

/* One implicit step on the two-level grid; arguments as rad_step, with the
 * geometry in geom, dx the coarse cell width and the arrays in the two-level
 * layout above (device pointers owned by the caller; E, F, T_gas updated in
 * place).  Errors: RAD_EINVAL for an invalid geometry (a box that neither
 * spans an axis nor stays inside it, more than 2^31 cells in all), the
 * conditions of rad_step otherwise.  The autotune cache is not consulted. */
int rad_step_amr2(const rad_amr2_t *geom, double *E, double *F, double *T_gas,
                  const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
                  double dt, double dx, const int bc[6], const rad_params_t *p,
                  void *workspace, size_t ws_bytes, void *stream, rad_stats_t *stats);

/* Autotune rad_step for this grid, boundary set, precision and coefficient
 * type on the caller's data (same arguments as rad_step; the state E, F, T_gas
 * is left as it was on entry).  Times the stencil's z-range per workgroup
 * (8..128 planes) separately for the Krylov apply and the FP64 residual, for
 * the apply also whether it reads the stored corrected face speeds or forms
 * them per face from f and sR, and, if tune_restart != 0, one full step for
 * each GMRES restart length in {6, 8, 10, 12, 16, 24, 32, 48, 64} up to
 * params->gmres_m (the workspace's size), with and without the Neumann
 * polynomial (krylov_poly 1 and 0) and, when params->krylov_poly = 2 (the
 * workspace then holds the multigrid levels), with the V-cycle too.  The choices are stored in the autotune
 * cache ($VETTAM_RAD_CACHE_DIR or ~/.cache/vettam_rad, one "key TAB kz_apply
 * kz_residual gmres_m load_speeds krylov_poly" line each) and the tiles and
 * face-speed variant are used by every later rad_step call with the same key;
 * the fastest converged restart length and Krylov operator are returned in
 * *gmres_m and *krylov_poly as recommendations (rad_step keeps the caller's).
 * Outputs may be NULL.  Synchronous. */
int rad_autotune_step(int nx, int ny, int nz, double *E, double *F, double *T_gas,
                      const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
                      double dt, double dx, const int bc[6], const rad_params_t *p,
                      void *workspace, size_t ws_bytes, void *stream, int tune_restart,
                      int *kz_apply, int *kz_residual, int *gmres_m, int *krylov_poly);

/* Nonlinear residual of the backward-Euler system at a state (E, F, T) given
 * the old state (E_n, F_n, T_n): R holds 5 planes [R_E | R_Fx | R_Fy | R_Fz | R_T]
 * (FP64, device).  Faces as in rad_step, Dirichlet faces with their data from
 * params->ghost.  Stream-ordered, asynchronous. */
int rad_residual(int nx, int ny, int nz, const double *E_n, const double *F_n, const double *T_n,
                 const double *E, const double *F, const double *T,
                 const void *rho, const void *kappa_P, const void *kappa_R, const void *f_ij,
                 double dt, double dx, const int bc[6], const rad_params_t *p, double *R, void *stream);

/* Corrected HLLE wave speed of every low face (Sec. 2.3.3): Cd[i] is the speed
 * of the face between cell i - e_d and cell i (three FP64 planes Cx|Cy|Cz);
 * the neighbour across a domain face follows bc (periodic: the opposite cell;
 * every other kind: the cell itself, whose coefficients a wall's or Dirichlet
 * ghost takes).  Stream-ordered, asynchronous. */
int rad_face_speeds(int nx, int ny, int nz, const void *rho, const void *kappa_R, const void *f_ij,
                    double dx, const int bc[6], const rad_params_t *p, double *C, void *stream);

/* Linear transport operator of one Picard iteration applied to x = (E, Fx, Fy, Fz):
 *   y_E = dE * E + (dt/h) div PhiE,  y_Fj = (1 + sR) F_j + (dt/h) div PhiF_j.
 * x, y: four planes; dE: one plane.  dtype RAD_F64 or RAD_F32 selects the
 * element type of x, y, dE and the arithmetic.  Faces as in rad_step with
 * their data dropped (a Dirichlet ghost is zero; params->ghost is not read).
 * Stream-ordered, asynchronous. */
int rad_apply(int nx, int ny, int nz, const void *x, void *y, const void *dE,
              const void *rho, const void *kappa_R, const void *f_ij,
              double dt, double dx, const int bc[6], const rad_params_t *p, int dtype, void *stream);

/* Per-cell gas temperature update of eq. PicardTemp: T >= 0 solving
 * alpha (T - T_n) + sP (aR T^4 - E) = 0 by Newton's method (FP64).
 * n cells; all arrays device.  Stream-ordered, asynchronous. */
int rad_exchange(long long n, const double *E, const double *T_n, double *T,
                 const void *rho, const void *kappa_P, double dt, const rad_params_t *p, void *stream);

/* ---------------------------------------------------------------- closures
 * Local closures of Sec. 4.1 (the comparison of closures), evaluated from the
 * time-lagged state to give f_ij for the next step:
 *   RAD_CLOSURE_EDDINGTON: f = I/3 (the Eddington approximation);
 *   RAD_CLOSURE_M1: f = (1 - chi)/2 I + (3 chi - 1)/2 n n, n = F/|F|,
 *     chi = (3 + 4 g^2) / (5 + 2 sqrt(4 - 3 g^2)), g = |F| / (c E),
 *     with g clipped to [0, 1]; where E <= 0, g = 1 if F != 0 and 0 if F = 0.
 * E (ncells) and F (three planes Fx|Fy|Fz of ncells) are FP64 device arrays;
 * f_ij (six planes xx|yy|zz|xy|xz|yz of ncells, caller-owned) is written in
 * out_dtype (RAD_F64 or RAD_F32).  FP64 arithmetic; one streaming pass,
 * asynchronous on `stream`.  ncells = 0 is a no-op. */
typedef enum { RAD_CLOSURE_EDDINGTON = 0, RAD_CLOSURE_M1 = 1 } rad_closure_kind;

int rad_closure(long long ncells, const double *E, const double *F, int kind, double c, void *f_ij,
                int out_dtype, void *stream);

/* ---------------------------------------------------------------- batched
 * Many independent blocks, each an n^3 interior with ng ghost layers of fixed
 * Dirichlet data (E, F and its own rho, kappa, f), solved in one persistent
 * launch replayed from a HIP graph.  Every packed arena (E, T, rho, kappa_P,
 * kappa_R: one arena each; F: 3 consecutive arenas Fx|Fy|Fz; f_ij: 6) holds
 * block b's (n+2ng)^3 region, x fastest, at element offset off[b]; each arena
 * has total_cells elements (the largest off + (n+2ng)^3).  Only the first
 * ghost layer enters the first-order stencil. */
typedef struct {
    int n;           /* interior edge length (cells), 1..64 */
    int ng;          /* ghost layers (>= 1) */
    double dx, dt;
    long long off;   /* element offset of the block in every arena */
} rad_block_desc_t;

typedef struct rad_plan_s *rad_plan;

/* Device workspace (bytes) for a batch. */
size_t rad_batched_workspace_bytes(int nblocks, const rad_block_desc_t *desc, const rad_params_t *p);

/* Build a plan: validate the descriptors, order blocks (largest first),
 * upload the descriptor table into the workspace and build the HIP graph of
 * the persistent launch.  The launch shape comes from the autotune cache
 * ($VETTAM_RAD_CACHE_DIR or ~/.cache/vettam_rad) when it holds this batch
 * signature, else 512-thread workgroups, one per CU.  The workspace must stay
 * valid for the plan's lifetime. */
int rad_plan_batched(int nblocks, const rad_block_desc_t *desc, const rad_params_t *p,
                     void *workspace, size_t ws_bytes, void *stream, rad_plan *out);

/* Time the candidate launch shapes on the given data (state restored after
 * each trial from a copy kept in scratch, which needs
 * rad_autotune_scratch_bytes()) and keep the fastest in the plan. */
size_t rad_autotune_scratch_bytes(rad_plan plan);
int rad_autotune_batched(rad_plan plan, double *E, double *F, double *T_gas, const void *rho,
                         const void *kappa_P, const void *kappa_R, const void *f_ij,
                         void *scratch, size_t scratch_bytes, void *stream);

/* One step of every block: a single graph launch, asynchronous on `stream`.
 * dev_stats: device array of nblocks rad_stats_t (per-block status etc.;
 * t_total_ms is the block's solve time on the device wall clock). */
int rad_step_batched(rad_plan plan, double *E, double *F, double *T_gas, const void *rho,
                     const void *kappa_P, const void *kappa_R, const void *f_ij,
                     rad_stats_t *dev_stats, void *stream);

/* The plan's launch shape: threads per workgroup, workgroups per CU and
 * whether blocks are queued largest first (any output may be NULL). */
int rad_plan_launch_shape(rad_plan plan, int *threads, int *per_cu, int *largest_first);

/* Queue the plan's blocks by the solve times of an earlier step, longest
 * first (longest-processing-time order on measured cost: a block's difficulty
 * -- its optical depth per cell and crossings per step -- persists between
 * steps, while the default order only knows its size).  dev_stats: the device
 * stats array that step filled, whose t_total_ms holds each block's solve
 * time on the device wall clock.  Synchronises `stream` (one small copy to
 * the host), then uploads the new order; the results of later steps do not
 * depend on the order.  The order holds until the next rad_plan_reorder or
 * rad_autotune_batched.  RAD_ENOTIMPL if the device has no wall-clock rate. */
int rad_plan_reorder(rad_plan plan, const rad_stats_t *dev_stats, void *stream);

void rad_plan_destroy(rad_plan plan);

/* ------------------------------------------------------------- profiling
 * Per-kernel-class timing with HIP events recorded around every launch on
 * the launch stream, plus the algorithmic bytes each launch moves (the
 * minimum HBM traffic of its inputs and outputs).  Off by default; costs
 * two event records per launch when on.  Not thread-safe.
 * on: 0 off; 1 every class timed; 2 only the operator-apply classes
 * (apply_fp32, apply_fp64) timed, the others counted (bytes and launches,
 * zero milliseconds) with no event on the stream, so that the step runs at
 * close to its unprofiled speed.  Any other nonzero value acts as 1. */
void rad_profile_enable(int on);
void rad_profile_reset(void);
/* Number of kernel classes with at least one timed launch. */
int rad_profile_count(void);
/* Class idx: name (static string), summed milliseconds, summed algorithmic
 * bytes and launch count.  Returns RAD_EINVAL for a bad index. */
int rad_profile_get(int idx, const char **name, double *ms, double *bytes, long long *launches);

/* Message of the last non-OK return on this thread ("" if none). */
const char *rad_last_error(void);

/* Build id: a hash of the sources the library was built from (also part of
 * every autotune cache key, so tuned entries of one build do not steer another). */
const char *rad_build_id(void);

#ifdef __cplusplus
}
#endif
#endif
