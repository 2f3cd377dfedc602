/*
 * oracle.h -- plain FP64 CPU oracle for the implicit VET radiation step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this code.  It shares no code, header, table or
 * helper with the GPU library; the two are written independently from the
 * paper (Menon et al. 2022, "VETTAM", Sec. 2.2-2.3).
 *
 * The oracle computes the solution of the coupled, nonlinear backward-Euler
 * system of the implicit radiation subsystem (Sec. 2.3.2 "Operator splitting",
 * eq. implicit1-3, with v = 0) discretised by the first-order Godunov/HLLE
 * scheme of Sec. 2.3.3 and the gas-energy exchange eq. PicardTemp:
 *
 *   R_E  = (1+sP) E - E_n - sP aR T^4 + (dt/h) sum_d (PhiE_{+d} - PhiE_{-d}) = 0
 *   R_Fj = (1+sR) F_j - F_n,j         + (dt/h) sum_d (PhiF_{+d} - PhiF_{-d}) = 0
 *   R_T  = alpha (T - T_n) + sP (aR T^4 - E)                                  = 0
 *
 * with sP = c dt rho kappa_P, sR = c dt rho kappa_R, alpha = rho c_v, and the
 * face fluxes PhiE = (F_L + F_R)/2 - C (E_R - E_L)/2,
 *              PhiF_j = c^2 (f_dj,L E_L + f_dj,R E_R)/2 - C (F_j,R - F_j,L)/2,
 * C being the corrected HLLE wave speed of eq. taucorrect / wavespeedtau.
 *
 * It reaches that solution the way the paper does: a Picard iteration (steps
 * iv-vi of Sec. 2.3.1) alternating a Krylov (GMRES) solve of the radiation
 * moment equations at a guessed temperature with a per-cell Newton solve of
 * the gas temperature.
 *
 * Arrays are "padded": one ghost layer on every side, x fastest,
 *   index(i,j,k) = (i+1) + (nx+2) * ((j+1) + (ny+2) * (k+1)),  i in [-1, nx].
 * Ghost values of periodic / outflow faces are filled by the oracle; ghost
 * values of Dirichlet faces are data supplied by the caller.
 */
#ifndef VETTAM_ORACLE_H
#define VETTAM_ORACLE_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Face boundary kinds (see or_fill_state_ghosts for what each puts in the ghost cell). */
enum { OR_PERIODIC = 0, OR_OUTFLOW = 1, OR_DIRICHLET = 2, OR_OPEN = 3, OR_MARSHAK = 4, OR_REFLECT = 5 };
enum { OR_LAGGED = 0, OR_LINEARISED = 1 };

typedef struct {
    int nx, ny, nz;
    double h;      /* cell width (cubic cells) */
    double dt;     /* time step */
    double c;      /* speed of light */
    double aR;     /* radiation constant */
    double cv;     /* gas heat capacity per unit mass: alpha = rho * cv */
    int bc[6];     /* faces -x,+x,-y,+y,-z,+z */
    int cv_cubic;  /* 0: E_int = alpha T; 1: C_v = alpha T^3, E_int = alpha T^4 / 4 (the Marshak-wave gas) */
    double finc[6];/* OR_MARSHAK faces: the incident flux F_inc (Sec. 3.4) */
} or_grid;

/* Padded input fields (see header comment). f holds xx,yy,zz,xy,xz,yz.
 * beta: the gas velocity over c, three padded planes, or NULL (v = 0).  With a
 * velocity the O(v/c) terms of G0 and G (eq. G, kappa_E = kappa_P and
 * kappa_F = kappa_R) enter the radiation rows; vel_implicit = 1 also moves the
 * O(v/c) part of cG0 into the gas energy row (the implicit alternative of
 * eq. G0explicit), 0 leaves it to the explicit hydro update (the default). */
typedef struct {
    const double *rho, *kP, *kR;
    const double *f[6];
    const double *beta[3];
    int vel_implicit;
} or_coef;

typedef struct {
    double tol;        /* target scaled nonlinear residual */
    double lin_rtol;   /* cap on the relative tolerance of each Krylov solve */
    int max_picard;
    int gmres_m;
    int max_krylov;    /* per linear solve */
    int mode;          /* OR_LAGGED (paper) or OR_LINEARISED */
    double eps_P;      /* if > 0: also stop when the relative change of x_P < eps_P */
    double eps_N;      /* relative tolerance of the per-cell Newton solve (0: iterate to round-off) */
    int energy_fix;    /* 1: commit the gas temperature with the energy correction of Sec. 2.3.4 (see
                          or_rad_step); 0: commit the last Newton root */
} or_params;

typedef struct {
    int picard_iters;
    int krylov_iters;
    int converged;     /* 1: tol met, 2: stagnated at the FP64 floor, 0: no */
    int neg_cells;     /* cells whose exchange right-hand side was <= 0 */
    double scaled_residual;
    double res_E, res_F, res_T;
    double rel_change;
    /* energy correction of Sec. 2.3.4 in the last Picard iteration, per cell
     * dt dE = sP (aR T_N^4 - e_rad): T_N the Newton root, e_rad the emission the radiation
     * solve used (aR T_o^4 in the lagged mode, its linearisation about T_o otherwise) */
    double energy_defect;  /* sum dt dE / sum (E_n + e(T_n)) */
    double dE_max;         /* max over cells of |dt dE| / (|E| + e(T_N)) */
} or_stats;

/* Fill the ghost layer of one padded coefficient field by the face boundary
 * conditions (periodic: wrap; Dirichlet: untouched; every other kind: copy of
 * the adjacent interior cell). */
void or_fill_ghosts(const or_grid *g, double *a);

/* The same for the six tensor planes; at a reflecting face the components
 * f_dj (j != d) of the mirrored cell change sign. */
void or_fill_tensor_ghosts(const or_grid *g, double *const f[6]);

/* Ghost cells of the radiation state x = (E, Fx, Fy, Fz), by face kind:
 *   periodic   wrap;
 *   outflow    zero gradient (Sec. 3.3): the ghost is the boundary cell;
 *   Dirichlet  data (left as given), or 0 for the linear operator;
 *   open       characteristic outflow: the boundary cell's state with the
 *              amplitude of the incoming characteristic of the d-flux
 *              (speed c sqrt(f_dd), left eigenvector (1/2, +-e_d / (2 c sqrt(f_dd))))
 *              replaced by its value in the old state xo (0 for the linear operator);
 *   Marshak    c E_w + 2 F_w,in = 4 F_inc at the wall (Sec. 3.4) with E_w, F_w the
 *              means of ghost and cell and F_in the flux component into the domain:
 *              F_ghost = F_cell, E_ghost = 8 F_inc / c -+ 4 F_d,cell / c - E_cell
 *              (F_inc dropped for the linear operator);
 *   reflect    mirror: E and the tangential F copied, F_d negated.
 * linear != 0 fills the ghosts of the linear operator (the affine parts dropped). */
void or_fill_state_ghosts(const or_grid *g, const or_coef *cf, double *const x[4], double *const xo[4],
                          int linear);

/* Corrected HLLE wave speed at all low faces: Cd[index(i,j,k)] is the speed
 * of the face between cell (i,j,k) - e_d and (i,j,k), for i_d in [0, n_d].
 * Coefficient ghosts must already hold their boundary values. */
void or_face_speeds(const or_grid *g, const or_coef *cf, double *Cx, double *Cy, double *Cz);

/* Linear transport operator applied to padded x = (E, Fx, Fy, Fz) with the
 * ghosts of x as given (caller fills them):
 *   y_E = dE * E + (dt/h) div PhiE,  y_Fj = (1 + sR) F_j + (dt/h) div PhiF_j.
 * dE is a padded per-cell diagonal of the E rows. Interior of y is written. */
void or_apply(const or_grid *g, const or_coef *cf, const double *dE,
              double *const x[4], double *const y[4]);

/* Nonlinear residual (R_E, R_Fx, R_Fy, R_Fz, R_T) of the backward-Euler system
 * at state (E, F, T); E/F ghosts are filled here for periodic/outflow faces,
 * Dirichlet ghost values are taken from the passed arrays. */
void or_residual(const or_grid *g, const or_coef *cf,
                 const double *En, double *const Fn[3], const double *Tn,
                 double *E, double *const F[3], const double *T,
                 double *const R[5]);

/* Scaled residual norms of a state: out[0..2] = E, F, T parts, out[3] = max. */
void or_scaled_residual(const or_grid *g, const or_coef *cf,
                        const double *En, double *const Fn[3], const double *Tn,
                        double *E, double *const F[3], const double *T, double out[4]);

/* Per-cell exchange solve: T >= 0 with alpha (T - Tn) + sP (aR T^4 - E) = 0. */
double or_exchange_T(double alpha, double Tn, double sP, double aR, double E, int *neg);

/* One implicit radiation step.  On entry E, F, T hold the old state (their
 * ghosts hold Dirichlet data where used); on exit they hold the new state.
 * With p->energy_fix the committed gas energy is e(T_N) + dt dE (see or_stats),
 * so that the exchange terms of the radiation and gas equations cancel. */
int or_rad_step(const or_grid *g, const or_coef *cf, const or_params *p,
                double *E, double *const F[3], double *T, or_stats *st);

/* Local closures (Sec. 4.1): kind OR_EDDINGTON gives f = I/3, OR_M1 the M1
 * tensor from the lagged (E, F) (see oracle.c for the readings).  Unpadded
 * arrays of ncells; f[0..5] = xx, yy, zz, xy, xz, yz. */
enum { OR_EDDINGTON = 0, OR_M1 = 1 };
void or_closure(long ncells, int kind, double c, const double *E, const double *Fx, const double *Fy,
                const double *Fz, double *const f[6]);

int or_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
