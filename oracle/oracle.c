/*
 * oracle.c -- plain FP64 CPU oracle for the implicit VET radiation step.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability, not speed:
 * every face flux is formed explicitly, every Krylov vector operation is a
 * plain loop, the Krylov solver is textbook restarted GMRES with modified
 * Gram-Schmidt (Saad & Schultz 1986, the solver the paper names in
 * Sec. 2.3.4), and the per-cell gas temperature solve is Newton's method on
 * the quartic of eq. PicardTemp.  OpenMP only splits independent per-cell
 * loops.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- indexing */

static size_t padded_size(const or_grid *g)
{
    return (size_t)(g->nx + 2) * (size_t)(g->ny + 2) * (size_t)(g->nz + 2);
}

static size_t idx(const or_grid *g, int i, int j, int k)
{
    return (size_t)(i + 1) + (size_t)(g->nx + 2) * ((size_t)(j + 1) + (size_t)(g->ny + 2) * (size_t)(k + 1));
}

/* offset of one cell step along direction d in the padded layout */
static size_t step(const or_grid *g, int d)
{
    if (d == 0) return 1;
    if (d == 1) return (size_t)(g->nx + 2);
    return (size_t)(g->nx + 2) * (size_t)(g->ny + 2);
}

/* component index of the symmetric tensor f_{ab} in the (xx,yy,zz,xy,xz,yz) order */
static int tens(int a, int b)
{
    if (a == b) return a;
    if (a > b) { int t = a; a = b; b = t; }
    if (a == 0 && b == 1) return 3;
    if (a == 0 && b == 2) return 4;
    return 5;
}

static double *alloc_padded(const or_grid *g)
{
    return (double *)calloc(padded_size(g), sizeof(double));
}

/* ----------------------------------------------------------- ghost layers */

/* Fill one face's ghost layer of a coefficient field.  face = 2*d + side (side 0: low, 1: high). */
static void fill_face(const or_grid *g, double *a, int face, int zero_dirichlet)
{
    int d = face / 2, side = face % 2;
    int n[3] = {g->nx, g->ny, g->nz};
    int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
    int kind = g->bc[face];
    for (int q2 = 0; q2 < n[a2]; ++q2)
        for (int q1 = 0; q1 < n[a1]; ++q1) {
            int gh[3], src[3];
            gh[a1] = src[a1] = q1;
            gh[a2] = src[a2] = q2;
            gh[d] = side ? n[d] : -1;
            if (kind == OR_PERIODIC)
                src[d] = side ? 0 : n[d] - 1;
            else
                src[d] = side ? n[d] - 1 : 0;
            size_t gi = idx(g, gh[0], gh[1], gh[2]);
            if (kind == OR_DIRICHLET) {
                if (zero_dirichlet) a[gi] = 0.0;
            } else {
                a[gi] = a[idx(g, src[0], src[1], src[2])];
            }
        }
}

void or_fill_ghosts(const or_grid *g, double *a)
{
    for (int f = 0; f < 6; ++f) fill_face(g, a, f, 0);
}

/* component index of the symmetric tensor f_{ab} in the (xx,yy,zz,xy,xz,yz) order */
static int tens(int a, int b);

void or_fill_tensor_ghosts(const or_grid *g, double *const f[6])
{
    for (int q = 0; q < 6; ++q) or_fill_ghosts(g, f[q]);
    int n[3] = {g->nx, g->ny, g->nz};
    for (int face = 0; face < 6; ++face) {
        if (g->bc[face] != OR_REFLECT) continue;
        int d = face / 2, side = face % 2, a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        for (int q2 = 0; q2 < n[a2]; ++q2)
            for (int q1 = 0; q1 < n[a1]; ++q1) {
                int gh[3];
                gh[a1] = q1;
                gh[a2] = q2;
                gh[d] = side ? n[d] : -1;
                size_t gi = (size_t)(gh[0] + 1) + (size_t)(g->nx + 2) * ((size_t)(gh[1] + 1) + (size_t)(g->ny + 2) * (size_t)(gh[2] + 1));
                for (int j = 0; j < 3; ++j)
                    if (j != d) f[tens(d, j)][gi] = -f[tens(d, j)][gi];
            }
    }
}

void or_fill_state_ghosts(const or_grid *g, const or_coef *cf, double *const x[4], double *const xo[4],
                          int linear)
{
    int n[3] = {g->nx, g->ny, g->nz};
    for (int face = 0; face < 6; ++face) {
        int kind = g->bc[face];
        int d = face / 2, side = face % 2, a1 = (d + 1) % 3, a2 = (d + 2) % 3;
        /* sign of the incoming direction along d: +1 at the low face, -1 at the high one */
        double sin_ = side ? -1.0 : 1.0;
        for (int q2 = 0; q2 < n[a2]; ++q2)
            for (int q1 = 0; q1 < n[a1]; ++q1) {
                int gh[3], src[3];
                gh[a1] = src[a1] = q1;
                gh[a2] = src[a2] = q2;
                gh[d] = side ? n[d] : -1;
                if (kind == OR_PERIODIC)
                    src[d] = side ? 0 : n[d] - 1;
                else
                    src[d] = side ? n[d] - 1 : 0;
                size_t gi = idx(g, gh[0], gh[1], gh[2]), c = idx(g, src[0], src[1], src[2]);
                if (kind == OR_PERIODIC || kind == OR_OUTFLOW) {
                    for (int q = 0; q < 4; ++q) x[q][gi] = x[q][c];
                } else if (kind == OR_DIRICHLET) {
                    if (linear)
                        for (int q = 0; q < 4; ++q) x[q][gi] = 0.0;
                } else if (kind == OR_OPEN) {
                    double fdd = cf->f[d][c];
                    for (int q = 0; q < 4; ++q) x[q][gi] = x[q][c];
                    if (fdd > 0.0) {
                        double a = g->c * sqrt(fdd);
                        double in_now = 0.5 * (x[0][c] + sin_ * x[1 + d][c] / a);
                        double in_old = (linear || !xo) ? 0.0 : 0.5 * (xo[0][c] + sin_ * xo[1 + d][c] / a);
                        double delta = in_old - in_now;
                        x[0][gi] += delta;
                        for (int j = 0; j < 3; ++j) x[1 + j][gi] += delta * sin_ * g->c * g->c * cf->f[tens(d, j)][c] / a;
                    }
                } else if (kind == OR_MARSHAK) {
                    for (int q = 1; q < 4; ++q) x[q][gi] = x[q][c];
                    x[0][gi] = (linear ? 0.0 : 8.0 * g->finc[face] / g->c) - 4.0 * sin_ * x[1 + d][c] / g->c - x[0][c];
                } else if (kind == OR_REFLECT) {
                    for (int q = 0; q < 4; ++q) x[q][gi] = x[q][c];
                    x[1 + d][gi] = -x[1 + d][c];
                }
            }
    }
}

/* ------------------------------------------------------ local coefficients */

static double sigma_R(const or_coef *cf, size_t i) { return cf->rho[i] * cf->kR[i]; }
static double s_P(const or_grid *g, const or_coef *cf, size_t i) { return g->c * g->dt * cf->rho[i] * cf->kP[i]; }
static double s_R(const or_grid *g, const or_coef *cf, size_t i) { return g->c * g->dt * sigma_R(cf, i); }
static double alpha_of(const or_grid *g, const or_coef *cf, size_t i) { return cf->rho[i] * g->cv; }

/* gas internal energy and heat capacity: alpha T and alpha, or (Sec. 3.4, the Marshak-wave
 * gas) C_v = alpha T^3 with E_int = alpha T^4 / 4 */
static double gas_e(const or_grid *g, double alpha, double T)
{
    return g->cv_cubic ? 0.25 * alpha * T * T * T * T : alpha * T;
}
static double gas_C(const or_grid *g, double alpha, double T) { return g->cv_cubic ? alpha * T * T * T : alpha; }

/* the exchange row with the cubic gas is linear in T^4:
 *   (alpha/4 + sP aR) T^4 = alpha Tn^4 / 4 + sP E + X */
static double exchange_T4(double alpha, double Tn, double sP, double aR, double E, double X, int *neg)
{
    double den = 0.25 * alpha + sP * aR;
    if (den == 0.0) return Tn;
    double num = 0.25 * alpha * Tn * Tn * Tn * Tn + sP * E + X;
    if (!(num > 0.0)) {
        if (neg) *neg = 1;
        return 0.0;
    }
    return sqrt(sqrt(num / den));
}

/* ------------------------------------------------------ velocity (O(v/c)) terms */

/* With beta = v/c, kappa_E = kappa_P and kappa_F = kappa_R, dt times the O(v/c)
 * parts of the four-force (eq. G and the G0 of the radiation energy equation):
 *   energy row:  (sR - 2 sP) beta.F / c + (sP - sR) (beta.beta + beta.f.beta) E
 *   flux row j: -sR c E (beta_j + (f beta)_j)
 * X (the first) is also the O(v/c) energy the gas receives (eq. G0explicit). */
static int has_velocity(const or_coef *cf) { return cf->beta[0] != NULL; }

static void vel_vectors(const or_coef *cf, size_t i, double b[3], double fb[3])
{
    for (int a = 0; a < 3; ++a) b[a] = cf->beta[a][i];
    for (int a = 0; a < 3; ++a) {
        fb[a] = 0.0;
        for (int k = 0; k < 3; ++k) fb[a] += cf->f[tens(a, k)][i] * b[k];
    }
}

/* the energy-row term X at cell i for the state (E, F) */
static double vel_energy(const or_grid *g, const or_coef *cf, size_t i, double E, const double F[3])
{
    double b[3], fb[3];
    vel_vectors(cf, i, b, fb);
    double bF = 0.0, bb = 0.0, bfb = 0.0;
    for (int a = 0; a < 3; ++a) {
        bF += b[a] * F[a];
        bb += b[a] * b[a];
        bfb += b[a] * fb[a];
    }
    double sP = g->c * g->dt * cf->rho[i] * cf->kP[i], sR = g->c * g->dt * cf->rho[i] * cf->kR[i];
    return (sR - 2.0 * sP) * bF / g->c + (sP - sR) * (bb + bfb) * E;
}

/* Optical-depth parameter of the wave-speed correction for one cell and one
 * direction (eq. taucorrect): tau = (10 dl rho kappa_R)^2 / (2 f), dl = h.
 * A cell with no opacity has tau = 0; a cell with zero diagonal Eddington
 * factor and nonzero opacity has tau = +inf. */
static double cell_tau(const or_grid *g, double sigR, double fdd)
{
    if (sigR == 0.0) return 0.0;
    if (fdd == 0.0) return INFINITY;
    double q = 10.0 * g->h * sigR;
    return q * q / (2.0 * fdd);
}

/* Corrected HLLE wave speed at a face (Sec. 2.3.3): C = sqrt(f) c sqrt((1-e^-tau)/tau),
 * tau = mean of the two cells' values (eq. wavespeedtau, same refinement level),
 * f = the larger of the two cells' diagonal factors along the face normal. */
static double face_speed(const or_grid *g, double fL, double fR, double sigL, double sigR)
{
    double tau = 0.5 * (cell_tau(g, sigL, fL) + cell_tau(g, sigR, fR));
    double fc = fL > fR ? fL : fR;
    double corr;
    if (tau == 0.0)
        corr = 1.0;
    else if (isinf(tau))
        corr = 0.0;
    else
        corr = sqrt(-expm1(-tau) / tau);
    return g->c * sqrt(fc) * corr;
}

void or_face_speeds(const or_grid *g, const or_coef *cf, double *Cx, double *Cy, double *Cz)
{
    double *C[3] = {Cx, Cy, Cz};
    int n[3] = {g->nx, g->ny, g->nz};
    for (int d = 0; d < 3; ++d) {
        size_t s = step(g, d);
#pragma omp parallel for
        for (int k = 0; k < g->nz + (d == 2); ++k)
            for (int j = 0; j < g->ny + (d == 1); ++j)
                for (int i = 0; i < g->nx + (d == 0); ++i) {
                    (void)n;
                    size_t R = idx(g, i, j, k), L = R - s;
                    C[d][R] = face_speed(g, cf->f[d][L], cf->f[d][R], sigma_R(cf, L), sigma_R(cf, R));
                }
    }
}

/* -------------------------------------------------------------- transport */

/* HLLE flux (first-order, piecewise-constant states) through the face between
 * padded cells L and R = L + e_d, with symmetric signal speeds -C, +C:
 *   Phi = (Flux(U_L) + Flux(U_R))/2 - C (U_R - U_L)/2,
 * where the flux of E along d is F_d and the flux of F_j along d is c^2 f_dj E. */
static void hlle_flux(const or_grid *g, const or_coef *cf, double *const x[4], int d,
                      size_t L, size_t R, double C, double phi[4])
{
    double c2 = g->c * g->c;
    double EL = x[0][L], ER = x[0][R];
    phi[0] = 0.5 * (x[1 + d][L] + x[1 + d][R]) - 0.5 * C * (ER - EL);
    for (int j = 0; j < 3; ++j) {
        const double *fdj = cf->f[tens(d, j)];
        phi[1 + j] = 0.5 * c2 * (fdj[L] * EL + fdj[R] * ER) - 0.5 * C * (x[1 + j][R] - x[1 + j][L]);
    }
}

/* y = diag * x + (dt/h) * sum_d (Phi_{i+1/2} - Phi_{i-1/2});  ghosts of x as given.
 * Face fluxes are formed once per face and then differenced.  With a velocity
 * the O(v/c) terms are added, those of the energy row times vscale (NULL: 1). */
static void transport_apply(const or_grid *g, const or_coef *cf, const double *const C[3],
                            const double *dE, double *const x[4], double *const y[4], const double *vscale)
{
    size_t np = padded_size(g);
    double lam = g->dt / g->h;
    double *phi[3][4];
    for (int d = 0; d < 3; ++d)
        for (int q = 0; q < 4; ++q) phi[d][q] = (double *)calloc(np, sizeof(double));

    for (int d = 0; d < 3; ++d) {
        size_t s = step(g, d);
#pragma omp parallel for
        for (int k = 0; k < g->nz + (d == 2); ++k)
            for (int j = 0; j < g->ny + (d == 1); ++j)
                for (int i = 0; i < g->nx + (d == 0); ++i) {
                    size_t R = idx(g, i, j, k), L = R - s;
                    double p[4];
                    hlle_flux(g, cf, x, d, L, R, C[d][R], p);
                    for (int q = 0; q < 4; ++q) phi[d][q][R] = p[q];
                }
    }

#pragma omp parallel for
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = idx(g, i, j, k);
                double sR = s_R(g, cf, c);
                for (int q = 0; q < 4; ++q) {
                    double div = 0.0;
                    for (int d = 0; d < 3; ++d) div += phi[d][q][c + step(g, d)] - phi[d][q][c];
                    double diag = (q == 0) ? dE[c] : 1.0 + sR;
                    y[q][c] = diag * x[q][c] + lam * div;
                }
                if (has_velocity(cf)) {
                    double b[3], fb[3], Fc[3] = {x[1][c], x[2][c], x[3][c]};
                    vel_vectors(cf, c, b, fb);
                    y[0][c] += (vscale ? vscale[c] : 1.0) * vel_energy(g, cf, c, x[0][c], Fc);
                    for (int q = 0; q < 3; ++q) y[1 + q][c] -= sR * g->c * x[0][c] * (b[q] + fb[q]);
                }
            }

    for (int d = 0; d < 3; ++d)
        for (int q = 0; q < 4; ++q) free(phi[d][q]);
}

static void all_face_speeds(const or_grid *g, const or_coef *cf, double *C[3])
{
    for (int d = 0; d < 3; ++d) C[d] = alloc_padded(g);
    or_face_speeds(g, cf, C[0], C[1], C[2]);
}

void or_apply(const or_grid *g, const or_coef *cf, const double *dE, double *const x[4], double *const y[4])
{
    double *C[3];
    all_face_speeds(g, cf, C);
    transport_apply(g, cf, (const double *const *)C, dE, x, y, NULL);
    for (int d = 0; d < 3; ++d) free(C[d]);
}

/* --------------------------------------------------------------- residual */

void or_residual(const or_grid *g, const or_coef *cf, const double *En, double *const Fn[3],
                 const double *Tn, double *E, double *const F[3], const double *T, double *const R[5])
{
    double *x[4] = {E, F[0], F[1], F[2]};
    double *xo[4] = {(double *)En, Fn[0], Fn[1], Fn[2]};
    or_fill_state_ghosts(g, cf, x, xo, 0);
    double *dE = alloc_padded(g);
#pragma omp parallel for
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = idx(g, i, j, k);
                dE[c] = 1.0 + s_P(g, cf, c);
            }
    or_apply(g, cf, dE, x, R);
#pragma omp parallel for
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = idx(g, i, j, k);
                double sP = s_P(g, cf, c), T4 = T[c] * T[c] * T[c] * T[c];
                R[0][c] += -En[c] - sP * g->aR * T4;
                for (int q = 0; q < 3; ++q) R[1 + q][c] -= Fn[q][c];
                double a = alpha_of(g, cf, c);
                R[4][c] = gas_e(g, a, T[c]) - gas_e(g, a, Tn[c]) + sP * (g->aR * T4 - E[c]);
                if (has_velocity(cf) && cf->vel_implicit) {
                    double Fc[3] = {F[0][c], F[1][c], F[2][c]};
                    R[4][c] -= vel_energy(g, cf, c, E[c], Fc);   /* the gas receives the O(v/c) energy */
                }
            }
    free(dE);
}

/* Scaling weights of the convergence test: W_E = 1 + sP + (dt/2h) sum_faces C,
 * W_F = 1 + sR + (dt/2h) sum_faces C, W_T = alpha + 4 sP aR T^3. */
static void weights(const or_grid *g, const or_coef *cf, double *const C[3], size_t c,
                    const double *T, double *WE, double *WF, double *WT)
{
    double sumC = 0.0;
    for (int d = 0; d < 3; ++d) sumC += C[d][c] + C[d][c + step(g, d)];
    double half = 0.5 * g->dt / g->h * sumC;
    double sP = s_P(g, cf, c);
    *WE = 1.0 + sP + half;
    *WF = 1.0 + s_R(g, cf, c) + half;
    *WT = gas_C(g, alpha_of(g, cf, c), T[c]) + 4.0 * sP * g->aR * T[c] * T[c] * T[c];
}

void or_scaled_residual(const or_grid *g, const or_coef *cf, const double *En, double *const Fn[3],
                        const double *Tn, double *E, double *const F[3], const double *T, double out[4])
{
    double *R[5];
    for (int q = 0; q < 5; ++q) R[q] = alloc_padded(g);
    or_residual(g, cf, En, Fn, Tn, E, F, T, R);
    double *C[3];
    all_face_speeds(g, cf, C);
    double rE = 0, rF = 0, rT = 0, nE = 0, nF = 0, nT = 0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t c = idx(g, i, j, k);
                double WE, WF, WT;
                weights(g, cf, C, c, T, &WE, &WF, &WT);
                rE += (R[0][c] / WE) * (R[0][c] / WE);
                for (int q = 1; q < 4; ++q) rF += (R[q][c] / WF) * (R[q][c] / WF);
                /* T >= 0 is the physical range: where the exchange equation has no
                 * non-negative root (R_T > 0 at T = 0) the constraint T = 0 is active
                 * and the exchange row counts as satisfied */
                double RT = (T[c] == 0.0 && R[4][c] > 0.0) ? 0.0 : R[4][c];
                if (WT > 0) rT += (RT / WT) * (RT / WT);   /* WT = 0 only at T = 0 with C_v(0) = 0 */
                nE += E[c] * E[c];
                for (int q = 0; q < 3; ++q) nF += F[q][c] * F[q][c];
                nT += T[c] * T[c];
            }
    double dEn = sqrt(nE) > 0 ? sqrt(nE) : 1e-300;
    double dFn = sqrt(nF) + g->c * sqrt(nE);
    if (dFn == 0) dFn = 1e-300;
    double dTn = sqrt(nT) > 0 ? sqrt(nT) : 1e-300;
    out[0] = sqrt(rE) / dEn;
    out[1] = sqrt(rF) / dFn;
    out[2] = sqrt(rT) / dTn;
    out[3] = out[0];
    if (out[1] > out[3]) out[3] = out[1];
    if (out[2] > out[3]) out[3] = out[2];
    for (int q = 0; q < 5; ++q) free(R[q]);
    for (int d = 0; d < 3; ++d) free(C[d]);
}

/* ---------------------------------------------------------------- exchange */

/* Gas temperature update of eq. PicardTemp with E_int = alpha T:
 *   g(T) = alpha (T - Tn) + sP (aR T^4 - E) = 0.
 * g is increasing and convex for T >= 0, so Newton's method (analytic
 * derivative, as the paper prescribes) started above the root descends
 * monotonically onto it; it stops once an iterate no longer decreases, i.e.
 * at round-off.  The start is the smaller of the two single-term bounds. */
static double exchange_newton(double alpha, double Tn, double sP, double aR, double E, double eps_N, int *neg)
{
    if (sP == 0.0) return Tn;
    double rhs = alpha * Tn + sP * E;
    if (!(rhs > 0.0)) {
        if (neg) *neg = 1;
        return 0.0;
    }
    double T = pow(rhs / (sP * aR), 0.25);
    if (alpha > 0.0 && rhs / alpha < T) T = rhs / alpha;
    for (int it = 0; it < 200; ++it) {
        double T3 = T * T * T;
        double gv = alpha * (T - Tn) + sP * (aR * T3 * T - E);
        double dg = alpha + 4.0 * sP * aR * T3;
        double Tnew = T - gv / dg;
        if (!(Tnew < T)) break;
        /* the paper's stop rule: relative change of T below eps_N */
        int done = eps_N > 0.0 && T - Tnew <= eps_N * Tnew;
        T = Tnew;
        if (done) break;
    }
    return T;
}

double or_exchange_T(double alpha, double Tn, double sP, double aR, double E, int *neg)
{
    return exchange_newton(alpha, Tn, sP, aR, E, 0.0, neg);
}

/* inverse of the gas internal energy e(T) (alpha T, or alpha T^4 / 4), clamped at T = 0 */
static double gas_T_of_e(const or_grid *g, double alpha, double e)
{
    if (!(e > 0.0) || !(alpha > 0.0)) return 0.0;
    return g->cv_cubic ? sqrt(sqrt(4.0 * e / alpha)) : e / alpha;
}

/* ------------------------------------------------------------------- GMRES */

typedef struct {
    const or_grid *g;
    const or_coef *cf;
    double *C[3];
    double *dE;      /* E-row diagonal of the current linear system */
    double *vscale;  /* factor of the energy row's O(v/c) terms in the linear system (NULL: 1) */
    double *pre[2];  /* Jacobi scaling: 1/D_E, 1/D_F */
    double *px[4], *py[4];
    size_t N;
} lin_ctx;

/* pack/unpack between interior vectors [E | Fx | Fy | Fz] and padded arrays */
static void unpack(const lin_ctx *o, const double *v, double *const a[4])
{
    const or_grid *g = o->g;
    for (int q = 0; q < 4; ++q) {
        size_t n = 0;
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) a[q][idx(g, i, j, k)] = v[q * o->N + n++];
    }
}

static void pack(const lin_ctx *o, double *const a[4], double *v)
{
    const or_grid *g = o->g;
    for (int q = 0; q < 4; ++q) {
        size_t n = 0;
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) v[q * o->N + n++] = a[q][idx(g, i, j, k)];
    }
}

/* The Krylov solve works on (E, F/c): radiation energy density and flux then
 * carry the same units, so the 2-norms GMRES minimises weigh both alike for
 * any unit system (the flux rows are divided by c, the flux unknowns
 * multiplied by c; the solution of the linear system is unchanged). */
static void to_physical(const lin_ctx *o, double *v)
{
    for (size_t n = o->N; n < 4 * o->N; ++n) v[n] *= o->g->c;
}

static void to_scaled(const lin_ctx *o, double *v)
{
    for (size_t n = o->N; n < 4 * o->N; ++n) v[n] /= o->g->c;
}

/* out = D^-1 A_lin v for v = (E, F/c): the linear operator with homogeneous
 * Dirichlet ghosts, flux rows divided by c, left-scaled by its diagonal */
static void lin_apply_prec(lin_ctx *o, const double *v, double *out)
{
    double *u = (double *)malloc(4 * o->N * sizeof(double));
    memcpy(u, v, 4 * o->N * sizeof(double));
    to_physical(o, u);
    unpack(o, u, o->px);
    free(u);
    or_fill_state_ghosts(o->g, o->cf, o->px, NULL, 1);
    transport_apply(o->g, o->cf, (const double *const *)o->C, o->dE, o->px, o->py, o->vscale);
    pack(o, o->py, out);
    to_scaled(o, out);
    for (size_t n = 0; n < 4 * o->N; ++n) out[n] *= o->pre[n < o->N ? 0 : 1][n % o->N];
}

static double dot(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Restarted GMRES(m), left-preconditioned, modified Gram-Schmidt with Givens
 * rotations.  Solves A_lin d = rhs for d (d starts at zero).  Stops when the
 * true preconditioned residual norm is <= target, when a restart cycle fails
 * to reduce it by 1%, or after max_it iterations.  Returns iterations used. */
static int gmres(lin_ctx *o, const double *rhs, double *d, double rtol, double atol, int m, int max_it)
{
    size_t n = 4 * o->N;
    double *V = (double *)malloc((size_t)(m + 1) * n * sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(m * sizeof(double)), *sn = (double *)malloc(m * sizeof(double));
    double *gv = (double *)malloc((m + 1) * sizeof(double)), *y = (double *)malloc(m * sizeof(double));
    double *r = (double *)malloc(n * sizeof(double)), *w = (double *)malloc(n * sizeof(double));
    int its = 0;
    memset(d, 0, n * sizeof(double));

    for (size_t i = 0; i < n; ++i) r[i] = rhs[i] * o->pre[i < o->N ? 0 : 1][i % o->N];
    double beta0 = sqrt(dot(r, r, n));
    double target = rtol * beta0 > atol ? rtol * beta0 : atol;
    double beta = beta0, prev_cycle = INFINITY;

    while (beta > target && its < max_it && beta < 0.99 * prev_cycle) {
        prev_cycle = beta;
        for (size_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        memset(gv, 0, (m + 1) * sizeof(double));
        gv[0] = beta;
        int j, cols = 0;
        for (j = 0; j < m && its < max_it; ++j) {
            double *vj = V + (size_t)j * n;
            lin_apply_prec(o, vj, w);
            ++its;
            for (int i = 0; i <= j; ++i) {
                double hij = dot(w, V + (size_t)i * n, n);
                H[i * m + j] = hij;
                for (size_t q = 0; q < n; ++q) w[q] -= hij * V[(size_t)i * n + q];
            }
            double hn = sqrt(dot(w, w, n));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], b = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * b;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            double a = H[j * m + j], b = H[(j + 1) * m + j];
            double rr = hypot(a, b);
            cs[j] = rr > 0 ? a / rr : 1.0;
            sn[j] = rr > 0 ? b / rr : 0.0;
            H[j * m + j] = rr;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            cols = j + 1;
            if (hn > 0)
                for (size_t q = 0; q < n; ++q) V[(size_t)(j + 1) * n + q] = w[q] / hn;
            if (fabs(gv[j + 1]) <= target || hn == 0.0) break;
        }
        for (int i = cols - 1; i >= 0; --i) {
            double s = gv[i];
            for (int l = i + 1; l < cols; ++l) s -= H[i * m + l] * y[l];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < cols; ++i)
            for (size_t q = 0; q < n; ++q) d[q] += y[i] * V[(size_t)i * n + q];
        /* true residual of the correction */
        lin_apply_prec(o, d, w);
        for (size_t i = 0; i < n; ++i) r[i] = rhs[i] * o->pre[i < o->N ? 0 : 1][i % o->N] - w[i];
        beta = sqrt(dot(r, r, n));
    }
    free(V); free(H); free(cs); free(sn); free(gv); free(y); free(r); free(w);
    return its;
}

/* ---------------------------------------------------------------- the step */

int or_rad_step(const or_grid *g, const or_coef *cf, const or_params *p,
                double *E, double *const F[3], double *T, or_stats *st)
{
    size_t np = padded_size(g);
    size_t N = (size_t)g->nx * g->ny * g->nz;
    memset(st, 0, sizeof(*st));

    /* old state (ghosts keep the Dirichlet data) */
    double *En = alloc_padded(g), *Fn[3], *Tn = alloc_padded(g);
    memcpy(En, E, np * sizeof(double));
    memcpy(Tn, T, np * sizeof(double));
    for (int q = 0; q < 3; ++q) {
        Fn[q] = alloc_padded(g);
        memcpy(Fn[q], F[q], np * sizeof(double));
    }

    lin_ctx o;
    o.g = g;
    o.cf = cf;
    o.N = N;
    all_face_speeds(g, cf, o.C);
    o.dE = alloc_padded(g);
    /* implicit O(v/c) gas energy with the linearised emission: eliminating the gas energy
     * leaves the fraction 1 - eta of the energy row's O(v/c) terms (Newton-consistent) */
    o.vscale = (has_velocity(cf) && cf->vel_implicit && p->mode != OR_LAGGED) ? alloc_padded(g) : NULL;
    for (int q = 0; q < 4; ++q) { o.px[q] = alloc_padded(g); o.py[q] = alloc_padded(g); }
    o.pre[0] = (double *)malloc(N * sizeof(double));
    o.pre[1] = (double *)malloc(N * sizeof(double));

    double *bE = alloc_padded(g), *Tstar = alloc_padded(g), *dE = alloc_padded(g);
    memcpy(Tstar, Tn, np * sizeof(double)); /* the first guess is the old temperature */
    double *x[4] = {E, F[0], F[1], F[2]};
    double *xo_state[4] = {En, Fn[0], Fn[1], Fn[2]};
    double *y[4];
    for (int q = 0; q < 4; ++q) y[q] = alloc_padded(g);
    double *rhs = (double *)malloc(4 * N * sizeof(double));
    double *dv = (double *)malloc(4 * N * sizeof(double));
    double *xprev = (double *)malloc(4 * N * sizeof(double));
    double lam = g->dt / g->h;
    double last_res = INFINITY;
    int stall = 0;

    for (int k = 1; k <= p->max_picard; ++k) {
        /* linear system of this Picard iteration, emission taken at Tstar */
#pragma omp parallel for
        for (int kk = 0; kk < g->nz; ++kk)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t c = idx(g, i, j, kk);
                    double sP = s_P(g, cf, c), a = alpha_of(g, cf, c);
                    double Ts = Tstar[c], Ts3 = Ts * Ts * Ts, Ts4 = Ts3 * Ts;
                    if (p->mode == OR_LAGGED) {
                        o.dE[c] = 1.0 + sP;
                        bE[c] = En[c] + sP * g->aR * Ts4;
                    } else {
                        /* emission and gas energy linearised about Tstar, gas energy eliminated */
                        double den = gas_C(g, a, Ts) + 4.0 * sP * g->aR * Ts3;
                        double eta = den > 0 ? 4.0 * sP * g->aR * Ts3 / den : 0.0;
                        o.dE[c] = 1.0 + sP * (1.0 - eta);
                        if (!g->cv_cubic)
                            bE[c] = En[c] + eta * a * Tn[c] - 3.0 * (1.0 - eta) * sP * g->aR * Ts4;
                        else
                            bE[c] = En[c] + (1.0 - eta) * sP * g->aR * Ts4 +
                                    eta * (gas_e(g, a, Tn[c]) - gas_e(g, a, Ts));
                        if (o.vscale) o.vscale[c] = 1.0 - eta;
                    }
                }
        /* Jacobi scaling of this system */
        {
            size_t n = 0;
            for (int kk = 0; kk < g->nz; ++kk)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i, ++n) {
                        size_t c = idx(g, i, j, kk);
                        double sumC = 0.0;
                        for (int d = 0; d < 3; ++d) sumC += o.C[d][c] + o.C[d][c + step(g, d)];
                        o.pre[0][n] = 1.0 / (o.dE[c] + 0.5 * lam * sumC);
                        o.pre[1][n] = 1.0 / (1.0 + s_R(g, cf, c) + 0.5 * lam * sumC);
                    }
        }
        /* residual of the linear system at the current iterate (boundary data in the ghosts) */
        or_fill_state_ghosts(g, cf, x, xo_state, 0);
        transport_apply(g, cf, (const double *const *)o.C, o.dE, x, y, o.vscale);
        {
            size_t n = 0;
            for (int kk = 0; kk < g->nz; ++kk)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i, ++n) {
                        size_t c = idx(g, i, j, kk);
                        rhs[n] = bE[c] - y[0][c];
                        for (int q = 0; q < 3; ++q) rhs[(q + 1) * N + n] = Fn[q][c] - y[q + 1][c];
                    }
        }
        pack(&o, x, xprev);
        /* Krylov solve for the correction, then update (E, F) */
        {
            double bn = 0.0;
            for (size_t n = 0; n < N; ++n) {
                size_t kk = n / ((size_t)g->nx * g->ny), rem = n % ((size_t)g->nx * g->ny);
                size_t c = idx(g, (int)(rem % g->nx), (int)(rem / g->nx), (int)kk);
                double v = bE[c] * o.pre[0][n];
                bn += v * v;
                for (int q = 0; q < 3; ++q) { double u = Fn[q][c] / g->c * o.pre[1][n]; bn += u * u; }
            }
            to_scaled(&o, rhs);
            st->krylov_iters += gmres(&o, rhs, dv, p->lin_rtol, 1e-15 * sqrt(bn), p->gmres_m, p->max_krylov);
            to_physical(&o, dv);
        }
        {
            double *xv = (double *)malloc(4 * N * sizeof(double));
            for (size_t n = 0; n < 4 * N; ++n) xv[n] = xprev[n] + dv[n];
            unpack(&o, xv, x);
            free(xv);
        }
        /* per-cell Newton solve for the gas temperature with the new E */
        int neg = 0;
#pragma omp parallel for reduction(| : neg)
        for (int kk = 0; kk < g->nz; ++kk)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t c = idx(g, i, j, kk);
                    int flag = 0;
                    double a = alpha_of(g, cf, c), sP = s_P(g, cf, c), Tb = Tn[c], Eb = E[c], X = 0.0;
                    if (has_velocity(cf) && cf->vel_implicit) {
                        double Fc[3] = {F[0][c], F[1][c], F[2][c]};
                        X = vel_energy(g, cf, c, E[c], Fc);
                    }
                    if (g->cv_cubic) {
                        T[c] = exchange_T4(a, Tn[c], sP, g->aR, E[c], X, &flag);
                    } else {
                        /* alpha (T - Tn) + sP (aR T^4 - E) = X: shift Tn (or E without heat capacity) */
                        if (a > 0)
                            Tb += X / a;
                        else if (sP > 0)
                            Eb += X / sP;
                        T[c] = exchange_newton(a, Tb, sP, g->aR, Eb, p->eps_N, &flag);
                    }
                    neg |= flag;
                }
        st->neg_cells = neg;
        /* Energy correction of Sec. 2.3.4.  The radiation solve took the emission at the guess
         * T_o = Tstar, the gas solve at its root T_N, so the two exchange terms differ by
         * dt dE = sP (aR T_N^4 - e_rad) per cell.  e_rad is read off the radiation row: with
         * diagonal 1 + sP (1 - eta) and right-hand side bE that row equals the plain one
         * (1 + sP) E - E_n - sP e_rad, so sP e_rad = sP eta E + bE - E_n (eta = 0 lagged). */
        {
            double defect = 0.0, scale = 0.0, dmax = 0.0;
#pragma omp parallel for reduction(+ : defect, scale) reduction(max : dmax)
            for (int kk = 0; kk < g->nz; ++kk)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i) {
                        size_t c = idx(g, i, j, kk);
                        double sP = s_P(g, cf, c), a = alpha_of(g, cf, c), eta = 0.0;
                        if (p->mode != OR_LAGGED) {
                            double Ts = Tstar[c], Ts3 = Ts * Ts * Ts;
                            double den = gas_C(g, a, Ts) + 4.0 * sP * g->aR * Ts3;
                            eta = den > 0 ? 4.0 * sP * g->aR * Ts3 / den : 0.0;
                        }
                        double TN4 = T[c] * T[c] * T[c] * T[c];
                        double dEc = sP * g->aR * TN4 - (sP * eta * E[c] + bE[c] - En[c]);
                        if (sP == 0.0) dEc = 0.0;
                        dE[c] = dEc;
                        defect += dEc;
                        scale += En[c] + gas_e(g, a, Tn[c]);
                        double loc = fabs(E[c]) + gas_e(g, a, T[c]);
                        double r = loc > 0 ? fabs(dEc) / loc : (dEc != 0.0 ? INFINITY : 0.0);
                        if (r > dmax) dmax = r;
                    }
            st->energy_defect = scale != 0.0 ? defect / scale : defect;
            st->dE_max = dmax;
        }
        /* relative change of x_P = [E, F, T] over the iteration (per field, max) */
        {
            double dE2 = 0, nE2 = 0, dF2 = 0, nF2 = 0, dT2 = 0, nT2 = 0;
            size_t n = 0;
            for (int kk = 0; kk < g->nz; ++kk)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i, ++n) {
                        size_t c = idx(g, i, j, kk);
                        dE2 += dv[n] * dv[n];
                        nE2 += E[c] * E[c];
                        for (int q = 0; q < 3; ++q) { dF2 += dv[(q + 1) * N + n] * dv[(q + 1) * N + n]; nF2 += F[q][c] * F[q][c]; }
                        dT2 += (T[c] - Tstar[c]) * (T[c] - Tstar[c]);
                        nT2 += T[c] * T[c];
                    }
            double a = nE2 > 0 ? sqrt(dE2 / nE2) : 0.0;
            double b = (nF2 + nE2) > 0 ? sqrt(dF2) / (sqrt(nF2) + g->c * sqrt(nE2)) : 0.0;
            double cT = nT2 > 0 ? sqrt(dT2 / nT2) : 0.0;
            st->rel_change = a > b ? a : b;
            if (cT > st->rel_change) st->rel_change = cT;
        }
        memcpy(Tstar, T, np * sizeof(double));
        st->picard_iters = k;

        double res[4];
        or_scaled_residual(g, cf, En, Fn, Tn, E, F, T, res);
        st->res_E = res[0];
        st->res_F = res[1];
        st->res_T = res[2];
        st->scaled_residual = res[3];
        if (res[3] <= p->tol) { st->converged = 1; break; }
        if (p->eps_P > 0 && st->rel_change < p->eps_P) { st->converged = 1; break; }
        /* floor detection: two iterations in a row without any reduction */
        if (res[3] >= last_res) {
            if (++stall >= 2) { st->converged = res[3] < 1e-9 ? 2 : 0; break; }
        } else {
            stall = 0;
        }
        last_res = res[3];
    }

    if (p->energy_fix) {
        /* commit the gas energy that makes the two exchange terms cancel: e(T) = e(T_N) + dt dE,
         * T = 0 where that energy is not positive.  Fed back into the next Picard iteration this
         * would be the gas update alpha (T - T_n) = sP (E - e_rad), which diverges where
         * 4 sP aR T^3 > (1 + sP) alpha; applied once at the end it only moves the committed T. */
#pragma omp parallel for
        for (int kk = 0; kk < g->nz; ++kk)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t c = idx(g, i, j, kk);
                    double a = alpha_of(g, cf, c);
                    if (dE[c] != 0.0) T[c] = gas_T_of_e(g, a, gas_e(g, a, T[c]) + dE[c]);
                }
    }
    or_fill_state_ghosts(g, cf, x, xo_state, 0);
    free(En); free(Tn); free(bE); free(Tstar); free(dE); free(rhs); free(dv); free(xprev);
    for (int q = 0; q < 3; ++q) free(Fn[q]);
    for (int q = 0; q < 4; ++q) { free(o.px[q]); free(o.py[q]); free(y[q]); }
    for (int d = 0; d < 3; ++d) free(o.C[d]);
    free(o.dE); free(o.pre[0]); free(o.pre[1]);
    free(o.vscale);
    return st->converged ? 0 : 1;
}

/* ------------------------------------------------------------------------
 * Local closures of the closure comparison (Sec. 4.1): the Eddington
 * approximation f = I/3, and the M1 closure from the time-lagged state,
 *   f = (1 - chi)/2 I + (3 chi - 1)/2 n n,   n = F / |F|,
 *   chi = (3 + 4 g^2) / (5 + 2 sqrt(4 - 3 g^2)),   g = |F| / (c E).
 * Readings where the paper is silent: g is clipped to [0, 1] (|F| <= cE for a
 * physical field); where E <= 0, g = 1 if F != 0 and g = 0 if F = 0; with F = 0
 * the n n term has zero weight (chi(0) = 1/3), so n is not needed. */
void or_closure(long ncells, int kind, double c, const double *E, const double *Fx, const double *Fy,
                const double *Fz, double *const f[6])
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < ncells; ++i) {
        double fxx = 1.0 / 3.0, fyy = 1.0 / 3.0, fzz = 1.0 / 3.0, fxy = 0.0, fxz = 0.0, fyz = 0.0;
        if (kind == OR_M1) {
            const double F2 = Fx[i] * Fx[i] + Fy[i] * Fy[i] + Fz[i] * Fz[i];
            const double Fm = sqrt(F2);
            double g;
            if (E[i] > 0.0)
                g = Fm / (c * E[i]);
            else
                g = F2 > 0.0 ? 1.0 : 0.0;
            if (g > 1.0) g = 1.0;
            const double chi = (3.0 + 4.0 * g * g) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * g * g));
            const double iso = 0.5 * (1.0 - chi), beam = 0.5 * (3.0 * chi - 1.0);
            double nx = 0.0, ny = 0.0, nz = 0.0;
            if (F2 > 0.0) { nx = Fx[i] / Fm; ny = Fy[i] / Fm; nz = Fz[i] / Fm; }
            fxx = iso + beam * nx * nx;
            fyy = iso + beam * ny * ny;
            fzz = iso + beam * nz * nz;
            fxy = beam * nx * ny;
            fxz = beam * nx * nz;
            fyz = beam * ny * nz;
        }
        f[0][i] = fxx; f[1][i] = fyy; f[2][i] = fzz;
        f[3][i] = fxy; f[4][i] = fxz; f[5][i] = fyz;
    }
}
