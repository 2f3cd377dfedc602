// rad_device.h -- device-side building blocks of the implicit VET radiation step (gfx950).
//
// Internally the flux is carried as Ft = F / c, so that the operator of one
// Picard iteration becomes dimensionless and symmetric in its use of c:
//   E rows:  dE E   + nu sum_d (PhiE_{+d} - PhiE_{-d}),
//            PhiE   = (Ft_d,L + Ft_d,R)/2 - Ct (E_R - E_L)/2
//   Ft rows: (1+sR) Ft_j + nu sum_d (PhiF_{+d} - PhiF_{-d}),
//            PhiF_j = (f_dj,L E_L + f_dj,R E_R)/2 - Ct (Ft_j,R - Ft_j,L)/2
// with nu = c dt / h and Ct = C / c the corrected HLLE speed of Sec. 2.3.3
// (eq. taucorrect, eq. wavespeedtau same-level rule) divided by c.  This is the
// paper's operator with the flux rows divided by c and the flux unknowns
// multiplied by c; FP32 Krylov vectors then hold E and Ft at the same scale
// in any unit system.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace vr {

constexpr int kBlock = 256;   // threads per workgroup of the streaming kernels (4 wave64)
constexpr int kMaxM = 64;     // largest GMRES restart length
constexpr int kMaxAnderson = 5;  // most past iterates of the Anderson-accelerated Picard map

// Face kinds (the values of rad_bc_kind).  Every kind but periodic maps the
// neighbour across the face to the boundary cell itself; outflow keeps it (zero
// gradient), Dirichlet, open, Marshak and reflect then replace its state by
// their ghost (wall_ghost).
enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_DIRICHLET = 2, BC_OPEN = 3, BC_MARSHAK = 4, BC_REFLECT = 5 };

// Faces whose ghost is not the boundary cell's own state: they correct the flux of the
// self-mapped neighbour (Dirichlet data and the open, Marshak and reflecting walls).
__host__ __device__ __forceinline__ constexpr bool ghost_face(int kind) { return kind >= BC_DIRICHLET; }

// Geometry and constants of one uniform grid.
struct Grid {
    int nx, ny, nz;
    long long N;      // cells
    int bclo[3];      // boundary kind of the low face of each axis
    int bchi[3];      // ... and of the high face
    double nu;        // c dt / h
    double cdt;       // c dt  (s = c dt rho kappa)
    double tau_k;     // tau_cell = tau_k * sR^2 / f_dd  with tau_k = 50 / nu^2
    double c, aR, cv;
    int cv_cubic;     // 0: E_int = alpha T; 1: C_v = alpha T^3, E_int = alpha T^4 / 4 (alpha = rho cv)
    double finc8[6];  // Marshak faces (-x,+x,-y,+y,-z,+z): 8 F_inc / c, the ghost's affine part
    double eps_N;     // relative tolerance of the per-cell Newton solve (0: to round-off)
    // Dirichlet faces (-x,+x,-y,+y,-z,+z): the ghost cells' E and F (physical), 4 planes of the
    // face's cells -- x faces [nz][ny], y faces [nz][nx], z faces [ny][nx]; null elsewhere
    const double *ghost[6];
};

// Cells on face d of a grid, and the index on that face of the cell with in-plane offset o
// (o = i + nx j) on plane k.
__host__ __device__ __forceinline__ long long face_area(const Grid &g, int d)
{
    return d == 0 ? (long long)g.ny * g.nz : (d == 1 ? (long long)g.nx * g.nz : (long long)g.nx * g.ny);
}
__device__ __forceinline__ long long face_index(const Grid &g, int d, int k, unsigned o)
{
    const unsigned j = o / (unsigned)g.nx, i = o - j * (unsigned)g.nx;
    return d == 0 ? (long long)k * g.ny + j : (d == 1 ? (long long)k * g.nx + i : (long long)j * g.nx + i);
}

// Kind of the wall on side `side` of axis d (periodic faces are no walls).
__host__ __device__ __forceinline__ int wall_kind(const Grid &g, int d, int side)
{
    return side ? g.bchi[d] : g.bclo[d];
}

// row d of the symmetric tensor in the (xx,yy,zz,xy,xz,yz) plane order: f_d0, f_d1, f_d2
__host__ __device__ __forceinline__ constexpr int tens_row(int d, int j)
{
    return d == j ? d : ((d + j) == 1 ? 3 : ((d + j) == 2 ? 4 : 5));
}

__device__ __forceinline__ float xexpm1(float x) { return expm1f(x); }
__device__ __forceinline__ double xexpm1(double x) { return expm1(x); }
__device__ __forceinline__ float xsqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double xsqrt(double x) { return sqrt(x); }

// Optical-depth parameter of the wave-speed correction for one cell along one
// axis, tau = (10 h rho kappa_R)^2 / (2 f_dd) = tau_k sR^2 / f_dd.
// No opacity: tau = 0.  Zero diagonal factor with opacity: tau = +inf.
template <class T>
__device__ __forceinline__ T cell_tau(T sR, T fdd, T tau_k)
{
    if (sR == T(0)) return T(0);
    if (fdd == T(0)) return T(INFINITY);
    return tau_k * sR * sR / fdd;
}

// Corrected HLLE signal speed divided by c at a face between two cells:
// sqrt(max f_dd) * sqrt((1 - exp(-tau)) / tau) with tau the mean of the cells' values.
template <class T>
__device__ __forceinline__ T face_speed(T fL, T fR, T sRL, T sRR, T tau_k)
{
    T tau = T(0.5) * (cell_tau(sRL, fL, tau_k) + cell_tau(sRR, fR, tau_k));
    T fc = fL > fR ? fL : fR;
    T corr;
    if (tau == T(0))
        corr = T(1);
    else if (isinf(tau))
        corr = T(0);
    else
        corr = xsqrt(-xexpm1(-tau) / tau);
    return xsqrt(fc) * corr;
}

// Cell (i,j,k) from a linear index (x fastest).
__device__ __forceinline__ void cell_ijk(const Grid &g, long long c, int &i, int &j, int &k)
{
    long long q = c / g.nx;
    i = (int)(c - q * g.nx);
    k = (int)(q / g.ny);
    j = (int)(q - (long long)k * g.ny);
}

// Linear index of the neighbour across face (d, side) of cell c = (i,j,k):
// periodic faces wrap, every other wall returns the cell itself (see wall_ghost).
__device__ __forceinline__ long long neighbour(const Grid &g, int i, int j, int k, long long c, int d, int side)
{
    int q = d == 0 ? i : (d == 1 ? j : k);
    int n = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
    long long stride = d == 0 ? 1LL : (d == 1 ? (long long)g.nx : (long long)g.nx * g.ny);
    if (side) {
        if (q + 1 < n) return c + stride;
        return g.bchi[d] == BC_PERIODIC ? c - (long long)(n - 1) * stride : c;
    }
    if (q > 0) return c - stride;
    return g.bclo[d] == BC_PERIODIC ? c + (long long)(n - 1) * stride : c;
}

// Ghost state across a face of kind Dirichlet, open, Marshak or reflect, in the
// scaled variables (E, Ft = F / c); (Eo, Fo, e8) are the affine data (Dirichlet:
// the ghost's given state; open: the old state at the cell; Marshak: 8 F_inc / c),
// all zero for the linear operator.  With s = +1 at a low face and -1 at a high
// one (the sign of the incoming direction along d):
//   Dirichlet: (Eo, Fo) itself;
//   open:    the cell's state with the amplitude of the incoming characteristic
//            of the d-flux, (E + s Ft_d / sqrt(f_dd)) / 2 (speed c sqrt(f_dd)),
//            replaced by its old value along the eigenvector
//            (1, s f_d. / sqrt(f_dd)); no wave along d (f_dd = 0): the cell;
//   Marshak: Ft_g = Ft, E_g = 8 F_inc / c - 4 s Ft_d - E, i.e. c E + 2 s F_d =
//            4 F_inc for the means of ghost and cell (Sec. 3.4);
//   reflect: E_g = E, Ft_g = Ft with Ft_d negated, tensor row with f_dj
//            (j != d) negated.
// The ghost's own tensor row is the cell's otherwise; its corrected speed is
// the cell's own (both cells have the same f_dd and sR): the ghost's
// coefficients are the boundary cell's, Dirichlet faces included.
template <class T>
__device__ __forceinline__ void wall_ghost(int kind, int d, int side, T Ec, const T (&Fc)[3], const T (&fcr)[3],
                                           T Eo, const T (&Fo)[3], T e8, T &Eg, T (&Fg)[3], T (&fg)[3])
{
    // d and kind may be run-time values (divergent among lanes): components and kinds are
    // selected, never indexed or branched on
    const T s = side ? T(-1) : T(1);
    const T fdd = d == 0 ? fcr[0] : (d == 1 ? fcr[1] : fcr[2]);
    const T Fcd = d == 0 ? Fc[0] : (d == 1 ? Fc[1] : Fc[2]);
    const T Fod = d == 0 ? Fo[0] : (d == 1 ? Fo[1] : Fo[2]);
    const bool op = kind == BC_OPEN && fdd > T(0), ms = kind == BC_MARSHAK, rf = kind == BC_REFLECT;
    const bool dr = kind == BC_DIRICHLET;
    const T ia = op ? T(1) / xsqrt(fdd) : T(0);
    const T delta = op ? T(0.5) * ((Eo + s * Fod * ia) - (Ec + s * Fcd * ia)) : T(0);
    const T Em = e8 - T(4) * s * Fcd - Ec;
    Eg = dr ? Eo : (ms ? Em : Ec + delta);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T Fj = Fc[j] + delta * s * fcr[j] * ia;
        Fg[j] = dr ? Fo[j] : ((rf && j == d) ? -Fc[j] : Fj);
        fg[j] = (rf && j != d) ? -fcr[j] : fcr[j];
    }
}

// The ghost face's share of the Jacobi diagonal (the derivative of its flux
// contribution with respect to the cell's own unknowns, to be multiplied by
// nu): open: (sqrt(f_dd) + C)/4 in the E and F_d rows; Marshak: C in the E row,
// 2 f_dd in the F_d row; reflect: C in the F_d row; Dirichlet (the ghost does not
// follow the cell): C/2 in every row, as a face between two cells.  The other
// rows get nothing from a wall (their ghost values follow the cell's one to
// one).  qE, qF, qX: the shares of the E row, of the F_d row and of each F_j
// row with j != d.
template <class T>
__device__ __forceinline__ void wall_diag_q(int kind, int d, const T (&fcr)[3], T C, T &qE, T &qF, T &qX)
{
    const T fdd = d == 0 ? fcr[0] : (d == 1 ? fcr[1] : fcr[2]);
    const bool op = kind == BC_OPEN && fdd > T(0), dr = kind == BC_DIRICHLET;
    const T qo = T(0.25) * (xsqrt(op ? fdd : T(0)) + C);
    qE = dr ? T(0.5) * C : (op ? qo : (kind == BC_MARSHAK ? C : T(0)));
    qF = dr ? T(0.5) * C : (op ? qo : (kind == BC_MARSHAK ? T(2) * fdd : (kind == BC_REFLECT ? C : T(0))));
    qX = dr ? T(0.5) * C : T(0);
}

// face_speed of a face between a cell and itself (a wall's speed), without branches; the same
// operations, so the same value.
template <class T>
__device__ __forceinline__ T self_face_speed(T fdd, T sR, T tau_k)
{
    T t = tau_k * sR * sR / fdd;
    t = fdd == T(0) ? T(INFINITY) : t;
    t = sR == T(0) ? T(0) : t;
    const T tau = T(0.5) * (t + t);
    const T r = xsqrt(-xexpm1(-tau) / tau);
    const T corr = tau == T(0) ? T(1) : (isinf(tau) ? T(0) : r);
    return xsqrt(fdd) * corr;
}

// Accumulate the HLLE flux of the face on side `side` (0: low, 1: high) along
// axis d into the divergence sums dE, dF of the centre cell.  c* are the
// centre's state (E, Ft) and tensor row d, n* the neighbour's; C the face speed.
template <class T>
__device__ __forceinline__ void face_flux_acc(int d, int side, T C, T Ec, const T (&Fc)[3], const T (&fcr)[3], T En,
                                              const T (&Fn)[3], const T (&fnr)[3], T &dE, T (&dF)[3])
{
    const T EL = side ? Ec : En, ER = side ? En : Ec;
    const T *FL_ = side ? Fc : Fn;
    const T *FR_ = side ? Fn : Fc;
    const T *fL = side ? fcr : fnr;
    const T *fR = side ? fnr : fcr;
    const T sgn = side ? T(1) : T(-1);
    const T phiE = T(0.5) * (FL_[d] + FR_[d]) - T(0.5) * C * (ER - EL);
    dE += sgn * phiE;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const T phiF = T(0.5) * (fL[q] * EL + fR[q] * ER) - T(0.5) * C * (FR_[q] - FL_[q]);
        dF[q] += sgn * phiF;
    }
}

// Transport part of the operator at one cell of a uniform grid.  `ld(q, idx)`
// returns component q (0: E, 1..3: Ft) of the operand at cell idx; `fl(t, idx)`
// the tensor plane t; `sr(idx)` the cell's sR.  Returns nu * div(Phi) in
// div[4], the sum of Ct over faces that carry dissipation (every face but a
// zero-gradient wall; the transport part of the Jacobi diagonal is 0.5 nu
// times that) and over all six faces.  Eo, Fo: the cell's old state and
// `affine` whether the walls take their data (the nonlinear residual) or not
// (the linear operator).
template <class T, class LD, class FL, class SR>
__device__ __forceinline__ void transport(const Grid &g, int i, int j, int k, long long c, LD ld, FL fl, SR sr,
                                          T div[4], T &sumC_nb, T &sumC_all, bool affine = false, T Eo = T(0),
                                          const T (&Fo)[3] = {T(0), T(0), T(0)})
{
    const T tk = (T)g.tau_k;
    const T Ec = ld(0, c);
    const T Fc[3] = {ld(1, c), ld(2, c), ld(3, c)};
    const T sRc = sr(c);
    T dE = 0, dF[3] = {0, 0, 0};
    sumC_nb = 0;
    sumC_all = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T fcr[3] = {fl(tens_row(d, 0), c), fl(tens_row(d, 1), c), fl(tens_row(d, 2), c)};
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const long long nb = neighbour(g, i, j, k, c, d, side);
            T En = ld(0, nb);
            T Fn[3] = {ld(1, nb), ld(2, nb), ld(3, nb)};
            T fnr[3] = {fl(tens_row(d, 0), nb), fl(tens_row(d, 1), nb), fl(tens_row(d, 2), nb)};
            const T C = face_speed<T>(fcr[d], fnr[d], sRc, sr(nb), tk);
            const int wk = nb == c ? wall_kind(g, d, side) : BC_PERIODIC;
            if (ghost_face(wk)) {
                T Ea = affine ? Eo : T(0), Fa[3] = {affine ? Fo[0] : T(0), affine ? Fo[1] : T(0),
                                                    affine ? Fo[2] : T(0)};
                if (affine && wk == BC_DIRICHLET) {   // the face's data at the cell's place on it
                    const double *gd = g.ghost[2 * d + side];
                    const long long fi = face_index(g, d, k, (unsigned)(i + (long long)g.nx * j)),
                                    ar = face_area(g, d);
                    Ea = (T)gd[fi];
#pragma unroll
                    for (int q = 0; q < 3; ++q) Fa[q] = (T)(gd[(1 + q) * ar + fi] / g.c);
                }
                wall_ghost<T>(wk, d, side, Ec, Fc, fcr, Ea, Fa,
                              affine && wk == BC_MARSHAK ? (T)g.finc8[2 * d + side] : T(0), En, Fn, fnr);
            }
            sumC_all += C;
            if (nb != c) sumC_nb += C;
            face_flux_acc<T>(d, side, C, Ec, Fc, fcr, En, Fn, fnr, dE, dF);
        }
    }
    const T nu = (T)g.nu;
    div[0] = nu * dE;
    div[1] = nu * dF[0];
    div[2] = nu * dF[1];
    div[3] = nu * dF[2];
}

// Gas temperature of eq. PicardTemp at one cell: the T >= 0 with
// alpha (T - Tn) + sP (aR T^4 - E) = 0.  The function is increasing and convex
// for T >= 0, so Newton's method (analytic derivative) started above the root,
// at the smaller of the two one-term bounds, descends monotonically and stops
// at round-off when an iterate no longer decreases.  With no non-negative root
// (alpha Tn + sP E <= 0) it returns 0 and sets neg.
__device__ __forceinline__ double exchange_T(double alpha, double Tn, double sP, double aR, double E, bool &neg,
                                             double eps_N = 0.0)
{
    if (sP == 0.0) return Tn;
    const double rhs = alpha * Tn + sP * E;
    if (!(rhs > 0.0)) {
        neg = true;
        return 0.0;
    }
    // start above the root (smaller of the two one-term bounds); g is convex and
    // increasing so Newton descends monotonically; stop when it stops decreasing
    double T = sqrt(sqrt(rhs / (sP * aR)));
    if (alpha > 0.0 && rhs / alpha < T) T = rhs / alpha;
    for (int it = 0; it < 200; ++it) {
        const double T3 = T * T * T;
        const double gv = alpha * (T - Tn) + sP * (aR * T3 * T - E);
        const double dg = alpha + 4.0 * sP * aR * T3;
        const double Tnew = T - gv / dg;
        if (!(Tnew < T)) break;
        const bool done = eps_N > 0.0 && T - Tnew <= eps_N * Tnew;   // relative change below eps_N
        T = Tnew;
        if (done) break;
    }
    return T;
}


// Gas internal energy and heat capacity at T.
__device__ __forceinline__ double gas_e(const Grid &g, double alpha, double T)
{
    return g.cv_cubic ? 0.25 * alpha * T * T * T * T : alpha * T;
}
__device__ __forceinline__ double gas_C(const Grid &g, double alpha, double T)
{
    return g.cv_cubic ? alpha * T * T * T : alpha;
}

// Gas temperature of the exchange row with an extra energy X the gas receives:
// e(T) - e(Tn) + sP (aR T^4 - E) = X.  Constant capacity: exchange_T with T_n
// shifted by X / alpha (or E by X / sP without capacity).  Cubic capacity: the
// row is linear in T^4 and solved in closed form.  No non-negative root: 0, neg.
__device__ __forceinline__ double gas_exchange(const Grid &g, double alpha, double Tn, double sP, double aR, double E,
                                               double X, bool &neg)
{
    if (g.cv_cubic) {
        const double den = 0.25 * alpha + sP * aR;
        if (den == 0.0) return Tn;
        const double num = 0.25 * alpha * Tn * Tn * Tn * Tn + sP * E + X;
        if (!(num > 0.0)) {
            neg = true;
            return 0.0;
        }
        return sqrt(sqrt(num / den));
    }
    if (alpha > 0)
        Tn += X / alpha;
    else if (sP > 0)
        E += X / sP;
    return exchange_T(alpha, Tn, sP, aR, E, neg, g.eps_N);
}

// Right-hand side of the energy row with the emission and the gas energy
// linearised at T* and the gas energy eliminated (Newton on the T-eliminated
// system); eta = 4 sP aR T*^3 / (C(T*) + 4 sP aR T*^3).  E diagonal 1 + sP (1 - eta).
__device__ __forceinline__ double lin_rhs(const Grid &g, double En, double alpha, double Tn, double Ts, double sP,
                                          double aR, double &eta)
{
    const double T3 = Ts * Ts * Ts, T4 = T3 * Ts;
    const double den = gas_C(g, alpha, Ts) + 4.0 * sP * aR * T3;
    eta = den > 0 ? 4.0 * sP * aR * T3 / den : 0.0;
    if (!g.cv_cubic) return En + eta * alpha * Tn - 3.0 * (1.0 - eta) * sP * aR * T4;
    return En + (1.0 - eta) * sP * aR * T4 + eta * (gas_e(g, alpha, Tn) - gas_e(g, alpha, Ts));
}

// Four consecutive elements of a Krylov vector, loaded/stored as one 16-byte
// (FP32) or two 16-byte (FP64) vector accesses and widened to FP64.
template <class KT>
struct Quad;
template <>
struct Quad<float> {
    static __device__ __forceinline__ void load_raw(const float *p, float (&v)[4])
    {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
    static __device__ __forceinline__ void load(const float *p, double (&v)[4])
    {
        const float4 q = *reinterpret_cast<const float4 *>(p);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    }
    static __device__ __forceinline__ void store(float *p, const double (&v)[4], double (&r)[4])
    {
        float4 q;
        q.x = (float)v[0]; q.y = (float)v[1]; q.z = (float)v[2]; q.w = (float)v[3];
        *reinterpret_cast<float4 *>(p) = q;
        r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
    }
};
template <>
struct Quad<double> {
    static __device__ __forceinline__ void load_raw(const double *p, double (&v)[4]) { load(p, v); }
    static __device__ __forceinline__ void load(const double *p, double (&v)[4])
    {
        const double2 a = *reinterpret_cast<const double2 *>(p), b = *reinterpret_cast<const double2 *>(p + 2);
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    static __device__ __forceinline__ void store(double *p, const double (&v)[4], double (&r)[4])
    {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2 *>(p + 2) = make_double2(v[2], v[3]);
        for (int k = 0; k < 4; ++k) r[k] = v[k];
    }
};

// ------------------------------------------------------------------ reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

// Sum NV per-thread values over the workgroup (NT threads, 1D) and store
// them at partials[slot * NV + q]; the last NMX columns take the maximum
// instead of the sum.  Fixed order: reruns are bitwise identical.
template <int NV, int NT = kBlock, int NMX = 0>
__device__ __forceinline__ void block_store(double (&v)[NV], double *partials, long long slot)
{
    __shared__ double sh[NV][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = q >= NV - NMX ? wave_max(v[q]) : wave_sum(v[q]);
        if (lane == 0) sh[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const bool mx = (int)threadIdx.x >= NV - NMX;
        double s = mx ? sh[threadIdx.x][0] : 0.0;
#pragma unroll
        for (int w = mx ? 1 : 0; w < NT / 64; ++w) s = mx ? fmax(s, sh[threadIdx.x][w]) : s + sh[threadIdx.x][w];
        partials[slot * NV + threadIdx.x] = s;
    }
}

}  // namespace vr
