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

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_DIRICHLET = 2 };

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
};

// row d of the symmetric tensor in the (xx,yy,zz,xy,xz,yz) plane order: f_d0, f_d1, f_d2
__host__ __device__ constexpr int tens_row(int d, int j)
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
// periodic faces wrap, outflow faces return the cell itself (zero-gradient ghost).
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
// div[4], the sum of Ct over faces whose neighbour is another cell (the
// transport part's diagonal is 0.5 nu times that) and over all six faces.
template <class T, class LD, class FL, class SR>
__device__ __forceinline__ void transport(const Grid &g, int i, int j, int k, long long c, LD ld, FL fl, SR sr,
                                          T div[4], T &sumC_nb, T &sumC_all)
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
            const T En = ld(0, nb);
            const T Fn[3] = {ld(1, nb), ld(2, nb), ld(3, nb)};
            const T fnr[3] = {fl(tens_row(d, 0), nb), fl(tens_row(d, 1), nb), fl(tens_row(d, 2), nb)};
            const T C = face_speed<T>(fcr[d], fnr[d], sRc, sr(nb), tk);
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
__device__ __forceinline__ double exchange_T(double alpha, double Tn, double sP, double aR, double E, bool &neg)
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
        T = Tnew;
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
    return exchange_T(alpha, Tn, sP, aR, E, neg);
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

// Sum NV per-thread values over the workgroup (NT threads, 1D) and store
// them at partials[slot * NV + q].  Fixed order: reruns are bitwise identical.
template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_store(double (&v)[NV], double *partials, long long slot)
{
    __shared__ double sh[NV][NT / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) sh[q][wid] = s;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += sh[threadIdx.x][w];
        partials[slot * NV + threadIdx.x] = s;
    }
}

}  // namespace vr
