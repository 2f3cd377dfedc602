// rad_single.hip -- one implicit radiation step on a uniform grid (gfx950).
//
// Host-driven Picard loop (Sec. 2.3.1 steps iv-vi):
//   residual   r = b(T*) - A(T*) X  in FP64 for the linear system of the current
//              iteration; its scaled norm is also the nonlinear residual
//   Krylov     restarted GMRES(m) on the Jacobi-scaled system B, right-multiplied
//              by the Neumann polynomial 2I - B by default (Arnoldi on 2B - B^2:
//              half the iterations, so half the orthogonalisation traffic, for
//              the same applies of B) or by one multigrid V-cycle of
//              re-discretised coarse levels, Arnoldi in FP32 (mixed) or FP64,
//              solution accumulated into the FP64 state; each restart
//              re-evaluates the FP64 residual (iterative refinement)
//   exchange   per-cell FP64 Newton solve of eq. PicardTemp for T
// Every vector operation and reduction runs in the kernels below; the host
// only keeps the (m+1) x m Hessenberg matrix and decides when to stop.
#include "rad_host.h"
#include "rad_apply_tiled.h"
#include "rad_amr.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

using namespace vr;

namespace {

// --------------------------------------------------------------- kernels

// Coefficient setup, once per step: sR in the apply precision, an FP32 copy of
// the tensor when the Krylov arithmetic is FP32 but the input is FP64, the
// FP64 state X = (E, F/c), its copy X0 and T* = T_n; counts invalid cells.
template <class CT, class AT>
__global__ void __launch_bounds__(kBlock) k_setup(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kP,
                                                  const CT *__restrict__ kR, const CT *__restrict__ f, AT *__restrict__ sR,
                                                  double *__restrict__ sR64, AT *__restrict__ fA,
                                                  const double *__restrict__ E,
                                                  const double *__restrict__ F, const double *__restrict__ T,
                                                  double *__restrict__ X, double *__restrict__ X0,
                                                  double *__restrict__ Tc, double *partials)
{
    const long long N = g.N;
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0};
    if (c < N) {
        double r = (double)rho[c], p = (double)kP[c], s = (double)kR[c];
        sR[c] = (AT)(g.cdt * r * s);
        if (sR64) sR64[c] = g.cdt * r * s;
        bool bad = !(r >= 0) || !(p >= 0) || !(s >= 0) || !isfinite(r) || !isfinite(p) || !isfinite(s);
        for (int t = 0; t < 6; ++t) {
            double ft = (double)f[t * N + c];
            if (!isfinite(ft) || (t < 3 && ft < 0)) bad = true;
            if (fA) fA[t * N + c] = (AT)ft;
        }
        v[0] = bad ? 1.0 : 0.0;
        double inv_c = 1.0 / g.c;
        X[c] = X0[c] = E[c];
        for (int q = 0; q < 3; ++q) X[(1 + q) * N + c] = X0[(1 + q) * N + c] = F[q * N + c] * inv_c;
        Tc[c] = T[c];
    }
    block_store<1>(v, partials, blockIdx.x);
}

enum { RES_KRYLOV = 0, RES_PHYSICAL = 1 };

// FP64 residual of the linear system of one Picard iteration at the state X,
// with the emission taken at Ts (lagged: paper; linearised: Newton-consistent).
// RES_KRYLOV: writes D^-1 r (Jacobi-scaled, Krylov precision) into out, the E
// diagonal in the apply precision into dEA, and partial sums
//   [sum (rE/WE)^2, sum (rF/WF)^2, sum E^2, sum Ft^2, sum (D^-1 r)^2].
// RES_PHYSICAL: writes the nonlinear residual (R_E, R_F (physical), R_T) of
// the state (X = E, F physical, Ts = T) into outR (5 planes).
template <class CT, class KT, class AT, int MODE>
__global__ void __launch_bounds__(kBlock)
    k_residual(Grid g, int picard_mode, const double *__restrict__ En, const double *__restrict__ Fn,
               const double *__restrict__ Tn, const double *__restrict__ Ts, const CT *__restrict__ rho,
               const CT *__restrict__ kP, const CT *__restrict__ kR, const CT *__restrict__ f,
               const double *__restrict__ XE, const double *__restrict__ XF, double xF, KT *__restrict__ out,
               AT *__restrict__ dEA, double *__restrict__ outR, double *partials)
{
    const long long N = g.N;
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (c < N) {
        int i, j, k;
        cell_ijk(g, c, i, j, k);
        const double cdt = g.cdt;
        auto ld = [&](int q, long long idx) -> double { return q == 0 ? XE[idx] : xF * XF[(q - 1) * N + idx]; };
        auto fl = [&](int t, long long idx) -> double { return (double)f[t * N + idx]; };
        auto sr = [&](long long idx) -> double { return cdt * (double)rho[idx] * (double)kR[idx]; };
        double div[4], sC_nb, sC_all;
        const double Fo[3] = {Fn[c] / g.c, Fn[N + c] / g.c, Fn[2 * N + c] / g.c};
        transport<double>(g, i, j, k, c, ld, fl, sr, div, sC_nb, sC_all, true, En[c], Fo);

        const double r_ = (double)rho[c];
        const double sP = cdt * r_ * (double)kP[c], sR = sr(c), alpha = r_ * g.cv, aR = g.aR;
        const double T = Ts[c], T3 = T * T * T, T4 = T3 * T;
        double dE, bE;
        if (picard_mode == 0) {
            dE = 1.0 + sP;
            bE = En[c] + sP * aR * T4;
        } else {
            double eta;
            bE = lin_rhs(g, En[c], alpha, Tn[c], T, sP, aR, eta);
            dE = 1.0 + sP * (1.0 - eta);
        }
        const double E = ld(0, c);
        const double rE = bE - (dE * E + div[0]);
        const double invc = 1.0 / g.c;
        double rF[3];
        for (int q = 0; q < 3; ++q) rF[q] = Fn[q * N + c] * invc - ((1.0 + sR) * ld(1 + q, c) + div[1 + q]);
        if (MODE == RES_PHYSICAL) {
            outR[c] = -rE;
            for (int q = 0; q < 3; ++q) outR[(1 + q) * N + c] = -rF[q] * g.c;
            outR[4 * N + c] = gas_e(g, alpha, T) - gas_e(g, alpha, Tn[c]) + sP * (aR * T4 - E);
        } else {
            const double half = 0.5 * g.nu;
            const double DE = dE + half * sC_nb, DF = 1.0 + sR + half * sC_nb;
            const double WE = 1.0 + sP + half * sC_all, WF = 1.0 + sR + half * sC_all;
            const double zE = rE / DE;
            out[c] = (KT)zE;
            dEA[c] = (AT)dE;
            double zz = zE * zE, wf = 0, fn = 0;
            for (int q = 0; q < 3; ++q) {
                const double z = rF[q] / DF;
                out[(1 + q) * N + c] = (KT)z;
                zz += z * z;
                wf += (rF[q] / WF) * (rF[q] / WF);
                const double Fq = ld(1 + q, c);
                fn += Fq * Fq;
            }
            v[0] = (rE / WE) * (rE / WE);
            v[1] = wf;
            v[2] = E * E;
            v[3] = fn;
            v[4] = zz;
        }
    }
    if (MODE == RES_KRYLOV) block_store<5>(v, partials, blockIdx.x);
}

// The RES_KRYLOV residual of k_residual as a tile sweep: FP64 state, stored
// coefficients, and the face speeds and sR precomputed in FP64 once per step
// (the same values k_residual derives per face).  Partial sums per tile.
// AMR: one level of the two-level composite grid (covered coarse cells keep
// their local terms only, jump cells add their level-jump corrections).
// VEL (moving medium): 1 adds the O(v/c) terms (coefficients VA, VB, VC of
// k_vel_coef) to the radiation rows; 2 (implicit switch) with the linearised
// emission keeps the fraction 1 - eta of the energy row's O(v/c) terms (the gas
// energy eliminated, as for the emission) and writes that row's coupling to Ft
// for the Krylov apply (vbw).
template <class CT, class KT, class DT, bool AMR = false, int VEL = 0, int WL = 0>
__global__ void __launch_bounds__(tile_threads<double>())
    k_residual_tiled(Grid g, TileGeom tg, int picard_mode, const double *__restrict__ En,
                     const double *__restrict__ Fn, const double *__restrict__ Tn, const double *__restrict__ Ts,
                     const CT *__restrict__ rho, const CT *__restrict__ kP, const CT *__restrict__ f,
                     const double *__restrict__ sR64, const double *__restrict__ Cf64, const double *__restrict__ X,
                     KT *__restrict__ out, DT *__restrict__ dEA, double *partials, AmrLv al = AmrLv{},
                     const double *__restrict__ VA = nullptr, const double *__restrict__ VB = nullptr,
                     const double *__restrict__ VC = nullptr, DT *__restrict__ vbw = nullptr,
                     const double *__restrict__ cw = nullptr)
{
    __shared__ double lds[2][Rec<true>::NL][TileShape<double>::LY][kLX];
    const long long N = g.N;
    const long long plane = (long long)g.nx * g.ny;
    const double invc = 1.0 / g.c, nu = g.nu, half = 0.5 * g.nu, aR = g.aR, cdt = g.cdt, cv = g.cv;
    double acc[5] = {0, 0, 0, 0, 0};
    constexpr int NEX = 8 + (VEL ? 7 : 0);
    auto lex = [&](int, long long pb, unsigned o, double(&e)[NEX]) __attribute__((always_inline)) {
        e[0] = ld_off(En + pb, o);
        for (int q = 0; q < 3; ++q) e[1 + q] = ld_off(Fn + q * N + pb, o);
        e[4] = ld_off(Tn + pb, o);
        e[5] = ld_off(Ts + pb, o);
        e[6] = (double)ld_off(rho + pb, o);
        e[7] = (double)ld_off(kP + pb, o);
        if constexpr (VEL) {
            e[8] = ld_off(VA + pb, o);
            for (int q = 0; q < 3; ++q) e[9 + q] = ld_off(VB + q * N + pb, o);
            for (int q = 0; q < 3; ++q) e[12 + q] = ld_off(VC + q * N + pb, o);
        }
    };
    auto epi = [&](int k, int, unsigned o, bool active, const CellSums<double> &S, const double(&e)[NEX])
                   __attribute__((always_inline)) {
        const long long pb = plane * k;
        const double r_ = e[6];
        const double sP = cdt * r_ * e[7], sR = S.sc, alpha = r_ * cv;
        const double T = e[5], T3 = T * T * T, T4 = T3 * T;
        double dE, bE;
        if (picard_mode == 0) {
            dE = 1.0 + sP;
            bE = e[0] + sP * aR * T4;
        } else {
            double eta;
            bE = lin_rhs(g, e[0], alpha, e[4], T, sP, aR, eta);
            dE = 1.0 + sP * (1.0 - eta);
        }
        const double E = S.Ec;
        double divE = nu * S.dEs, divF[3] = {nu * S.dF[0], nu * S.dF[1], nu * S.dF[2]};
        double vf = 1.0;   // factor of the energy row's O(v/c) terms
        if constexpr (VEL) {   // O(v/c) terms: local couplings, the E one joins the diagonal
            if constexpr (VEL == 2)
                if (picard_mode != 0)
                    vf = 1.0 - 4.0 * sP * aR * T3 / fmax(gas_C(g, alpha, T) + 4.0 * sP * aR * T3, 1e-300);
            dE += vf * e[8];
            for (int q = 0; q < 3; ++q) {
                divE += vf * e[9 + q] * S.Fc[q];
                divF[q] += e[12 + q] * E;
            }
        }
        double dtr = half * S.sumC_nb;   // transport part of the Jacobi diagonal
        if constexpr (AMR) {
            const int jj = (int)(o / (unsigned)g.nx), ii = (int)(o - (unsigned)jj * (unsigned)g.nx);
            const int role = amr_role(al, ii, jj, k);
            if (role == AMR_COVERED) {
                divE = divF[0] = divF[1] = divF[2] = 0.0;
                dtr = 0.0;
            } else if (role == AMR_JUMP) {
                const long long c = pb + o;
                const double *corr = (const double *)al.corr;
                divE += corr[c];
                for (int q = 0; q < 3; ++q) divF[q] += corr[(1 + q) * N + c];
                dtr += corr[4 * N + c];
            }
        }
        const double rE = bE - (dE * E + divE);
        const double DE = dE + dtr + (WL ? nu * S.wE : 0.0), DF = 1.0 + sR + dtr;
        const double WE = 1.0 + sP + half * S.sumC_all, WF = 1.0 + sR + half * S.sumC_all;
        const double zE = rE / DE;
        double zF[3], zz = zE * zE, wf = 0, fn = 0;
        for (int q = 0; q < 3; ++q) {
            const double rF = e[1 + q] * invc - ((1.0 + sR) * S.Fc[q] + divF[q]);
            zF[q] = rF / (WL ? DF + nu * S.wF[q] : DF);
            zz += zF[q] * zF[q];
            wf += (rF / WF) * (rF / WF);
            fn += S.Fc[q] * S.Fc[q];
        }
        if (active) {
            st_off(out + pb, o, (KT)zE);
            for (int q = 0; q < 3; ++q) st_off(out + (1 + q) * N + pb, o, (KT)zF[q]);
            st_off(dEA + pb, o, (DT)dE);
            if constexpr (VEL == 2)
                for (int q = 0; q < 3; ++q) st_off(vbw + q * N + pb, o, (DT)(vf * e[9 + q]));
            acc[0] += (rE / WE) * (rE / WE);
            acc[1] += wf;
            acc[2] += E * E;
            acc[3] += fn;
            acc[4] += zz;
        }
    };
    // the ghosts with their data: a Dirichlet face's given state at the cell's place on the face,
    // the old state (E_n, F_n / c) of an open wall and 8 F_inc / c
    auto wall = [&](int kind, int d, int side, double Ec, const double(&Fc)[3], const double(&fcr)[3],
                    const double(&e)[NEX], unsigned fi, double &En_, double(&Fn_)[3], double(&fnr)[3])
                    __attribute__((always_inline)) {
        double Eo = e[0], Fo[3] = {e[1] * invc, e[2] * invc, e[3] * invc};
        if (kind == BC_DIRICHLET) {   // (kind, d and side are constants here; 32 fi < 2^31 checked on the host)
            const double *gd = g.ghost[2 * d + side];
            const long long ar = face_area(g, d);
            Eo = ld_off(gd, fi);
            for (int q = 0; q < 3; ++q) Fo[q] = ld_off(gd + (1 + q) * ar, fi) * invc;
        }
        wall_ghost<double>(kind, d, side, Ec, Fc, fcr, Eo, Fo, g.finc8[2 * d + side], En_, Fn_, fnr);
    };
    tile_sweep<double, CT, true, true, NEX, true, WL>(g, tg, f, sR64, (const CT *)nullptr, (const CT *)nullptr, Cf64,
                                                      X, 1.0, 1.0, lds, lex, epi, wall, MgFuse<double>{}, cw);
    block_store<5, tile_threads<double>()>(acc, partials, blockIdx.x);
}

// Raw dots <V_i, w> for i in [i0, i0+NV) and <w, w>, FP64 accumulation.  The
// vector count is a template parameter so all NV+1 loads of an element group
// are issued back to back.  n (= 4N) is a multiple of 4.
template <class KT, int NV>
__global__ void __launch_bounds__(kBlock)
    k_multidot(const KT *__restrict__ V, long long stride, int i0, const KT *__restrict__ w, long long n,
               double *partials)
{
    double acc[NV + 1];
#pragma unroll
    for (int q = 0; q <= NV; ++q) acc[q] = 0;
    const long long step = (long long)gridDim.x * kBlock * 4;
    const KT *Vb = V + (long long)i0 * stride;
    for (long long e = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; e < n; e += step) {
        double wv[4];
        Quad<KT>::load(w + e, wv);
        double vv[NV][4];
#pragma unroll
        for (int q = 0; q < NV; ++q) Quad<KT>::load(Vb + (long long)q * stride + e, vv[q]);
#pragma unroll
        for (int q = 0; q < NV; ++q) acc[q] += vv[q][0] * wv[0] + vv[q][1] * wv[1] + vv[q][2] * wv[2] + vv[q][3] * wv[3];
        acc[NV] += wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2] + wv[3] * wv[3];
    }
    block_store<NV + 1>(acc, partials, blockIdx.x);
}

template <class KT, int NV>
void launch_multidot(int cnt, dim3 g, hipStream_t st, const KT *V, long long stride, int i0, const KT *w, long long n,
                     double *partials)
{
    if constexpr (NV > 1) {
        if (cnt < NV) return launch_multidot<KT, NV - 1>(cnt, g, st, V, stride, i0, w, n, partials);
    }
    hipLaunchKernelGGL((k_multidot<KT, NV>), g, dim3(kBlock), 0, st, V, stride, i0, w, n, partials);
}

// out = w - sum_i s_i^2 d_i V_i  (i < cnt), accumulating ||out||^2 of the stored
// (rounded) values.  out may alias w.  The basis is consumed in fully unrolled
// chunks of 16 vectors; indices past cnt are clamped to cnt-1 with a zero
// coefficient, so all loads of a chunk issue back to back.
template <class KT, int CH>
__global__ void __launch_bounds__(kBlock)
    k_orth_update(const KT *__restrict__ V, long long stride, int cnt, const KT *w, KT *out,
                  const double *__restrict__ dots, const double *__restrict__ s, long long n, double *partials)
{
    __shared__ double cf[kMaxM + CH];
    for (int t = threadIdx.x; t < kMaxM + CH; t += kBlock)
        cf[t] = t < cnt ? s[t] * s[t] * dots[t] : 0.0;
    __syncthreads();
    double acc[1] = {0};
    const long long step = (long long)gridDim.x * kBlock * 4;
    for (long long e = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; e < n; e += step) {
        double val[4];
        Quad<KT>::load(w + e, val);
        for (int i0 = 0; i0 < cnt; i0 += CH) {
            double a[CH][4];
#pragma unroll
            for (int u = 0; u < CH; ++u) Quad<KT>::load(V + (long long)min(i0 + u, cnt - 1) * stride + e, a[u]);
#pragma unroll
            for (int u = 0; u < CH; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k) val[k] -= cf[i0 + u] * a[u][k];
        }
        double r[4];
        Quad<KT>::store(out + e, val, r);
        acc[0] += r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
    }
    block_store<1>(acc, partials, blockIdx.x);
}

// chunk width by basis size: small counts do not pay for a 16-wide chunk
template <class KT>
void launch_orth_update(int cnt, dim3 g, hipStream_t st, const KT *V, long long stride, const KT *w, KT *out,
                        const double *dots, const double *s, long long n, double *partials)
{
    if (cnt <= 4)
        hipLaunchKernelGGL((k_orth_update<KT, 4>), g, dim3(kBlock), 0, st, V, stride, cnt, w, out, dots, s, n, partials);
    else if (cnt <= 8)
        hipLaunchKernelGGL((k_orth_update<KT, 8>), g, dim3(kBlock), 0, st, V, stride, cnt, w, out, dots, s, n, partials);
    else
        hipLaunchKernelGGL((k_orth_update<KT, 16>), g, dim3(kBlock), 0, st, V, stride, cnt, w, out, dots, s, n,
                           partials);
}

// X += sum_i a_i V_i over the 4N-vector (FP64 state, Krylov-precision basis).
struct Coefs {
    double a[kMaxM + 1];
};

template <class KT>
__global__ void __launch_bounds__(kBlock)
    k_update_x(double *__restrict__ X, const KT *__restrict__ V, long long stride, int cnt, Coefs cf, long long n)
{
    const long long step = (long long)gridDim.x * kBlock * 4;
    for (long long e = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; e < n; e += step) {
        double acc[4], r[4];
        Quad<double>::load(X + e, acc);
        for (int i = 0; i < cnt; ++i) {
            double a[4];
            Quad<KT>::load(V + (long long)i * stride + e, a);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += cf.a[i] * a[k];
        }
        Quad<double>::store(X + e, acc, r);
    }
}

// z = sum_i a_i V_i over the 4N-vector, stored in the Krylov precision.
template <class KT>
__global__ void __launch_bounds__(kBlock)
    k_combine(KT *__restrict__ z, const KT *__restrict__ V, long long stride, int cnt, Coefs cf, long long n)
{
    const long long step = (long long)gridDim.x * kBlock * 4;
    for (long long e = ((long long)blockIdx.x * kBlock + threadIdx.x) * 4; e < n; e += step) {
        double acc[4] = {0, 0, 0, 0}, r[4];
        for (int i = 0; i < cnt; ++i) {
            double a[4];
            Quad<KT>::load(V + (long long)i * stride + e, a);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += cf.a[i] * a[k];
        }
        Quad<KT>::store(z + e, acc, r);
    }
}

// ---- multigrid cycle of the Krylov preconditioner (krylov_poly = 2).  Level l+1
// halves every extent of level l; a coarse cell's children are (2i+a, 2j+b, 2k+e).

__device__ __forceinline__ long long mg_child(const Grid &gf, int ic, int jc, int kc, int t)
{
    return (long long)(2 * ic + (t & 1)) + (long long)gf.nx * ((2 * jc + ((t >> 1) & 1)) +
                                                                 (long long)gf.ny * (2 * kc + (t >> 2)));
}

// dst (np planes of the coarse grid) = mean of the 8 children of src (np planes, stride sN)
template <class ST, class AT>
__global__ void __launch_bounds__(kBlock)
    k_mg_average(Grid gf, Grid gc, int np, const ST *__restrict__ src, long long sN, AT *__restrict__ dst)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= gc.N) return;
    int i, j, k;
    cell_ijk(gc, c, i, j, k);
    for (int q = 0; q < np; ++q) {
        double a = 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) a += (double)src[q * sN + mg_child(gf, i, j, k, t)];
        dst[q * gc.N + c] = (AT)(0.125 * a);
    }
}

// corrected low-face speeds of a coarse level from its sR and tensor (as k_face_coef)
template <class AT>
__global__ void __launch_bounds__(kBlock)
    k_mg_face(Grid g, const AT *__restrict__ sR, const AT *__restrict__ f, AT *__restrict__ Cf)
{
    const long long N = g.N;
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= N) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    for (int d = 0; d < 3; ++d) {
        const long long nb = neighbour(g, i, j, k, c, d, 0);
        Cf[d * N + c] = (AT)face_speed<double>((double)f[d * N + nb], (double)f[d * N + c], (double)sR[nb],
                                                (double)sR[c], g.tau_k);
    }
}

// coarse right-hand side of the scaled system: q_c = Dc^-1 mean_children(Df t)
template <class AT>
__global__ void __launch_bounds__(kBlock)
    k_mg_restrict(Grid gf, Grid gc, const AT *__restrict__ t, const AT *__restrict__ Df, const AT *__restrict__ Dc,
                  AT *__restrict__ q)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= gc.N) return;
    int i, j, k;
    cell_ijk(gc, c, i, j, k);
    const long long Nf = gf.N, Nc = gc.N;
    double a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const long long f = mg_child(gf, i, j, k, u);
        const double dE = (double)Df[f], dF = (double)Df[Nf + f];
        a[0] += dE * (double)t[f];
#pragma unroll
        for (int r = 1; r < 4; ++r) a[r] += dF * (double)t[r * Nf + f];
    }
    q[c] = (AT)(0.125 * a[0] / (double)Dc[c]);
    const double iF = 0.125 / (double)Dc[Nc + c];
#pragma unroll
    for (int r = 1; r < 4; ++r) q[r * Nc + c] = (AT)(a[r] * iF);
}

// e = qs q + (the coarse correction of the cell's parent)
template <class AT>
__global__ void __launch_bounds__(kBlock)
    k_mg_inject(Grid gf, Grid gc, const AT *__restrict__ q, AT qs, const AT *__restrict__ ec, AT *__restrict__ e)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= gf.N) return;
    int i, j, k;
    cell_ijk(gf, c, i, j, k);
    const long long pc = (long long)(i >> 1) + (long long)gc.nx * ((j >> 1) + (long long)gc.ny * (k >> 1));
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r * gf.N + c] = qs * q[r * gf.N + c] + ec[r * gc.N + pc];
}

// Per-cell exchange solve (eq. PicardTemp) for T with E = X_E; then the
// diagnostics of the Picard iteration, and X0 = X.  Partials:
//   [sum (R_T/W_T)^2, sum T^2, sum dT^2, sum dE^2, sum E^2, sum dFt^2, sum Ft^2, neg,
//    sum dt dE, sum (E_n + e(T_n)), max |dt dE| / (|E| + e(T))]
// with dt dE = sP (aR T^4 - e_rad) the energy correction of Sec. 2.3.4: the
// radiation row solved at the guess T_o (the T* it held) equals the plain row
// (1 + sP) E - E_n - sP e_rad with sP e_rad = sP eta E + b_E - E_n (eta = 0 and
// b_E = E_n + sP aR T_o^4 lagged).  Tfix (non-null): the gas temperature whose
// energy is e(T) + dt dE (clamped at 0), committed by the energy fix.
// VI (moving medium, implicit switch): the gas also receives the O(v/c) energy
// X = VA E + VB.Ft of the new state.
template <class CT, bool VI = false>
__global__ void __launch_bounds__(kBlock)
    k_exchange(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kP, const double *__restrict__ Tn,
               double *__restrict__ Tc, double *__restrict__ X, double *__restrict__ X0, double *partials,
               double *__restrict__ Gk, double *__restrict__ fk, const double *__restrict__ VA,
               const double *__restrict__ VB, const double *__restrict__ En, int picard_mode,
               double *__restrict__ Tfix)
{
    const long long N = g.N;
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (c < N) {
        const double r_ = (double)rho[c];
        const double sP = g.cdt * r_ * (double)kP[c], alpha = r_ * g.cv, aR = g.aR;
        const double E = X[c];
        bool neg = false;
        double Xv = 0.0;
        if constexpr (VI) {
            Xv = VA[c] * E;
            for (int q = 0; q < 3; ++q) Xv += VB[q * N + c] * X[(1 + q) * N + c];
        }
        const double T = gas_exchange(g, alpha, Tn[c], sP, aR, E, Xv, neg);
        const double T3 = T * T * T;
        // where no non-negative root exists T = 0 is the active bound (R_T > 0 there)
        const double RT0 = gas_e(g, alpha, T) - gas_e(g, alpha, Tn[c]) + sP * (aR * T3 * T - E) - Xv;
        const double RT = (T == 0.0 && RT0 > 0.0) ? 0.0 : RT0;
        const double WT = gas_C(g, alpha, T) + 4.0 * sP * aR * T3;
        const double To = Tc[c];
        const double dT = T - To;
        Tc[c] = T;
        // energy correction: the emission the radiation solve used against the gas root's
        double dEc = 0.0;
        if (sP != 0.0) {
            const double En_ = En[c];
            double eta = 0.0, bE;
            if (picard_mode == 0)
                bE = En_ + sP * aR * To * To * To * To;
            else
                bE = lin_rhs(g, En_, alpha, Tn[c], To, sP, aR, eta);
            dEc = sP * aR * T3 * T - (sP * eta * E + bE - En_);
        }
        const double eT = gas_e(g, alpha, T);
        v[8] = dEc;
        v[9] = En[c] + gas_e(g, alpha, Tn[c]);
        const double loc = fabs(E) + eT;
        v[10] = loc > 0.0 ? fabs(dEc) / loc : (dEc != 0.0 ? INFINITY : 0.0);
        if (Tfix) {
            const double e1 = eT + dEc;
            Tfix[c] = !(e1 > 0.0) || !(alpha > 0.0) ? 0.0
                      : (g.cv_cubic ? sqrt(sqrt(4.0 * e1 / alpha)) : e1 / alpha);
            if (dEc == 0.0) Tfix[c] = T;
        }
        if (Gk) {  // Picard map value and its residual for the Anderson history
            Gk[c] = T;
            fk[c] = dT;
        }
        v[0] = WT > 0 ? (RT / WT) * (RT / WT) : 0.0;
        v[1] = T * T;
        v[2] = dT * dT;
        const double dE = E - X0[c];
        v[3] = dE * dE;
        v[4] = E * E;
        X0[c] = E;
        for (int q = 1; q < 4; ++q) {
            const double x = X[q * N + c], d = x - X0[q * N + c];
            v[5] += d * d;
            v[6] += x * x;
            X0[q * N + c] = x;
        }
        v[7] = neg ? 1.0 : 0.0;
    }
    block_store<11, kBlock, 1>(v, partials, blockIdx.x);
}

// Moving medium, once per step: the O(v/c) coefficients of eq. G and G0 with
// beta = v/c (kappa_E = kappa_P, kappa_F = kappa_R), in FP64 and, for the
// Krylov apply, copies in its precision:
//   VA = (sP - sR)(b.b + b.f.b)   energy row, on E (joins the E diagonal)
//   VB = (sR - 2 sP) b            energy row, on Ft
//   VC = -sR (b + f b)            flux rows, on E
// Counts non-finite beta.
template <class CT, class AT>
__global__ void __launch_bounds__(kBlock)
    k_vel_coef(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kP, const CT *__restrict__ kR,
               const CT *__restrict__ f, const CT *__restrict__ beta, double *__restrict__ VA,
               double *__restrict__ VB, double *__restrict__ VC, AT *__restrict__ VBA, AT *__restrict__ VCA,
               double *partials)
{
    const long long N = g.N;
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double v[1] = {0};
    if (c < N) {
        const double r_ = (double)rho[c];
        const double sP = g.cdt * r_ * (double)kP[c], sR = g.cdt * r_ * (double)kR[c];
        double b[3], fb[3], bb = 0, bfb = 0;
        for (int q = 0; q < 3; ++q) b[q] = (double)beta[q * N + c];
        for (int a = 0; a < 3; ++a) {
            fb[a] = 0;
            for (int k = 0; k < 3; ++k) fb[a] += (double)f[tens_row(a, k) * N + c] * b[k];
        }
        for (int q = 0; q < 3; ++q) {
            bb += b[q] * b[q];
            bfb += b[q] * fb[q];
        }
        v[0] = (isfinite(b[0]) && isfinite(b[1]) && isfinite(b[2])) ? 0.0 : 1.0;
        const double va = (sP - sR) * (bb + bfb);
        VA[c] = va;
        for (int q = 0; q < 3; ++q) {
            const double vb = (sR - 2.0 * sP) * b[q], vc = -sR * (b[q] + fb[q]);
            VB[q * N + c] = vb;
            VC[q * N + c] = vc;
            VBA[q * N + c] = (AT)vb;
            VCA[q * N + c] = (AT)vc;
        }
    }
    block_store<1>(v, partials, blockIdx.x);
}

// Anderson acceleration of the Picard map T_* -> G(T_*) = T(E(T_*)) (the
// acceleration Sec. 4.3 names for the linearly convergent lagged iteration).
// History slots i < H hold past map values G_i and residuals f_i = G_i - T_*,i.
struct AAHist {
    const double *f[kMaxAnderson];
    const double *G[kMaxAnderson];
    double gamma[kMaxAnderson];
};

// Normal equations of min_gamma || f_k - sum_i gamma_i (f_k - f_i) ||: with
// d_i = f_k - f_i, partial sums of d_i d_j (i <= j), then d_i f_k, then f_k f_k.
template <int H>
__global__ void __launch_bounds__(kBlock)
    k_aa_gram(long long N, const double *__restrict__ fk, AAHist h, double *partials)
{
    constexpr int NV = H * (H + 1) / 2 + H + 1;
    double v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0;
    const long long step = (long long)gridDim.x * kBlock;
    for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < N; c += step) {
        const double r = fk[c];
        double d[H];
#pragma unroll
        for (int i = 0; i < H; ++i) d[i] = r - h.f[i][c];
        int q = 0;
#pragma unroll
        for (int i = 0; i < H; ++i)
#pragma unroll
            for (int j = i; j < H; ++j) v[q++] += d[i] * d[j];
#pragma unroll
        for (int i = 0; i < H; ++i) v[q++] += d[i] * r;
        v[q] += r * r;
    }
    block_store<NV>(v, partials, blockIdx.x);
}

// Next guess T_* = G_k - sum_i gamma_i (G_k - G_i), kept >= 0, and the scaled
// gas-energy residual R_T at (E, T_*) for the convergence test of that state.
template <class CT, int H>
__global__ void __launch_bounds__(kBlock)
    k_aa_mix(Grid g, const double *__restrict__ Gk, AAHist h, const CT *__restrict__ rho, const CT *__restrict__ kP,
             const double *__restrict__ Tn, const double *__restrict__ X, double *__restrict__ Tc, double *partials)
{
    const long long N = g.N;
    double v[2] = {0, 0};
    const long long step = (long long)gridDim.x * kBlock;
    for (long long c = (long long)blockIdx.x * kBlock + threadIdx.x; c < N; c += step) {
        const double gk = Gk[c];
        double T = gk;
#pragma unroll
        for (int i = 0; i < H; ++i) T -= h.gamma[i] * (gk - h.G[i][c]);
        T = fmax(T, 0.0);
        Tc[c] = T;
        const double r_ = (double)rho[c];
        const double sP = g.cdt * r_ * (double)kP[c], alpha = r_ * g.cv, aR = g.aR, E = X[c];
        const double T3 = T * T * T;
        const double RT0 = gas_e(g, alpha, T) - gas_e(g, alpha, Tn[c]) + sP * (aR * T3 * T - E);
        const double RT = (T == 0.0 && RT0 > 0.0) ? 0.0 : RT0;
        const double WT = gas_C(g, alpha, T) + 4.0 * sP * aR * T3;
        v[0] += WT > 0 ? (RT / WT) * (RT / WT) : 0.0;
        v[1] += T * T;
    }
    block_store<2>(v, partials, blockIdx.x);
}

template <int H>
void launch_aa_gram(int h, dim3 g, hipStream_t st, long long N, const double *fk, const AAHist &hist,
                    double *partials)
{
    if constexpr (H > 1) {
        if (h < H) return launch_aa_gram<H - 1>(h, g, st, N, fk, hist, partials);
    }
    hipLaunchKernelGGL((k_aa_gram<H>), g, dim3(kBlock), 0, st, N, fk, hist, partials);
}

template <class CT, int H>
void launch_aa_mix(int h, dim3 gr, hipStream_t st, const Grid &g, const double *Gk, const AAHist &hist,
                   const CT *rho, const CT *kP, const double *Tn, const double *X, double *Tc, double *partials)
{
    if constexpr (H > 1) {
        if (h < H) return launch_aa_mix<CT, H - 1>(h, gr, st, g, Gk, hist, rho, kP, Tn, X, Tc, partials);
    }
    hipLaunchKernelGGL((k_aa_mix<CT, H>), gr, dim3(kBlock), 0, st, g, Gk, hist, rho, kP, Tn, X, Tc, partials);
}

// Solve (D + lambda I) gamma = b for a symmetric positive semi-definite D of
// order n by Cholesky; lambda = 1e-12 max diag.  False if a pivot vanishes.
bool aa_solve(int n, const double *D, const double *b, double *gamma)
{
    double L[kMaxAnderson][kMaxAnderson] = {};
    double dmax = 0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, D[i * n + i]);
    if (!(dmax > 0)) return false;
    const double lam = 1e-12 * dmax;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = D[i * n + j] + (i == j ? lam : 0.0);
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 1e-14 * dmax)) return false;
                L[i][i] = std::sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[kMaxAnderson];
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * gamma[k];
        gamma[i] = s / L[i][i];
    }
    return true;
}

__global__ void __launch_bounds__(kBlock)
    k_commit(long long N, double c_light, const double *__restrict__ X, const double *__restrict__ Tc,
             double *__restrict__ E, double *__restrict__ F, double *__restrict__ T)
{
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= N) return;
    E[c] = X[c];
    for (int q = 0; q < 3; ++q) F[q * N + c] = X[(1 + q) * N + c] * c_light;
    T[c] = Tc[c];
}

// Sums the nv columns of partials[nblk][nv] in a fixed order: columns [0, na)
// go to out_a, columns [na, nv) to out_b; columns q >= mx take the maximum
// (of non-negative values) instead.  If sq_col >= 0, 1/sqrt of that column's
// sum is also written to *sdev (scale of a new Krylov vector).
__global__ void __launch_bounds__(kBlock)
    k_reduce(const double *__restrict__ partials, long long nblk, int nv, int na, double *out_a, double *out_b,
             int sq_col, double *sdev, int mx)
{
    __shared__ double sh[kBlock / 64];
    for (int q = 0; q < nv; ++q) {
        const bool m = q >= mx;
        double s = 0;
        for (long long b = threadIdx.x; b < nblk; b += kBlock)
            s = m ? fmax(s, partials[b * nv + q]) : s + partials[b * nv + q];
        s = m ? wave_max(s) : wave_sum(s);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int w = 0; w < kBlock / 64; ++w) t = m ? fmax(t, sh[w]) : t + sh[w];
            if (q < na)
                out_a[q] = t;
            else
                out_b[q - na] = t;
            if (q == sq_col) *sdev = t > 0 ? 1.0 / sqrt(t) : 0.0;
        }
        __syncthreads();
    }
}

// First stage of a long reduction: block b sums rows [256 b, 256 b + 256) of
// partials[nblk][nv] into out[b][nv] (fixed order, so reruns are bitwise equal).
__global__ void __launch_bounds__(kBlock)
    k_reduce_rows(const double *__restrict__ partials, long long nblk, int nv, double *__restrict__ out, int mx)
{
    __shared__ double sh[kBlock / 64];
    const long long row = (long long)blockIdx.x * kBlock + threadIdx.x;
    for (int q = 0; q < nv; ++q) {
        const bool m = q >= mx;
        double s = row < nblk ? partials[row * nv + q] : 0.0;
        s = m ? wave_max(s) : wave_sum(s);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0;
            for (int w = 0; w < kBlock / 64; ++w) t = m ? fmax(t, sh[w]) : t + sh[w];
            out[(long long)blockIdx.x * nv + q] = t;
        }
        __syncthreads();
    }
}

// Per-face speeds (FP64, physical units) for the rad_face_speeds entry point.
template <class CT>
__global__ void __launch_bounds__(kBlock)
    k_face_speeds(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kR, const CT *__restrict__ f,
                  double *__restrict__ C)
{
    const long long N = g.N;
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= N) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const double sRc = g.cdt * (double)rho[c] * (double)kR[c];
    for (int d = 0; d < 3; ++d) {
        long long nb = neighbour(g, i, j, k, c, d, 0);
        const double sRn = g.cdt * (double)rho[nb] * (double)kR[nb];
        C[d * N + c] = g.c * face_speed<double>((double)f[d * N + nb], (double)f[d * N + c], sRn, sRc, g.tau_k);
    }
}

template <class CT>
__global__ void __launch_bounds__(kBlock)
    k_exchange_only(long long n, Grid g, const CT *__restrict__ rho, const CT *__restrict__ kP,
                    const double *__restrict__ E, const double *__restrict__ Tn, double *__restrict__ T)
{
    long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    const double r_ = (double)rho[c];
    bool neg = false;
    T[c] = gas_exchange(g, r_ * g.cv, Tn[c], g.cdt * r_ * (double)kP[c], g.aR, E[c], 0.0, neg);
}

// --------------------------------------------------------------- host side

Grid make_grid(int nx, int ny, int nz, const int bc[6], double dt, double dx, const rad_params_t &p)
{
    Grid g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.N = (long long)nx * ny * nz;
    for (int a = 0; a < 3; ++a) {
        g.bclo[a] = bc[2 * a];
        g.bchi[a] = bc[2 * a + 1];
    }
    g.c = p.c;
    g.aR = p.a_R;
    g.cv = p.c_v;
    g.cdt = p.c * dt;
    g.nu = p.c * dt / dx;
    g.tau_k = 50.0 / (g.nu * g.nu);
    g.cv_cubic = p.cv_cubic;
    for (int f = 0; f < 6; ++f) g.finc8[f] = 8.0 * p.F_inc[f] / p.c;
    g.eps_N = p.eps_N;
    for (int f = 0; f < 6; ++f) g.ghost[f] = bc[f] == RAD_BC_DIRICHLET ? p.ghost[f] : nullptr;
    return g;
}

// Dirichlet faces on a uniform single grid: rejected, accepted (calls that never read the ghost
// data: the linear operator, the face speeds) or accepted with params->ghost of each such face set.
enum { DIR_NO = 0, DIR_ANY = 1, DIR_DATA = 2 };

// allow_walls: the open, Marshak and reflecting faces (uniform single grids)
int check_grid_args(int nx, int ny, int nz, double dt, double dx, const int bc[6], const rad_params_t *p,
                    int dirichlet, bool allow_walls = true)
{
    if (!p) return fail(RAD_EINVAL, "params is NULL");
    if (nx < 1 || ny < 1 || nz < 1) return fail(RAD_EINVAL, "grid extents must be >= 1");
    if ((long long)nx * ny * nz > (1LL << 31)) return fail(RAD_EINVAL, "grid larger than 2^31 cells");
    // the stencil addresses one z plane through a buffer descriptor (bytes < 2^31)
    if ((long long)nx * ny > (1LL << 27)) return fail(RAD_EINVAL, "nx * ny larger than 2^27 cells");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(RAD_EINVAL, "dt must be positive and finite");
    if (!(dx > 0) || !std::isfinite(dx)) return fail(RAD_EINVAL, "dx must be positive and finite");
    if (!bc) return fail(RAD_EINVAL, "bc is NULL");
    for (int f = 0; f < 6; ++f) {
        const bool wall = bc[f] == RAD_BC_OPEN || bc[f] == RAD_BC_MARSHAK || bc[f] == RAD_BC_REFLECT;
        if (bc[f] != RAD_BC_PERIODIC && bc[f] != RAD_BC_OUTFLOW && !(dirichlet && bc[f] == RAD_BC_DIRICHLET) &&
            !(allow_walls && wall))
            return fail(RAD_EINVAL, "unsupported boundary kind %d on face %d", bc[f], f);
        if (dirichlet == DIR_DATA && bc[f] == RAD_BC_DIRICHLET && !p->ghost[f])
            return fail(RAD_EINVAL, "Dirichlet face %d without ghost data (params->ghost[%d] is NULL)", f, f);
        // the sweep addresses a face's data plane by a 32-bit byte offset
        const long long n[3] = {nx, ny, nz}, area = n[(f / 2 + 1) % 3] * n[(f / 2 + 2) % 3];
        if (bc[f] == RAD_BC_DIRICHLET && area > (1LL << 26))
            return fail(RAD_EINVAL, "Dirichlet face %d larger than 2^26 cells", f);
    }
    for (int a = 0; a < 3; ++a)
        if ((bc[2 * a] == RAD_BC_PERIODIC) != (bc[2 * a + 1] == RAD_BC_PERIODIC))
            return fail(RAD_EINVAL, "periodic faces must come in pairs (axis %d)", a);
    return check_params(p);
}

struct Layout {
    size_t X, X0, Tc, Tfix, sR, dEA, fA, Cf, CW, CW64, sR64, Cf64, AAG, AAf, AMRC, AMRCA, VA, VB, VC, VBA, VCA, V, W, MG,
        part, small, total;
    long long nblk_cells, nblk_vec;
    size_t ksz;
};

long long wall_area(int nx, int ny, int nz) { return (long long)nx * ny + (long long)ny * nz + (long long)nx * nz; }

long long vec_blocks(long long n) { return std::min<long long>((n / 4 + kBlock - 1) / kBlock, 2048); }

// Upper bound on the workgroups of a tile sweep over an nx x ny x nz grid (tiles of
// 64 x 4 or more cells; z-ranges of all nz <= 8 planes, else at least 4): partial-sum rows.
long long tile_bound(int nx, int ny, int nz)
{
    return (long long)((nx + 63) / 64) * ((ny + 3) / 4) * (nz <= 8 ? 1 : (nz + 3) / 4);
}

// Multigrid levels below an nx x ny x nz grid: halve while every extent is even and
// the halves stay >= 4 cells, at most 5 levels in all (at 256^3 the coarsest is 16^3:
// a sixth level of 8^3 kept the iteration count and added two latency-bound sweeps to
// every cycle; four levels took more iterations).  Returns the level count (1: no
// coarse level) and the cells of the coarse levels.
constexpr int kMaxMg = 5;
int mg_levels(int nx, int ny, int nz, long long &coarse_cells)
{
    int L = 1;
    coarse_cells = 0;
    while (L < kMaxMg && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && nx >= 8 && ny >= 8 && nz >= 8) {
        nx /= 2;
        ny /= 2;
        nz /= 2;
        coarse_cells += (long long)nx * ny * nz;
        ++L;
    }
    return L;
}

// part_rows: partial-sum rows the sweeps of every level need (tile_bound summed);
// amr: room for the level-jump corrections (5 planes over the composite grid, FP64 for the
// residual and in the Krylov precision for the apply); vel: the O(v/c) coefficients of a
// moving medium (7 FP64 planes, the 6 couplings again in the Krylov precision for the apply).
// mg_cells: cells of the multigrid levels below the grid (krylov_poly = 2): per coarse cell 25
// values (sR, tensor, face speeds, E diagonal, Jacobi diagonal, right-hand side, residual,
// correction), and per grid cell 6 more (Jacobi diagonal, the fine correction)
// wall_area: cells on the three high faces of the grid (the high walls' own speeds of the grid and,
// in as much room again, of its multigrid levels)
Layout layout(long long N, const rad_params_t &p, long long part_rows, bool amr = false, bool vel = false,
              long long mg_cells = 0, long long wall_area = 0)
{
    Layout L;
    const bool mixed = p.prec == RAD_MIXED;
    const size_t ksz = mixed ? 4 : 8;
    L.ksz = ksz;
    const int m = p.gmres_m;
    L.nblk_cells = (N + kBlock - 1) / kBlock;
    L.nblk_vec = vec_blocks(4 * N);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align_up(bytes);
        return at;
    };
    L.X = take(4 * N * 8);
    L.X0 = take(4 * N * 8);
    L.Tc = take(N * 8);
    L.Tfix = take(p.energy_fix ? N * 8 : 0);   // the energy-corrected temperature of the last exchange
    L.sR = take(N * ksz);
    L.dEA = take(N * ksz);
    L.fA = (mixed && p.coef_dtype == RAD_F64) ? take(6 * N * ksz) : take(0);
    L.Cf = take(3 * N * ksz);
    L.CW = take(2 * wall_area * ksz);
    L.CW64 = take(mixed ? wall_area * 8 : 0);   // the grid's, in FP64 for the mixed path's residual
    // FP64 sR and face speeds of the FP64 residual (the FP64 path shares sR and Cf)
    L.sR64 = take(mixed ? N * 8 : 0);
    L.Cf64 = take(mixed ? 3 * N * 8 : 0);
    // Anderson history: m+1 slots of map values and residuals (N FP64 each)
    const int ma = p.anderson_m;
    L.AAG = take(ma > 0 ? (size_t)(ma + 1) * N * 8 : 0);
    L.AAf = take(ma > 0 ? (size_t)(ma + 1) * N * 8 : 0);
    L.AMRC = take(amr ? 5 * N * 8 : 0);
    L.AMRCA = take(amr ? 5 * N * ksz : 0);   // the same corrections in the Krylov precision, for the apply
    L.VA = take(vel ? N * 8 : 0);
    L.VB = take(vel ? 3 * N * 8 : 0);
    L.VC = take(vel ? 3 * N * 8 : 0);
    L.VBA = take(vel ? 3 * N * ksz : 0);
    L.VCA = take(vel ? 3 * N * ksz : 0);
    L.V = take((size_t)(m + 1) * 4 * N * ksz);
    L.W = take(4 * N * ksz);
    L.MG = take(mg_cells > 0 ? (size_t)(6 * N + 25 * mg_cells) * ksz : 0);
    // per-cell kernels of a two-level grid use one more (partial) block than the cell count gives
    L.part = take((size_t)std::max(std::max<long long>(L.nblk_cells + 2, L.nblk_vec), part_rows) * 24 * 8);
    L.small = take(512 * 8);
    L.total = o;
    return L;
}

// Small device area (doubles) that reductions write and the host reads back.
enum {
    SM_RED = 0,     // generic reduction results (<= 32)
    SM_DOTS = 32,   // <v_i, w>, i <= kMaxM (+16 slack for chunked writes)
    SM_WW = 120,    // <w, w>
    SM_NRM = 121,   // ||v_{j+1}||^2 after orthogonalisation
    SM_S = 128,     // basis scales s_i = 1 / ||v_i||, i <= kMaxM
    SM_TOTAL = 200
};

struct Solver {
    Grid g;        // the single grid, or the coarse level
    // levels: one uniform grid, or the coarse and fine levels of a two-level
    // composite grid stored one after the other (level l starts at cell c0[l]
    // of every per-cell array; each level is a complete single-grid array set)
    int nlev = 1;
    Grid gl[2];
    int mgL = 1;          // multigrid levels (krylov_poly = 2), the grid included
    Grid mg[kMaxMg];      // their grids (mg[0] = g)
    long long c0[2] = {0, 0};
    bool amr = false;
    bool walls = false;   // a Dirichlet, open, Marshak or reflecting face (uniform single grids only)
    bool dirichlet = false;   // ... of which a Dirichlet face
    Amr A{};
    long long nshell = 0, ncoarse = 0;  // threads of the level-jump kernel
    long long Ntot = 0;                 // cells of all levels
    const void *beta = nullptr;         // moving medium: v / c (3 planes, coefficient type), else null
    rad_params_t p;
    hipStream_t st;
    char *ws;
    Layout L;
    const void *rho, *kP, *kR, *f;
    const double *En, *Fn, *Tn;
    double *E, *F, *T;
    double *host;  // pinned staging, SM_TOTAL doubles
    rad_stats_t stats;
    int kz_apply = 0, kz_res = 0;  // tile z-ranges (0: default rule)
    int loadc = 1;                 // the Krylov apply reads the stored face speeds (0: forms them per face)
    // tuning mode: after the setup and the first residual, time these z-ranges
    // for the apply and the residual instead of stepping
    const std::vector<int> *tune_kz = nullptr;
    int tuned_apply = 0, tuned_res = 0, tuned_loadc = 1;

    template <class P>
    P *at(size_t off) { return reinterpret_cast<P *>(ws + off); }
    double *sm() { return at<double>(L.small); }
    double *part() { return at<double>(L.part); }

    // Sum the nv columns of part()[nblk][nv]; past 4096 rows a first pass folds every 256
    // rows into one (written after the rows in use; the partials area holds 24 values per
    // cell block, so it has room whenever nv <= 23).
    // columns q >= mx of the partials are maxima (non-negative), the others sums
    void reduce(long long nblk, int nv, int na, double *out_a, double *out_b = nullptr, int sq_col = -1,
                double *sdev = nullptr, int mx = 1 << 30)
    {
        const double *src = part();
        if (nblk > 4096 && nv <= 23) {
            const long long nb2 = (nblk + kBlock - 1) / kBlock;
            double *dst = part() + nblk * nv;
            hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)nb2), dim3(kBlock), 0, st, part(), nblk, nv, dst, mx);
            src = dst;
            nblk = nb2;
        }
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, src, nblk, nv, na, out_a, out_b, sq_col, sdev, mx);
    }
    // launch under the kernel-class profiler (no-op when profiling is off)
    template <class F>
    void timed(int kid, double bytes, F &&launch)
    {
        const int tok = prof_begin(kid, st);
        launch();
        prof_end(tok, st, bytes);
        stats.bytes_moved += bytes;
    }
    // copy sm()[off, off+count) to host[off...] and wait
    int read(int off, int count)
    {
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(host + off, sm() + off, count * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return RAD_OK;
    }
};

template <class CT, class KT>
int run_step(Solver &S)
{
    using AT = KT;
    Grid &g = S.g;
    const rad_params_t &p = S.p;
    const long long N = S.Ntot, n4 = 4 * N;
    const int NL = S.nlev;
    // gf: one 4-element group per thread for the Krylov streaming passes (their per-block
    // partial sums go through the two-stage reduction); gv: a capped grid for the rest
    const dim3 gv((unsigned)S.L.nblk_vec), gf((unsigned)S.L.nblk_cells), bl(kBlock);
    const CT *rho = (const CT *)S.rho, *kP = (const CT *)S.kP, *kR = (const CT *)S.kR, *f = (const CT *)S.f;
    double *X = S.at<double>(S.L.X), *X0 = S.at<double>(S.L.X0), *Tc = S.at<double>(S.L.Tc);
    double *Tfix = p.energy_fix ? S.at<double>(S.L.Tfix) : nullptr;
    bool exchanged = false;
    AT *sR = S.at<AT>(S.L.sR), *dEA = S.at<AT>(S.L.dEA);
    AT *fA = (p.prec == RAD_MIXED && p.coef_dtype == RAD_F64) ? S.at<AT>(S.L.fA) : nullptr;
    KT *V = S.at<KT>(S.L.V), *W = S.at<KT>(S.L.W);
    double *part = S.part(), *sm = S.sm(), *h = S.host;
    const int m = p.gmres_m;
    const bool poly = p.krylov_poly != 0;
    const long long stride = n4;
    rad_stats_t &st = S.stats;

    const bool mixed = sizeof(KT) == 4;
    double *sR64 = mixed ? S.at<double>(S.L.sR64) : (double *)sR;
    const double cb = sizeof(CT), kb = sizeof(KT), Nd = (double)N;
    // per-cell kernels run once per level; their partial sums are stacked level after level
    auto cell_grid = [&](int l) { return dim3((unsigned)((S.gl[l].N + kBlock - 1) / kBlock)); };
    long long rows = 0;
    S.timed(K_SETUP, Nd * (9 * cb + 40 + kb + (mixed ? 8 : 0) + (fA ? 6 * kb : 0) + 72), [&] {
        for (int l = 0; l < NL; ++l) {
            const long long o = S.c0[l];
            hipLaunchKernelGGL((k_setup<CT, AT>), cell_grid(l), bl, 0, S.st, S.gl[l], rho + o, kP + o, kR + o,
                               f + 6 * o, sR + o, mixed ? sR64 + o : nullptr, fA ? fA + 6 * o : nullptr, S.En + o,
                               S.Fn + 3 * o, S.Tn + o, X + 4 * o, X0 + 4 * o, Tc + o, part + rows);
            rows += cell_grid(l).x;
        }
    });
    S.reduce(rows, 1, 1, sm + SM_RED);
    RAD_TRY(S.read(SM_RED, 1));
    st.bad_cells = (int)h[SM_RED];
    if (st.bad_cells > 0) return fail(RAD_EDATA, "%d cells with invalid rho/kappa/f data", st.bad_cells);

    const int kApply = sizeof(KT) == 4 ? K_APPLY32 : K_APPLY64;
    const int kDot = sizeof(KT) == 4 ? K_MULTIDOT32 : K_MULTIDOT64;
    const int kOrth = sizeof(KT) == 4 ? K_ORTH32 : K_ORTH64;
    const int kUpd = sizeof(KT) == 4 ? K_UPDATEX32 : K_UPDATEX64;
    const double fb = fA ? kb : cb;   // bytes per stored tensor component read by the apply
    TileGeom tg[2], tgr[2];
    for (int l = 0; l < NL; ++l) {
        tg[l] = tile_geom<AT>(S.gl[l], S.kz_apply);
        tgr[l] = tile_geom<double>(S.gl[l], S.kz_res, 32, 256);
    }
    auto tiles = [](const TileGeom &t) { return dim3((unsigned)(t.tiles_x * t.tiles_y * t.tiles_z)); };
    const dim3 bt(tile_threads<AT>()), bt64(tile_threads<double>());
    AT *Cf = S.at<AT>(S.L.Cf);
    double *Cf64 = mixed ? S.at<double>(S.L.Cf64) : (double *)Cf;
    S.timed(K_SETUP, Nd * (3 * cb + 3 * kb), [&] {
        for (int l = 0; l < NL; ++l) {
            const long long o = S.c0[l];
            hipLaunchKernelGGL((k_face_coef<CT, AT>), cell_grid(l), bl, 0, S.st, S.gl[l], rho + o, kR + o, f + 6 * o,
                               Cf + 3 * o);
        }
    });
    if (mixed)
        S.timed(K_SETUP, Nd * (3 * cb + 3 * 8), [&] {
            for (int l = 0; l < NL; ++l) {
                const long long o = S.c0[l];
                hipLaunchKernelGGL((k_face_coef<CT, double>), cell_grid(l), bl, 0, S.st, S.gl[l], rho + o, kR + o,
                                   f + 6 * o, Cf64 + 3 * o);
            }
        });
    // the high walls' own speeds (FP32 Krylov apply)
    const bool walls = S.walls;
    const int wl = walls ? (S.dirichlet ? 2 : 1) : 0;   // the sweep's wall level
    AT *CwA = walls ? S.at<AT>(S.L.CW) : nullptr;
    double *Cw64 = walls ? (mixed ? S.at<double>(S.L.CW64) : (double *)CwA) : nullptr;
    if (walls && !S.amr)
        S.timed(K_SETUP, 0.0, [&] {
            const long long nw = wall_area(g.nx, g.ny, g.nz);
            hipLaunchKernelGGL((k_wall_speed<CT, AT>), dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, S.st, g, rho,
                               kR, (const AT *)nullptr, f, CwA);
            if (mixed)
                hipLaunchKernelGGL((k_wall_speed<CT, double>), dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, S.st,
                                   g, rho, kR, (const double *)nullptr, f, Cw64);
        });
    // moving medium: the O(v/c) coefficients, once per step
    const bool vel = S.beta != nullptr;
    const int vimp = vel && p.vel_implicit;
    double *VA = vel ? S.at<double>(S.L.VA) : nullptr, *VB = vel ? S.at<double>(S.L.VB) : nullptr;
    double *VC = vel ? S.at<double>(S.L.VC) : nullptr;
    AT *VBA = vel ? S.at<AT>(S.L.VBA) : nullptr, *VCA = vel ? S.at<AT>(S.L.VCA) : nullptr;
    if (vel) {
        S.timed(K_SETUP, Nd * (12 * cb + 56 + 6 * kb), [&] {
            hipLaunchKernelGGL((k_vel_coef<CT, AT>), cell_grid(0), bl, 0, S.st, g, rho, kP, kR, f, (const CT *)S.beta,
                               VA, VB, VC, VBA, VCA, part);
        });
        S.reduce(cell_grid(0).x, 1, 1, sm + SM_RED);
        RAD_TRY(S.read(SM_RED, 1));
        if (h[SM_RED] > 0) {
            st.bad_cells = (int)h[SM_RED];
            return fail(RAD_EDATA, "%d cells with non-finite velocity", st.bad_cells);
        }
    }
    // two-level grid: level-jump corrections of the operand x (scaled by *xs), read by the sweeps' epilogues
    double *corr = S.amr ? S.at<double>(S.L.AMRC) : nullptr;
    AT *corrA = S.amr ? S.at<AT>(S.L.AMRCA) : nullptr;
    auto level_view = [&](int l, const void *cbase, size_t esz) {
        AmrLv v;
        v.a = S.A;
        v.lev = l;
        v.corr = cbase ? (const char *)cbase + esz * 5 * S.c0[l] : nullptr;
        return v;
    };
    auto jump = [&](auto x, const double *xs, auto Cc, auto out) {
        using XT = std::remove_const_t<std::remove_pointer_t<decltype(x)>>;
        using FT = std::remove_const_t<std::remove_pointer_t<decltype(Cc)>>;
        using OT = std::remove_pointer_t<decltype(out)>;
        const long long nt = S.nshell + S.ncoarse;
        S.timed(K_AMR, (double)nt * 10 * 8 * sizeof(XT), [&] {
            hipLaunchKernelGGL((k_amr_jump<XT, CT, FT, OT>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, S.st,
                               S.A, S.gl[0], S.gl[1], S.nshell, S.ncoarse, (const XT *)x, xs, f,
                               (const double *)sR64, (const FT *)Cc, out);
        });
    };
    // mgm, mf: the multigrid transfer fused into the sweep (1: restriction of y into mf, which is then
    // not written; 2: injection of mf's coarse correction into the operand; FP32 only)
    auto apply = [&](const KT *x, const double *xs, KT *y, AT pg = AT(0), AT xm = AT(1), const AT *qv = nullptr,
                     AT qm = AT(0), AT qs = AT(1), AT *dout = nullptr, int mgm = 0,
                     const MgFuse<AT> &mf = MgFuse<AT>{}) {
        if (S.amr) jump(x, xs, (const AT *)Cf, corrA);
        const int tok = prof_begin(kApply, S.st);
        for (int l = 0; l < NL; ++l) {
            const long long o = S.c0[l];
            auto go = [&](auto amr_c, auto vel_c, auto lc_c, auto wl_c, auto mg_c) {
                constexpr bool AM = decltype(amr_c)::value, VL = decltype(vel_c)::value, LC = decltype(lc_c)::value;
                constexpr int WLc = decltype(wl_c)::value;
                constexpr int MG = decltype(mg_c)::value;
                const dim3 bta(tile_threads<AT, AM>());   // the two-level grid's sweep shape
                // not built: walls on the two-level grid, fused transfers outside the plain FP32 apply,
                // Dirichlet faces with the face speeds formed per face
                if constexpr (!(AM && WLc) && (MG == 0 || (!AM && !VL && std::is_same<AT, float>::value)) &&
                              !(WLc == 2 && !LC)) {
                    if (fA)
                        hipLaunchKernelGGL((k_apply_tiled<AT, AT, true, AM, VL, LC, WLc, MG>), tiles(tg[l]), bta, 0,
                                           S.st, S.gl[l], tg[l], (const AT *)fA + 6 * o, sR + o, (const AT *)nullptr,
                                           (const AT *)nullptr, (const AT *)Cf + 3 * o, dEA + o, x + 4 * o, xs,
                                           y + 4 * o, AT(1), AT(1), level_view(l, corrA, sizeof(AT)),
                                           (const AT *)VBA, (const AT *)VCA, pg, xm, qv, qm, qs, dout, mf,
                                           (const AT *)CwA);
                    else
                        hipLaunchKernelGGL((k_apply_tiled<AT, CT, true, AM, VL, LC, WLc, MG>), tiles(tg[l]), bta, 0,
                                           S.st, S.gl[l], tg[l], f + 6 * o, sR + o, (const CT *)nullptr,
                                           (const CT *)nullptr, (const AT *)Cf + 3 * o, dEA + o, x + 4 * o, xs,
                                           y + 4 * o, AT(1), AT(1), level_view(l, corrA, sizeof(AT)),
                                           (const AT *)VBA, (const AT *)VCA, pg, xm, qv, qm, qs, dout, mf,
                                           (const AT *)CwA);
                }
            };
            // grids with Dirichlet, open, Marshak or reflecting faces take the sweep with the wall code
            // (Dirichlet faces: its own level, with the stored face speeds)
            auto go2 = [&](auto amr_c, auto vel_c, auto lc_c) {
                using I0 = std::integral_constant<int, 0>;
                using I1 = std::integral_constant<int, 1>;
                using I2 = std::integral_constant<int, 2>;
                auto go3 = [&](auto wl_c, auto lc2) {
                    if (mgm == 1) go(amr_c, vel_c, lc2, wl_c, I1{});
                    else if (mgm == 2) go(amr_c, vel_c, lc2, wl_c, I2{});
                    else go(amr_c, vel_c, lc2, wl_c, I0{});
                };
                if (wl == 2) go3(I2{}, std::true_type{});
                else if (wl == 1) go3(I1{}, lc_c);
                else go3(I0{}, lc_c);
            };
            if (S.amr)
                go2(std::true_type{}, std::false_type{}, std::true_type{});
            else if (vel)
                go2(std::false_type{}, std::true_type{}, std::true_type{});
            else if (S.loadc)
                go2(std::false_type{}, std::false_type{}, std::true_type{});
            else
                go2(std::false_type{}, std::false_type{}, std::false_type{});
        }
        // the smoothing form also reads q (4 planes), the diagonal form writes D (2 planes); the fused
        // restriction writes an eighth of y, the fused injection reads an eighth more operand
        const double ybytes = mgm == 1 ? 0.5 * kb : 4 * kb, xbytes = mgm == 2 ? 4.5 * kb : 4 * kb;
        prof_end(tok, S.st, Nd * (xbytes + ybytes + 6 * fb + 5 * kb + (qv ? 4 * kb : 0) + (dout ? 2 * kb : 0)));
    };
    // ---- multigrid cycle (krylov_poly = 2): levels l >= 1 halve the grid; each carries the
    // children's mean sR, tensor and E diagonal, its own corrected face speeds and Jacobi
    // diagonal, and a right-hand side q, residual t and correction e.  One V-cycle with one
    // damped Jacobi sweep (weight kOm) before and after the coarse correction, and kCoarse + 1
    // sweeps from zero on the coarsest level (the first is e = om q; more did not pay at 256^3,
    // whose coarsest level is 16^3), is the (fixed, linear) right preconditioner M^-1 of B.
    // The weight is small because the scaled operator has eigenvalues far off the real axis
    // in optically thin media, which larger weights amplify.
    constexpr double kOm = 0.4;
    constexpr int kCoarse = 1;
    const int mgL = p.krylov_poly == 2 ? S.mgL : 1;
    bool use_mg = mgL > 1;   // cleared for the rest of the step if a cycle stalls
    struct MgLev {
        AT *sR, *f, *Cf, *dE, *D, *q, *t, *e;
        AT *Cw;   // the high walls' own speeds (grids with Dirichlet, open, Marshak or reflecting faces)
        TileGeom tg;
    };
    MgLev ml[kMaxMg] = {};
    AT *mgE0 = nullptr;
    auto mg_cells = [&](const Grid &g) { return dim3((unsigned)((g.N + kBlock - 1) / kBlock)); };
    if (mgL > 1) {
        AT *b = S.at<AT>(S.L.MG);
        ml[0].D = b;
        b += 2 * N;
        mgE0 = b;
        b += 4 * N;
        ml[0].tg = tg[0];
        for (int l = 1; l < mgL; ++l) {
            const long long Nl = S.mg[l].N;
            AT **dst[8] = {&ml[l].sR, &ml[l].f, &ml[l].Cf, &ml[l].dE, &ml[l].D, &ml[l].q, &ml[l].t, &ml[l].e};
            const int planes[8] = {1, 6, 3, 1, 2, 4, 4, 4};
            for (int u = 0; u < 8; ++u) {
                *dst[u] = b;
                b += planes[u] * Nl;
            }
            // the level's high-wall speeds, after the grid's in the same area
            ml[l].Cw = walls ? (l == 1 ? CwA + wall_area(g.nx, g.ny, g.nz) : ml[l - 1].Cw + wall_area(S.mg[l - 1].nx, S.mg[l - 1].ny, S.mg[l - 1].nz))
                             : nullptr;
            // small levels: short z-ranges, so that their few columns still give a few hundred workgroups
            // (a sweep of one workgroup over 8 planes is latency-bound)
            ml[l].tg = tile_geom<AT>(S.mg[l]);
            const long long cols = (long long)ml[l].tg.tiles_x * ml[l].tg.tiles_y;
            if (cols * ml[l].tg.tiles_z < 256) ml[l].tg = tile_geom<AT>(S.mg[l], 2);
        }
        S.timed(K_SETUP, Nd * (7 * kb + 1.25 * kb), [&] {
            for (int l = 1; l < mgL; ++l) {
                const Grid &gf = S.mg[l - 1], &gc = S.mg[l];
                if (l == 1) {
                    hipLaunchKernelGGL((k_mg_average<AT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 1, (const AT *)sR,
                                       N, ml[1].sR);
                    if (fA)
                        hipLaunchKernelGGL((k_mg_average<AT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 6,
                                           (const AT *)fA, N, ml[1].f);
                    else
                        hipLaunchKernelGGL((k_mg_average<CT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 6, f, N,
                                           ml[1].f);
                } else {
                    hipLaunchKernelGGL((k_mg_average<AT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 1,
                                       (const AT *)ml[l - 1].sR, gf.N, ml[l].sR);
                    hipLaunchKernelGGL((k_mg_average<AT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 6,
                                       (const AT *)ml[l - 1].f, gf.N, ml[l].f);
                }
                hipLaunchKernelGGL((k_mg_face<AT>), mg_cells(gc), bl, 0, S.st, gc, (const AT *)ml[l].sR,
                                   (const AT *)ml[l].f, ml[l].Cf);
                if (walls) {
                    const long long nw = wall_area(gc.nx, gc.ny, gc.nz);
                    hipLaunchKernelGGL((k_wall_speed<AT, AT, true>), dim3((unsigned)((nw + 255) / 256)), dim3(256), 0,
                                       S.st, gc, (const AT *)nullptr, (const AT *)nullptr, (const AT *)ml[l].sR,
                                       (const AT *)ml[l].f, ml[l].Cw);
                }
            }
        });
    }
    // the operator of level l >= 1 (same sweep as the grid's apply, coarse coefficients)
    // (profiled as the multigrid class, so the grid's apply keeps its own class)
    auto mg_apply = [&](int l, const AT *x, AT xm, AT *y, AT pg, const AT *qv, AT qm, AT *dout, int mgm = 0,
                        const MgFuse<AT> &mf = MgFuse<AT>{}) {
        const int tok = prof_begin(K_MG, S.st);
        auto pick = [&](auto wl_c, auto mg_c) {
            constexpr int WLc = decltype(wl_c)::value;
            constexpr int MG = decltype(mg_c)::value;
            if constexpr (MG == 0 || std::is_same<AT, float>::value)
                return &k_apply_tiled<AT, AT, true, false, false, true, WLc, MG>;
            else
                return &k_apply_tiled<AT, AT, true, false, false, true, WLc, 0>;
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        auto pick3 = [&](auto wl_c) { return mgm == 1 ? pick(wl_c, I1{}) : mgm == 2 ? pick(wl_c, I2{}) : pick(wl_c, I0{}); };
        auto kern = wl == 2 ? pick3(I2{}) : wl == 1 ? pick3(I1{}) : pick3(I0{});
        hipLaunchKernelGGL(kern, tiles(ml[l].tg), bt, 0, S.st, S.mg[l], ml[l].tg, (const AT *)ml[l].f,
                           (const AT *)ml[l].sR, (const AT *)nullptr, (const AT *)nullptr, (const AT *)ml[l].Cf,
                           (const AT *)ml[l].dE, x, (const double *)nullptr, y, AT(1), AT(1), AmrLv{},
                           (const AT *)nullptr, (const AT *)nullptr, pg, xm, qv, qm, AT(1), dout, mf,
                           (const AT *)ml[l].Cw);
        const double ybytes = mgm == 1 ? 0.5 * kb : 4 * kb, xbytes = mgm == 2 ? 4.5 * kb : 4 * kb;
        prof_end(tok, S.st,
                 (double)S.mg[l].N * (xbytes + ybytes + 6 * kb + 5 * kb + (qv ? 4 * kb : 0) + (dout ? 2 * kb : 0)));
    };
    // the transfers between levels l and l+1 fused into level l's sweeps: FP32 tiles over even z-ranges
    auto fusable = [&](int l) {
        return std::is_same<AT, float>::value && (l == 0 ? tg[0].kz : ml[l].tg.kz) % 2 == 0;
    };
    auto fuse_to = [&](int l) {   // the coarse level l + 1 as the fused transfers see it
        MgFuse<AT> m;
        const Grid &gc = S.mg[l + 1];
        m.qc = ml[l + 1].q;
        m.Dc = ml[l + 1].D;
        m.ec = ml[l + 1].e;
        m.Nc = gc.N;
        m.ncx = gc.nx;
        m.ncy = gc.ny;
        return m;
    };
    // this Picard iteration's Jacobi diagonals of every level (dE changes with T*)
    auto mg_diagonals = [&]() {
        // (the grid's own diagonal only serves the unfused restriction)
        if (!fusable(0)) apply(V, nullptr, mgE0, AT(0), AT(1), nullptr, AT(0), AT(1), ml[0].D);
        for (int l = 1; l < mgL; ++l) {
            const Grid &gf = S.mg[l - 1], &gc = S.mg[l];
            hipLaunchKernelGGL((k_mg_average<AT, AT>), mg_cells(gc), bl, 0, S.st, gf, gc, 1,
                               (const AT *)(l == 1 ? dEA : ml[l - 1].dE), gf.N, ml[l].dE);
            mg_apply(l, ml[l].f, AT(1), ml[l].t, AT(0), nullptr, AT(0), ml[l].D);
        }
    };
    // q_{l+1} = D_{l+1}^-1 mean(D_l t) and e = qs q + P e_c, between levels l and l+1
    auto mg_restrict = [&](int l, const AT *t, const AT *D) {
        const Grid &gf = S.mg[l], &gc = S.mg[l + 1];
        S.timed(K_MG, (double)kb * (6.0 * gf.N + 6.0 * gc.N), [&] {
            hipLaunchKernelGGL((k_mg_restrict<AT>), mg_cells(gc), bl, 0, S.st, gf, gc, t, D, (const AT *)ml[l + 1].D,
                               ml[l + 1].q);
        });
    };
    auto mg_inject = [&](int l, const AT *q, AT qs, const AT *ec, AT *e) {
        const Grid &gf = S.mg[l], &gc = S.mg[l + 1];
        S.timed(K_MG, (double)kb * (8.0 * gf.N + 4.0 * gc.N), [&] {
            hipLaunchKernelGGL((k_mg_inject<AT>), mg_cells(gf), bl, 0, S.st, gf, gc, q, qs, ec, e);
        });
    };
    // V-cycle on level l >= 1 for B_l e = q_l; returns the buffer holding e.  The coarse correction
    // is always left in ml[l].e (the fused injection reads it there).
    std::function<AT *(int)> mg_cycle = [&](int l) -> AT * {
        if (l == mgL - 1) {   // coarsest: kCoarse sweeps after e = om q
            AT *cur = ml[l].t, *nxt = ml[l].e;
            if (kCoarse % 2) std::swap(cur, nxt);
            mg_apply(l, ml[l].q, AT(kOm), cur, AT(0), ml[l].q, AT(kOm), nullptr);
            for (int k = 1; k < kCoarse; ++k) {
                mg_apply(l, cur, AT(1), nxt, AT(0), ml[l].q, AT(kOm), nullptr);
                std::swap(cur, nxt);
            }
            return cur;
        }
        AT *out = ml[l].e;
        if (fusable(l)) {
            const MgFuse<AT> mf = fuse_to(l);
            // t = q - B (om q), restricted into q_{l+1} as it is formed
            mg_apply(l, ml[l].q, AT(kOm), ml[l].t, AT(1.0 / kOm), nullptr, AT(0), nullptr, 1, mf);
            mg_cycle(l + 1);
            // the sweep on e = om q + P e_{l+1}, injected as it is loaded
            MgFuse<AT> mi = mf;
            mi.a = AT(kOm);
            mg_apply(l, ml[l].q, AT(1), out, AT(0), ml[l].q, AT(kOm), nullptr, 2, mi);
            return out;
        }
        // t = q - B (om q): the residual after the first sweep from zero
        mg_apply(l, ml[l].q, AT(kOm), ml[l].t, AT(1.0 / kOm), nullptr, AT(0), nullptr);
        mg_restrict(l, ml[l].t, ml[l].D);
        AT *ec = mg_cycle(l + 1);
        mg_inject(l, ml[l].q, AT(kOm), ec, ml[l].t);
        mg_apply(l, ml[l].t, AT(1), out, AT(0), ml[l].q, AT(kOm), nullptr);
        return out;
    };
    // out = M^-1 (sx x) on the grid; xs: the device copy of the scale sx (or null for 1)
    auto mg_precond = [&](const KT *x, const double *xs, double sx, KT *out) {
        if (fusable(0)) {
            const MgFuse<AT> mf = fuse_to(0);
            apply(x, xs, W, AT(1.0 / kOm), AT(kOm), nullptr, AT(0), AT(1), nullptr, 1, mf);   // q_1 from q - B (om q)
            mg_cycle(1);
            MgFuse<AT> mi = mf;
            mi.a = AT(kOm * sx);   // the sweep on e = om sx x + P e_1
            apply(x, nullptr, out, AT(0), AT(1), (const AT *)x, AT(kOm), AT(sx), nullptr, 2, mi);
            return;
        }
        apply(x, xs, W, AT(1.0 / kOm), AT(kOm));   // W = q - B (om q), q = sx x
        mg_restrict(0, W, ml[0].D);
        AT *ec = mg_cycle(1);
        mg_inject(0, x, AT(kOm * sx), ec, mgE0);
        apply(mgE0, nullptr, out, AT(0), AT(1), (const AT *)x, AT(kOm), AT(sx));
    };

    // FP64 residual of the current linear system at X, Jacobi-scaled, into V[0];
    // its norm's inverse becomes the scale s_0 of V[0].
    double nrm[5];
    auto residual = [&]() -> int {
        if (S.amr) jump((const double *)X, (const double *)nullptr, (const double *)Cf64, corr);
        // streams X, En/Fn/Tn/Ts, sR and face speeds (FP64), f, rho, kP; writes V[0], dE
        long long rrows = 0;
        S.timed(K_RESIDUAL, Nd * (32 + 48 + 32 + 8 * cb + 5 * kb), [&] {
            for (int l = 0; l < NL; ++l) {
                const long long o = S.c0[l];
                auto go = [&](auto amr_c, auto vel_c) {
                    constexpr bool AM = decltype(amr_c)::value;
                    constexpr int VL = decltype(vel_c)::value;
                    auto kern = (wl == 2 && !AM)   ? k_residual_tiled<CT, KT, AT, false, VL, 2>
                                : (wl == 1 && !AM) ? k_residual_tiled<CT, KT, AT, false, VL, 1>
                                                   : k_residual_tiled<CT, KT, AT, AM, VL, 0>;
                    hipLaunchKernelGGL(kern, tiles(tgr[l]), bt64, 0, S.st, S.gl[l], tgr[l], p.mode, S.En + o,
                                       S.Fn + 3 * o, S.Tn + o, Tc + o, rho + o, kP + o, f + 6 * o, sR64 + o,
                                       Cf64 + 3 * o, X + 4 * o, V + 4 * o, dEA + o, part + rrows * 5,
                                       level_view(l, corr, sizeof(double)), (const double *)VA, (const double *)VB,
                                       (const double *)VC, VBA, (const double *)Cw64);
                };
                if (S.amr)
                    go(std::true_type{}, std::integral_constant<int, 0>{});
                else if (vimp)
                    go(std::false_type{}, std::integral_constant<int, 2>{});
                else if (vel)
                    go(std::false_type{}, std::integral_constant<int, 1>{});
                else
                    go(std::false_type{}, std::integral_constant<int, 0>{});
                rrows += tiles(tgr[l]).x;
            }
        });
        S.reduce(rrows, 5, 5, sm + SM_RED, nullptr, 4, sm + SM_S);
        RAD_TRY(S.read(SM_RED, 5));
        for (int q = 0; q < 5; ++q) nrm[q] = h[SM_RED + q];
        st.refine_sweeps++;
        return RAD_OK;
    };
    // <V_i, w> for i < cnt into SM_DOTS and <w, w> into SM_WW
    auto multidot = [&](int cnt, const KT *w) {
        for (int i0 = 0; i0 < cnt; i0 += 16) {
            const int c = std::min(16, cnt - i0);
            S.timed(kDot, 4 * Nd * kb * (c + 1),
                    [&] { launch_multidot<KT, 16>(c, gf, S.st, V, stride, i0, w, n4, part); });
            S.reduce(S.L.nblk_cells, c + 1, c, sm + SM_DOTS + i0, sm + SM_WW);
        }
    };

    double resT = 0, best_res = INFINITY;
    int best_at = 0;
    int status = RAD_NOT_CONVERGED;
    // Anderson acceleration of the Picard map (off when anderson_m = 0)
    const int aa_m = p.anderson_m;
    double *AAG = aa_m > 0 ? S.at<double>(S.L.AAG) : nullptr, *AAf = aa_m > 0 ? S.at<double>(S.L.AAf) : nullptr;
    std::vector<int> aa_hist;  // history slots, most recent first
    double aa_best = INFINITY;
    const bool trace = trace_enabled();
    int reorth = 0, cycles = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gvec(m + 1), y(m), sv(m + 1);

    if (S.tune_kz) {
        // time each candidate z-range: 1 warm-up + 5 applies, 1 warm-up + 3 residuals
        RAD_TRY(residual());
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        float best_a = INFINITY, best_r = INFINITY;
        int rc = RAD_OK;
        for (int kz : *S.tune_kz) {
            tg[0] = tile_geom<AT>(g, kz);
            tgr[0] = tile_geom<double>(g, kz);
            float ms_r = 0;
            // the apply with stored face speeds, then with face speeds formed per face
            for (int lc = 1; lc >= 0 && rc == RAD_OK; --lc) {
                S.loadc = lc;
                float ms_a = 0;
                apply(V, sm + SM_S, W);
                if (hipEventRecord(e0, S.st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
                for (int r = 0; r < 5 && rc == RAD_OK; ++r) apply(V, sm + SM_S, W);
                if (rc == RAD_OK && hipEventRecord(e1, S.st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
                if (rc == RAD_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(RAD_EHIP, "apply trial failed");
                if (rc == RAD_OK && hipEventElapsedTime(&ms_a, e0, e1) != hipSuccess)
                    rc = fail(RAD_EHIP, "timing failed");
                if (rc != RAD_OK) break;
                if (trace) std::fprintf(stderr, "[rad] tune kz=%d loadc=%d: apply %.3f ms\n", kz, lc, ms_a / 5);
                if (ms_a < best_a) {
                    best_a = ms_a;
                    S.tuned_apply = kz;
                    S.tuned_loadc = lc;
                }
            }
            S.loadc = 1;
            if (rc == RAD_OK) rc = residual();
            if (rc == RAD_OK && hipEventRecord(e0, S.st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
            for (int r = 0; r < 3 && rc == RAD_OK; ++r) rc = residual();
            if (rc == RAD_OK && hipEventRecord(e1, S.st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
            if (rc == RAD_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(RAD_EHIP, "residual trial failed");
            if (rc == RAD_OK && hipEventElapsedTime(&ms_r, e0, e1) != hipSuccess) rc = fail(RAD_EHIP, "timing failed");
            if (rc != RAD_OK) break;
            if (trace) std::fprintf(stderr, "[rad] tune kz=%d: residual %.3f ms\n", kz, ms_r / 3);
            if (ms_r < best_r) {
                best_r = ms_r;
                S.tuned_res = kz;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
    }

    for (int k = 0;; ++k) {
        RAD_TRY(residual());
        const double nE = std::sqrt(nrm[2]), nF = std::sqrt(nrm[3]);
        st.res_E = nE > 0 ? std::sqrt(nrm[0]) / nE : std::sqrt(nrm[0]);
        st.res_F = (nF + nE) > 0 ? std::sqrt(nrm[1]) / (nF + nE) : std::sqrt(nrm[1]);
        st.res_T = resT;
        const double res = std::max(std::max(st.res_E, st.res_F), resT);
        st.scaled_residual = res;
        if (k > 0 && (res <= p.tol || (p.eps_P > 0 && st.rel_change < p.eps_P))) {
            status = RAD_OK;
            break;
        }
        if (k >= p.max_picard) break;
        // stall: no new best residual within the last 5 Picard iterations (active-set cycling);
        // with Anderson mixing the residual is not monotone: its history restarts after
        // max(3, m) iterations without a new best, and the step gives up after 15
        if (res < best_res) {
            best_res = res;
            best_at = k;
        } else if (k - best_at >= (aa_m > 0 ? 15 : 5)) {
            break;
        } else if (aa_m > 0 && k - best_at >= std::max(3, aa_m)) {
            aa_hist.clear();
        }

        // ---- Krylov solve of A d = r for the correction, accumulated into X.
        // Linear tolerance: eps_R relative, tightened so the last solve reaches tol.
        if (use_mg) mg_diagonals();
        double beta = std::sqrt(nrm[4]);
        const double rtol = std::min(1.0, std::max(std::min(p.eps_R, 1.0), 0.1 * p.tol / std::max(res, 1e-300)));
        const double target = beta * rtol;
        const double inner_floor = (sizeof(KT) == 4) ? 1e-5 : 0.0;  // FP32 Arnoldi resolves ~5 decades per cycle
        int its = 0;
        double beta_prev = INFINITY;
        int restarts = 0;
        while (beta > target && beta > 0 && its < p.max_krylov && beta < 0.999 * beta_prev &&
               (p.max_refine == 0 || restarts++ < p.max_refine)) {
            beta_prev = beta;
            const double cycle_target = std::max(target, beta * inner_floor);
            RAD_TRY(S.read(SM_S, 1));
            sv[0] = h[SM_S];
            std::fill(gvec.begin(), gvec.end(), 0.0);
            gvec[0] = beta;
            int cols = 0;
            for (int j = 0; j < m && its < p.max_krylov; ++j) {
                KT *vn = V + (long long)(j + 1) * stride;
                KT *wv = W;   // the new Krylov direction before orthogonalisation
                if (use_mg) {   // w = B M^-1 (s_j V_j), formed in the slot of V_j+1
                    mg_precond(V + (long long)j * stride, sm + SM_S + j, sv[j], W);
                    apply(W, nullptr, vn);
                    wv = vn;
                } else if (poly) {   // W = (2I - B) B (s_j V_j); B (s_j V_j) parks in the slot of V_j+1
                    apply(V + (long long)j * stride, sm + SM_S + j, vn);
                    apply(vn, nullptr, W, AT(2));
                } else {
                    apply(V + (long long)j * stride, sm + SM_S + j, W);
                }
                ++its;
                multidot(j + 1, wv);
                S.timed(kOrth, 4 * Nd * kb * (j + 3), [&] {
                    launch_orth_update<KT>(j + 1, gf, S.st, V, stride, wv, vn, sm + SM_DOTS, sm + SM_S, n4, part);
                });
                S.reduce(S.L.nblk_cells, 1, 1, sm + SM_NRM, nullptr, 0, sm + SM_S + j + 1);
                RAD_TRY(S.read(0, SM_TOTAL));
                const double ww = h[SM_WW];
                double nn = h[SM_NRM];
                for (int i = 0; i <= j; ++i) H[i * m + j] = sv[i] * h[SM_DOTS + i];
                // classical Gram-Schmidt, one pass (as PETSc's default GMRES); a second pass
                // only when cancellation left less than 1e-3 of the norm
                if (nn < 1e-6 * ww) {
                    ++reorth;
                    multidot(j + 1, vn);
                    S.timed(kOrth, 4 * Nd * kb * (j + 3), [&] {
                        launch_orth_update<KT>(j + 1, gf, S.st, V, stride, vn, vn, sm + SM_DOTS, sm + SM_S, n4, part);
                    });
                    S.reduce(S.L.nblk_cells, 1, 1, sm + SM_NRM, nullptr, 0, sm + SM_S + j + 1);
                    RAD_TRY(S.read(0, SM_TOTAL));
                    nn = h[SM_NRM];
                    for (int i = 0; i <= j; ++i) H[i * m + j] += sv[i] * h[SM_DOTS + i];
                }
                const double hn = std::sqrt(nn);
                sv[j + 1] = h[SM_S + j + 1];
                H[(j + 1) * m + j] = hn;
                for (int i = 0; i < j; ++i) {
                    const double a = H[i * m + j], b = H[(i + 1) * m + j];
                    H[i * m + j] = cs[i] * a + sn[i] * b;
                    H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
                }
                const double a = H[j * m + j], b = H[(j + 1) * m + j];
                const double rr = std::hypot(a, b);
                cs[j] = rr > 0 ? a / rr : 1.0;
                sn[j] = rr > 0 ? b / rr : 0.0;
                H[j * m + j] = rr;
                H[(j + 1) * m + j] = 0.0;
                gvec[j + 1] = -sn[j] * gvec[j];
                gvec[j] = cs[j] * gvec[j];
                cols = j + 1;
                if (std::fabs(gvec[j + 1]) <= cycle_target || hn <= 1e-14 * std::sqrt(ww)) break;
            }
            // y = H^-1 g;  X += sum_i y_i s_i V_i
            Coefs cf;
            for (int i = cols - 1; i >= 0; --i) {
                double s = gvec[i];
                for (int l = i + 1; l < cols; ++l) s -= H[i * m + l] * y[l];
                y[i] = H[i * m + i] != 0 ? s / H[i * m + i] : 0.0;
            }
            for (int i = 0; i < cols; ++i) cf.a[i] = y[i] * sv[i];
            if (poly) {
                // X += (2I - B) z or M^-1 z, z = sum_i a_i V_i formed in the slot of V_cols (not part of
                // the combination)
                KT *z = V + (long long)cols * stride;
                S.timed(kUpd, 4 * Nd * kb * (cols + 1), [&] {
                    hipLaunchKernelGGL((k_combine<KT>), gf, bl, 0, S.st, z, V, stride, cols, cf, n4);
                });
                if (use_mg)
                    mg_precond(z, nullptr, 1.0, W);
                else
                    apply(z, nullptr, W, AT(2));
                Coefs one;
                one.a[0] = 1.0;
                S.timed(kUpd, 4 * Nd * (16 + kb),
                        [&] { hipLaunchKernelGGL((k_update_x<KT>), gf, bl, 0, S.st, X, W, stride, 1, one, n4); });
            } else {
                S.timed(kUpd, 4 * Nd * (16 + kb * cols),
                        [&] { hipLaunchKernelGGL((k_update_x<KT>), gf, bl, 0, S.st, X, V, stride, cols, cf, n4); });
            }
            RAD_TRY(residual());
            ++cycles;
            if (trace)
                std::fprintf(stderr, "[rad]   cycle: %d Arnoldi steps, estimate %.3e, true %.3e (target %.3e)\n", cols,
                             std::fabs(gvec[cols]), std::sqrt(nrm[4]), target);
            beta = std::sqrt(nrm[4]);
            // safeguard: a V-cycle-preconditioned cycle that gains less than 10% means the cycle is not
            // a preconditioner for this state (seen where many cells sit at the T >= 0 bound); the rest
            // of the step runs the Neumann operator, whose cycles are tested by the loop as before
            if (use_mg && beta > 0.9 * beta_prev) {
                use_mg = false;
                beta_prev = INFINITY;
                if (trace) std::fprintf(stderr, "[rad]   multigrid cycle stalled: Neumann operator from here\n");
            }
        }
        st.krylov_iters += its;

        // ---- exchange: per-cell Newton for T, diagnostics of the iteration
        const int aslot = aa_m > 0 ? k % (aa_m + 1) : 0;
        double *Gk = aa_m > 0 ? AAG + (size_t)aslot * N : nullptr, *fk = aa_m > 0 ? AAf + (size_t)aslot * N : nullptr;
        long long xrows = 0;
        S.timed(K_EXCHANGE, Nd * (2 * cb + 24 + 64 + 40 + (aa_m > 0 ? 16 : 0) + (Tfix ? 8 : 0)), [&] {
            for (int l = 0; l < NL; ++l) {
                const long long o = S.c0[l];
                if (vimp)   // one level: moving media run on the single grid only
                    hipLaunchKernelGGL((k_exchange<CT, true>), cell_grid(l), bl, 0, S.st, S.gl[l], rho, kP, S.Tn, Tc,
                                       X, X0, part, Gk, fk, (const double *)VA, (const double *)VB, S.En, p.mode,
                                       Tfix);
                else
                    hipLaunchKernelGGL((k_exchange<CT>), cell_grid(l), bl, 0, S.st, S.gl[l], rho + o, kP + o,
                                       S.Tn + o, Tc + o, X + 4 * o, X0 + 4 * o, part + xrows * 11,
                                       Gk ? Gk + o : nullptr, fk ? fk + o : nullptr, (const double *)nullptr,
                                       (const double *)nullptr, S.En + o, p.mode, Tfix ? Tfix + o : nullptr);
                xrows += cell_grid(l).x;
            }
        });
        S.reduce(xrows, 11, 11, sm + SM_RED, nullptr, -1, nullptr, 10);
        RAD_TRY(S.read(SM_RED, 11));
        const double *e = h + SM_RED;
        st.energy_defect = e[9] != 0.0 ? e[8] / e[9] : e[8];
        st.dE_max = e[10];
        exchanged = true;
        resT = e[1] > 0 ? std::sqrt(e[0] / e[1]) : std::sqrt(e[0]);
        const double e1 = e[1], e2 = e[2], e3 = e[3], e4 = e[4], e5 = e[5], e6 = e[6], e7 = e[7];
        if (aa_m > 0) {
            // Anderson mixing of the map values: restart the history when the map residual
            // grows a hundredfold over the best one seen (the mixing is then not helping)
            const double fn = std::sqrt(e2);
            if (fn > 1e2 * aa_best) aa_hist.clear();
            aa_best = std::min(aa_best, fn);
            int H = (int)aa_hist.size();
            if (H > 0) {
                AAHist hh{};
                for (int i = 0; i < H; ++i) {
                    hh.f[i] = AAf + (size_t)aa_hist[i] * N;
                    hh.G[i] = AAG + (size_t)aa_hist[i] * N;
                }
                const int nv = H * (H + 1) / 2 + H + 1;
                S.timed(K_EXCHANGE, Nd * 8 * (H + 1), [&] {
                    launch_aa_gram<kMaxAnderson>(H, gv, S.st, N, fk, hh, part);
                });
                S.reduce(S.L.nblk_vec, nv, nv, sm + SM_RED);
                RAD_TRY(S.read(SM_RED, nv));
                double D[kMaxAnderson * kMaxAnderson], b[kMaxAnderson], gam[kMaxAnderson];
                // the most recent H' <= H entries form the leading block; drop the oldest until it solves
                int Hs = H;
                for (; Hs > 0; --Hs) {
                    int q = 0;
                    for (int i = 0; i < H; ++i)
                        for (int j = i; j < H; ++j, ++q)
                            if (i < Hs && j < Hs) D[i * Hs + j] = D[j * Hs + i] = h[SM_RED + q];
                    for (int i = 0; i < Hs; ++i) b[i] = h[SM_RED + H * (H + 1) / 2 + i];
                    if (aa_solve(Hs, D, b, gam)) break;
                }
                if (Hs > 0) {
                    for (int i = 0; i < Hs; ++i) hh.gamma[i] = gam[i];
                    S.timed(K_EXCHANGE, Nd * (8 * (Hs + 1) + 2 * cb + 32), [&] {
                        for (int l = 0; l < NL; ++l) {
                            const long long o = S.c0[l];
                            AAHist hl = hh;
                            for (int i = 0; i < Hs; ++i) {
                                hl.f[i] = hh.f[i] + o;
                                hl.G[i] = hh.G[i] + o;
                            }
                            launch_aa_mix<CT, kMaxAnderson>(Hs, gv, S.st, S.gl[l], Gk + o, hl, rho + o, kP + o,
                                                            S.Tn + o, X + 4 * o, Tc + o, part + (long long)l * gv.x * 2);
                        }
                    });
                    S.reduce((long long)NL * gv.x, 2, 2, sm + SM_RED);
                    RAD_TRY(S.read(SM_RED, 2));
                    resT = h[SM_RED + 1] > 0 ? std::sqrt(h[SM_RED] / h[SM_RED + 1]) : std::sqrt(h[SM_RED]);
                }
            }
            aa_hist.insert(aa_hist.begin(), aslot);
            if ((int)aa_hist.size() > aa_m) aa_hist.pop_back();
        }
        const double cE = e4 > 0 ? std::sqrt(e3 / e4) : 0.0;
        const double cF = (e6 + e4) > 0 ? std::sqrt(e5) / (std::sqrt(e6) + std::sqrt(e4)) : 0.0;
        const double cT = e1 > 0 ? std::sqrt(e2 / e1) : 0.0;
        st.rel_change = std::max(cE, std::max(cF, cT));
        st.neg_cells = (int)e7;
        st.picard_iters = k + 1;
        if (trace)
            std::fprintf(stderr,
                         "[rad] picard %d: residual %.3e (E %.2e F %.2e T %.2e) -> krylov %d (total %d, cycles %d, "
                         "reorth %d), rel_change %.2e, neg %d\n",
                         k, res, st.res_E, st.res_F, resT, its, st.krylov_iters, cycles, reorth, st.rel_change,
                         st.neg_cells);
    }
    // the energy fix commits the gas temperature of the corrected energy (the last exchange's)
    const double *Tcommit = (Tfix && exchanged) ? Tfix : Tc;
    S.timed(K_COMMIT, Nd * 80, [&] {
        for (int l = 0; l < NL; ++l) {
            const long long o = S.c0[l];
            hipLaunchKernelGGL(k_commit, cell_grid(l), bl, 0, S.st, S.gl[l].N, g.c, X + 4 * o, Tcommit + o, S.E + o,
                               S.F + 3 * o, S.T + o);
        }
        if (S.amr) {
            const long long nb = (long long)(S.A.hi[0] - S.A.lo[0]) * (S.A.hi[1] - S.A.lo[1]) * (S.A.hi[2] - S.A.lo[2]);
            hipLaunchKernelGGL(k_amr_restrict, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, S.st, S.A, S.E, S.F,
                               S.T);
        }
    });
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(S.st));
    prof_resolve();
    st.status = status;
    if (status != RAD_OK)
        return fail(status, "not converged: scaled residual %.3e after %d Picard iterations", st.scaled_residual,
                    st.picard_iters);
    return RAD_OK;
}

double *pinned_staging()
{
    static thread_local double *buf = nullptr;
    if (!buf && hipHostMalloc((void **)&buf, SM_TOTAL * sizeof(double), hipHostMallocDefault) != hipSuccess)
        buf = nullptr;
    return buf;
}

template <class AT, class CT>
void launch_apply_phys(const Grid &g, const void *x, void *y, const void *dE, const void *rho, const void *kR,
                       const void *f, double c, hipStream_t st)
{
    const TileGeom tg = tile_geom<AT>(g);
    int wl = 0;
    for (int a = 0; a < 3; ++a) {
        wl = std::max(wl, ghost_face(g.bclo[a]) || ghost_face(g.bchi[a]) ? 1 : 0);
        wl = g.bclo[a] == BC_DIRICHLET || g.bchi[a] == BC_DIRICHLET ? 2 : wl;
    }
    auto kern = wl == 2   ? k_apply_tiled<AT, CT, false, false, false, true, 2>
                : wl == 1 ? k_apply_tiled<AT, CT, false, false, false, true, 1>
                          : k_apply_tiled<AT, CT, false>;
    hipLaunchKernelGGL(kern, dim3((unsigned)(tg.tiles_x * tg.tiles_y * tg.tiles_z)),
                       dim3(tile_threads<AT>()), 0, st, g, tg, (const CT *)f, (const AT *)nullptr, (const CT *)rho, (const CT *)kR,
                       (const AT *)nullptr, (const AT *)dE, (const AT *)x, (const double *)nullptr, (AT *)y,
                       (AT)(1.0 / c), (AT)c, AmrLv{}, (const AT *)nullptr, (const AT *)nullptr, AT(0), AT(1),
                       (const AT *)nullptr, AT(0), AT(1), (AT *)nullptr, MgFuse<AT>{}, (const AT *)nullptr);
}

}  // namespace

// ------------------------------------------------------------------ C ABI

// cells of the multigrid levels the configuration needs (0 unless krylov_poly = 2);
// fails when the grid has no coarse level
int mg_cells_for(int nx, int ny, int nz, const rad_params_t &p, long long &cells)
{
    cells = 0;
    if (p.krylov_poly != 2) return RAD_OK;
    if (mg_levels(nx, ny, nz, cells) < 2)
        return fail(RAD_EINVAL, "krylov_poly = 2 (multigrid) needs even grid extents of at least 8 cells");
    return RAD_OK;
}

extern "C" size_t rad_workspace_bytes(int nx, int ny, int nz, const rad_params_t *p)
{
    if (!p || nx < 1 || ny < 1 || nz < 1 || check_params(p) != RAD_OK) return 0;
    long long mgc = 0;
    if (mg_cells_for(nx, ny, nz, *p, mgc) != RAD_OK) return 0;
    return layout((long long)nx * ny * nz, *p, tile_bound(nx, ny, nz), false, false, mgc, wall_area(nx, ny, nz)).total;
}

namespace {

// autotune cache key of a single-grid configuration
std::string single_key(int nx, int ny, int nz, const int bc[6], const rad_params_t &p)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "single|%s|%dx%dx%d|p%d|c%d|bc%d%d%d%d%d%d", device_tag().c_str(), nx, ny, nz,
                  p.prec, p.coef_dtype, bc[0], bc[1], bc[2], bc[3], bc[4], bc[5]);
    return buf;
}

// tuned choices per key (apply z-range, residual z-range, face speeds read by the
// apply), read from the cache file once per process; entries are "kz_apply
// kz_res gmres_m loadc krylov_poly" (older ones without loadc read the stored speeds;
// gmres_m and krylov_poly are recommendations only)
struct Tuned {
    int kz_apply, kz_res, loadc;
};
std::mutex g_tile_mu;
std::map<std::string, Tuned> g_tiles;

void tile_lookup(const std::string &key, int &kz_apply, int &kz_res, int &loadc)
{
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tiles.find(key);
    if (it == g_tiles.end()) {
        std::string v;
        int a = 0, r = 0, m = 0, lc = 1;
        const int n = cache_get(key, v) ? std::sscanf(v.c_str(), "%d %d %d %d", &a, &r, &m, &lc) : 0;
        if (n < 2 || a < 1 || r < 1) a = r = 0;
        if (n < 4 || (lc != 0 && lc != 1)) lc = 1;
        it = g_tiles.emplace(key, Tuned{a, r, lc}).first;
    }
    kz_apply = it->second.kz_apply;
    kz_res = it->second.kz_res;
    loadc = it->second.loadc;
}

int dispatch_step(Solver &S)
{
    const bool mixed = S.p.prec == RAD_MIXED;
    if (S.p.coef_dtype == RAD_F64) return mixed ? run_step<double, float>(S) : run_step<double, double>(S);
    return mixed ? run_step<float, float>(S) : run_step<float, double>(S);
}

int init_solver(Solver &S, int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx, const int bc[6],
                const rad_params_t *p, void *workspace, size_t ws_bytes, void *stream, double *host = nullptr)
{
    RAD_TRY(check_grid_args(nx, ny, nz, dt, dx, bc, p, DIR_DATA));
    if (!E || !F || !T_gas || !rho || !kappa_P || !kappa_R || !f_ij) return fail(RAD_EINVAL, "NULL data pointer");
    if (!workspace) return fail(RAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace) % 256) return fail(RAD_EINVAL, "workspace must be 256-byte aligned");
    S.p = *p;
    long long mgc = 0;
    RAD_TRY(mg_cells_for(nx, ny, nz, *p, mgc));
    S.L = layout((long long)nx * ny * nz, *p, tile_bound(nx, ny, nz), false, false, mgc, wall_area(nx, ny, nz));
    if (ws_bytes < S.L.total) return fail(RAD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, S.L.total);
    S.host = host ? host : pinned_staging();
    if (!S.host) return fail(RAD_EHIP, "pinned host staging allocation failed");
    S.g = make_grid(nx, ny, nz, bc, dt, dx, *p);
    for (int a = 0; a < 6; ++a) {
        S.walls |= ghost_face(bc[a]);
        S.dirichlet |= bc[a] == RAD_BC_DIRICHLET;
    }
    S.nlev = 1;
    S.gl[0] = S.g;
    S.mgL = 1;
    S.mg[0] = S.g;
    if (p->krylov_poly == 2) {
        long long cells = 0;
        S.mgL = mg_levels(nx, ny, nz, cells);
        for (int l = 1; l < S.mgL; ++l) {
            S.mg[l] = make_grid(S.mg[l - 1].nx / 2, S.mg[l - 1].ny / 2, S.mg[l - 1].nz / 2, bc, dt,
                                dx * (double)(1 << l), *p);
            for (int f = 0; f < 6; ++f) S.mg[l].ghost[f] = nullptr;   // coarse operators take no data
        }
    }
    S.Ntot = S.g.N;
    S.st = (hipStream_t)stream;
    S.ws = (char *)workspace;
    S.rho = rho;
    S.kP = kappa_P;
    S.kR = kappa_R;
    S.f = f_ij;
    S.En = E;
    S.Fn = F;
    S.Tn = T_gas;
    S.E = E;
    S.F = F;
    S.T = T_gas;
    std::memset(&S.stats, 0, sizeof(S.stats));
    tile_lookup(single_key(nx, ny, nz, bc, *p), S.kz_apply, S.kz_res, S.loadc);
    return RAD_OK;
}

}  // namespace

namespace vr {
int step_with_staging(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                      const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                      const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes, void *stream,
                      rad_stats_t *stats, double *host)
{
    static_assert(SM_TOTAL <= kStagingDoubles, "host staging too small");
    clear_error();
    auto t0 = std::chrono::steady_clock::now();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Solver S;
    RAD_TRY(init_solver(S, nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, workspace, ws_bytes,
                        stream, host));
    int rc;
    try {  // small host vectors of the GMRES least-squares problem
        rc = dispatch_step(S);
    } catch (const std::bad_alloc &) {
        rc = fail(RAD_ENOMEM, "host memory");
    }
    S.stats.status = rc;
    S.stats.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S.stats;
    return rc;
}
}  // namespace vr

extern "C" int rad_step(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                        const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                        const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes, void *stream,
                        rad_stats_t *stats)
{
    return step_with_staging(nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, workspace, ws_bytes,
                             stream, stats, nullptr);
}

extern "C" size_t rad_workspace_bytes_moving(int nx, int ny, int nz, const rad_params_t *p)
{
    if (!p || nx < 1 || ny < 1 || nz < 1 || check_params(p) != RAD_OK) return 0;
    if (p->krylov_poly == 2) return (void)fail(RAD_EINVAL, "the moving-medium step has no multigrid Krylov operator"), 0;
    return layout((long long)nx * ny * nz, *p, tile_bound(nx, ny, nz), false, true, 0, wall_area(nx, ny, nz)).total;
}

extern "C" int rad_step_moving(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                               const void *kappa_P, const void *kappa_R, const void *f_ij, const void *beta, double dt,
                               double dx, const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes,
                               void *stream, rad_stats_t *stats)
{
    clear_error();
    auto t0 = std::chrono::steady_clock::now();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Solver S;
    RAD_TRY(check_grid_args(nx, ny, nz, dt, dx, bc, p, DIR_DATA));
    if (!beta) return fail(RAD_EINVAL, "beta (velocity) is NULL");
    if (p->vel_implicit && p->anderson_m > 0)
        return fail(RAD_EINVAL, "anderson_m must be 0 with vel_implicit = 1");
    if (p->energy_fix) return fail(RAD_EINVAL, "energy_fix: rad_step (no velocity) only");
    if (p->krylov_poly == 2) return fail(RAD_EINVAL, "the moving-medium step has no multigrid Krylov operator");
    RAD_TRY(init_solver(S, nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, workspace,
                        (size_t)-1, stream));
    S.L = layout(S.Ntot, *p, tile_bound(nx, ny, nz), false, true, 0, wall_area(nx, ny, nz));
    if (ws_bytes < S.L.total) return fail(RAD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, S.L.total);
    S.beta = beta;
    S.kz_apply = S.kz_res = 0;   // the velocity variants are not in the autotune cache
    S.loadc = 1;
    int rc;
    try {
        rc = dispatch_step(S);
    } catch (const std::bad_alloc &) {
        rc = fail(RAD_ENOMEM, "host memory");
    }
    S.stats.status = rc;
    S.stats.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S.stats;
    return rc;
}

namespace {

// Geometry of a two-level grid: its levels' grids, the box and the level-jump thread counts.
int amr_setup(const rad_amr2_t *geom, const int bc[6], double dt, double dx, const rad_params_t *p, Solver &S)
{
    if (!geom) return fail(RAD_EINVAL, "geometry is NULL");
    if (p && p->cv_cubic) return fail(RAD_EINVAL, "the two-level grid requires cv_cubic = 0");
    if (p && p->krylov_poly == 2) return fail(RAD_EINVAL, "the two-level grid has no multigrid Krylov operator");
    const int nc[3] = {geom->nx, geom->ny, geom->nz};
    RAD_TRY(check_grid_args(nc[0], nc[1], nc[2], dt, dx, bc, p, DIR_NO, false));
    if (p->energy_fix) return fail(RAD_EINVAL, "energy_fix: single-grid rad_step only");
    Amr &A = S.A;
    int fbc[6];
    for (int d = 0; d < 3; ++d) {
        const int lo = geom->lo[d], hi = geom->hi[d];
        const bool span = lo == 0 && hi == nc[d];
        if (!span && !(1 <= lo && lo < hi && hi <= nc[d] - 1))
            return fail(RAD_EINVAL, "refined box must span axis %d or stay one coarse cell inside it", d);
        A.lo[d] = lo;
        A.hi[d] = hi;
        A.nc[d] = nc[d];
        A.nf[d] = 2 * (hi - lo);
        A.jump[d] = span ? 0 : 1;
        fbc[2 * d] = span ? bc[2 * d] : RAD_BC_OUTFLOW;
        fbc[2 * d + 1] = span ? bc[2 * d + 1] : RAD_BC_OUTFLOW;
    }
    if ((long long)A.nf[0] * A.nf[1] > (1LL << 27)) return fail(RAD_EINVAL, "fine level nx * ny larger than 2^27");
    A.Nc = (long long)nc[0] * nc[1] * nc[2];
    A.Nf = (long long)A.nf[0] * A.nf[1] * A.nf[2];
    if (A.Nc + A.Nf > (1LL << 31)) return fail(RAD_EINVAL, "two-level grid larger than 2^31 cells");
    S.nlev = 2;
    S.amr = true;
    S.gl[0] = make_grid(nc[0], nc[1], nc[2], bc, dt, dx, *p);
    S.gl[1] = make_grid(A.nf[0], A.nf[1], A.nf[2], fbc, dt, 0.5 * dx, *p);
    S.g = S.gl[0];
    S.c0[0] = 0;
    S.c0[1] = A.Nc;
    S.Ntot = A.Nc + A.Nf;
    const long long a = A.nf[0], b = A.nf[1], c = A.nf[2];
    S.nshell = 2 * b * c + 2 * (a - 2) * c + 2 * (a - 2) * (b - 2);
    S.ncoarse = 0;
    for (int d = 0; d < 3; ++d) {
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        if (A.jump[d]) S.ncoarse += 2LL * (A.hi[e1] - A.lo[e1]) * (A.hi[e2] - A.lo[e2]);
    }
    return RAD_OK;
}

Layout amr_layout(const Solver &S, const rad_params_t &p)
{
    const Amr &A = S.A;
    return layout(S.Ntot, p, tile_bound(A.nc[0], A.nc[1], A.nc[2]) + tile_bound(A.nf[0], A.nf[1], A.nf[2]), true);
}

}  // namespace

extern "C" size_t rad_workspace_bytes_amr2(const rad_amr2_t *geom, const rad_params_t *p)
{
    Solver S;
    const int bc[6] = {RAD_BC_PERIODIC, RAD_BC_PERIODIC, RAD_BC_PERIODIC, RAD_BC_PERIODIC, RAD_BC_PERIODIC,
                       RAD_BC_PERIODIC};
    if (!p || amr_setup(geom, bc, 1.0, 1.0, p, S) != RAD_OK) {
        clear_error();
        return 0;
    }
    return amr_layout(S, *p).total;
}

extern "C" int rad_step_amr2(const rad_amr2_t *geom, double *E, double *F, double *T_gas, const void *rho,
                             const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                             const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes, void *stream,
                             rad_stats_t *stats)
{
    clear_error();
    auto t0 = std::chrono::steady_clock::now();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    Solver S;
    RAD_TRY(amr_setup(geom, bc, dt, dx, p, S));
    if (!E || !F || !T_gas || !rho || !kappa_P || !kappa_R || !f_ij) return fail(RAD_EINVAL, "NULL data pointer");
    if (!workspace) return fail(RAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace) % 256) return fail(RAD_EINVAL, "workspace must be 256-byte aligned");
    S.p = *p;
    S.L = amr_layout(S, *p);
    if (ws_bytes < S.L.total) return fail(RAD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, S.L.total);
    S.host = pinned_staging();
    if (!S.host) return fail(RAD_EHIP, "pinned host staging allocation failed");
    S.st = (hipStream_t)stream;
    S.ws = (char *)workspace;
    S.rho = rho;
    S.kP = kappa_P;
    S.kR = kappa_R;
    S.f = f_ij;
    S.En = S.E = E;
    S.Fn = S.F = F;
    S.Tn = S.T = T_gas;
    std::memset(&S.stats, 0, sizeof(S.stats));
    int rc;
    try {
        rc = dispatch_step(S);
    } catch (const std::bad_alloc &) {
        rc = fail(RAD_ENOMEM, "host memory");
    }
    S.stats.status = rc;
    S.stats.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S.stats;
    return rc;
}

namespace {
int autotune_step(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho, const void *kappa_P,
                  const void *kappa_R, const void *f_ij, double dt, double dx, const int bc[6], const rad_params_t *p,
                  void *workspace, size_t ws_bytes, void *stream, int tune_restart, int *kz_apply, int *kz_residual,
                  int *gmres_m, int *krylov_poly)
{
    Solver S;
    RAD_TRY(init_solver(S, nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, workspace, ws_bytes,
                        stream));
    // z-range candidates (planes per workgroup), clipped to the grid and deduplicated
    std::vector<int> cand;
    for (int kz : {8, 16, 32, 64, 128}) {
        const int k = std::min(kz, nz);
        if (std::find(cand.begin(), cand.end(), k) == cand.end()) cand.push_back(k);
    }
    S.tune_kz = &cand;
    RAD_TRY(dispatch_step(S));
    const int ka = S.tuned_apply, kr = S.tuned_res, lc = S.tuned_loadc;
    int best_m = p->gmres_m, best_poly = p->krylov_poly;
    if (tune_restart) {
        // full steps at each restart length the workspace allows, with and without the
        // Neumann polynomial, from the same state
        const size_t N = (size_t)nx * ny * nz;
        std::vector<double> save(5 * N);
        hipStream_t st = (hipStream_t)stream;
        HIP_TRY(hipMemcpyAsync(save.data(), E, N * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(save.data() + N, F, 3 * N * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(save.data() + 4 * N, T_gas, N * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        auto restore = [&]() -> int {
            HIP_TRY(hipMemcpyAsync(E, save.data(), N * 8, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(F, save.data() + N, 3 * N * 8, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(T_gas, save.data() + 4 * N, N * 8, hipMemcpyHostToDevice, st));
            HIP_TRY(hipStreamSynchronize(st));
            return RAD_OK;
        };
        std::vector<int> ms;
        for (int m : {6, 8, 10, 12, 16, 24, 32, 48, 64})
            if (m <= p->gmres_m) ms.push_back(m);
        if (std::find(ms.begin(), ms.end(), p->gmres_m) == ms.end()) ms.push_back(p->gmres_m);
        double best_t = INFINITY;
        // Krylov operators: the multigrid one too when the caller's workspace holds its levels
        std::vector<int> polys = {1, 0};
        if (p->krylov_poly == 2) polys.insert(polys.begin(), 2);
        for (int m : ms)
            for (int poly : polys) {
                RAD_TRY(restore());
                Solver T;
                RAD_TRY(init_solver(T, nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p,
                                    workspace, ws_bytes, stream));
                T.p.gmres_m = m;  // the layout keeps the caller's (largest) restart length
                T.p.krylov_poly = poly;
                T.kz_apply = ka;
                T.kz_res = kr;
                T.loadc = lc;
                const auto t0 = std::chrono::steady_clock::now();
                const int rc = dispatch_step(T);
                const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                if (rc < 0) {
                    (void)restore();
                    return rc;
                }
                clear_error();
                if (trace_enabled())
                    std::fprintf(stderr, "[rad] tune m=%d poly=%d: %.3f s, rc %d, %d Krylov\n", m, poly, sec, rc,
                                 T.stats.krylov_iters);
                if (rc == RAD_OK && sec < best_t) {
                    best_t = sec;
                    best_m = m;
                    best_poly = poly;
                }
            }
        RAD_TRY(restore());
    }
    const std::string key = single_key(nx, ny, nz, bc, *p);
    cache_put(key, std::to_string(ka) + " " + std::to_string(kr) + " " + std::to_string(best_m) + " " +
                       std::to_string(lc) + " " + std::to_string(best_poly));
    {
        std::lock_guard<std::mutex> lk(g_tile_mu);
        g_tiles[key] = Tuned{ka, kr, lc};
    }
    if (kz_apply) *kz_apply = ka;
    if (kz_residual) *kz_residual = kr;
    if (gmres_m) *gmres_m = best_m;
    if (krylov_poly) *krylov_poly = best_poly;
    return RAD_OK;
}
}  // namespace

extern "C" int rad_autotune_step(int nx, int ny, int nz, double *E, double *F, double *T_gas, const void *rho,
                                 const void *kappa_P, const void *kappa_R, const void *f_ij, double dt, double dx,
                                 const int bc[6], const rad_params_t *p, void *workspace, size_t ws_bytes,
                                 void *stream, int tune_restart, int *kz_apply, int *kz_residual, int *gmres_m,
                                 int *krylov_poly)
{
    clear_error();
    try {  // the host copy of the state is the one large host allocation
        return autotune_step(nx, ny, nz, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dt, dx, bc, p, workspace, ws_bytes,
                             stream, tune_restart, kz_apply, kz_residual, gmres_m, krylov_poly);
    } catch (const std::bad_alloc &) {
        return fail(RAD_ENOMEM, "host memory for the autotuner's copy of the state");
    }
}

extern "C" int rad_residual(int nx, int ny, int nz, const double *E_n, const double *F_n, const double *T_n,
                            const double *E, const double *F, const double *T, const void *rho, const void *kappa_P,
                            const void *kappa_R, const void *f_ij, double dt, double dx, const int bc[6],
                            const rad_params_t *p, double *R, void *stream)
{
    clear_error();
    RAD_TRY(check_grid_args(nx, ny, nz, dt, dx, bc, p, DIR_DATA));
    if (!E_n || !F_n || !T_n || !E || !F || !T || !rho || !kappa_P || !kappa_R || !f_ij || !R)
        return fail(RAD_EINVAL, "NULL data pointer");
    Grid g = make_grid(nx, ny, nz, bc, dt, dx, *p);
    const dim3 gc((unsigned)((g.N + kBlock - 1) / kBlock)), bl(kBlock);
    hipStream_t st = (hipStream_t)stream;
    // the state's own temperature is the emission temperature: lagged form, T* = T
    if (p->coef_dtype == RAD_F64)
        hipLaunchKernelGGL((k_residual<double, double, double, RES_PHYSICAL>), gc, bl, 0, st, g, 0, E_n, F_n, T_n, T,
                           (const double *)rho, (const double *)kappa_P, (const double *)kappa_R,
                           (const double *)f_ij, E, F, 1.0 / p->c, (double *)nullptr, (double *)nullptr, R,
                           (double *)nullptr);
    else
        hipLaunchKernelGGL((k_residual<float, double, double, RES_PHYSICAL>), gc, bl, 0, st, g, 0, E_n, F_n, T_n, T,
                           (const float *)rho, (const float *)kappa_P, (const float *)kappa_R, (const float *)f_ij,
                           E, F, 1.0 / p->c, (double *)nullptr, (double *)nullptr, R, (double *)nullptr);
    HIP_TRY(hipGetLastError());
    return RAD_OK;
}

extern "C" int rad_face_speeds(int nx, int ny, int nz, const void *rho, const void *kappa_R, const void *f_ij,
                               double dx, const int bc[6], const rad_params_t *p, double *C, void *stream)
{
    clear_error();
    RAD_TRY(check_grid_args(nx, ny, nz, 1.0, dx, bc, p, DIR_ANY));
    if (!rho || !kappa_R || !f_ij || !C) return fail(RAD_EINVAL, "NULL data pointer");
    // the wave speed does not depend on dt: evaluate with dt = dx / c (nu = 1)
    Grid g = make_grid(nx, ny, nz, bc, dx / p->c, dx, *p);
    const dim3 gc((unsigned)((g.N + kBlock - 1) / kBlock)), bl(kBlock);
    hipStream_t st = (hipStream_t)stream;
    if (p->coef_dtype == RAD_F64)
        hipLaunchKernelGGL((k_face_speeds<double>), gc, bl, 0, st, g, (const double *)rho, (const double *)kappa_R,
                           (const double *)f_ij, C);
    else
        hipLaunchKernelGGL((k_face_speeds<float>), gc, bl, 0, st, g, (const float *)rho, (const float *)kappa_R,
                           (const float *)f_ij, C);
    HIP_TRY(hipGetLastError());
    return RAD_OK;
}

extern "C" int rad_apply(int nx, int ny, int nz, const void *x, void *y, const void *dE, const void *rho,
                         const void *kappa_R, const void *f_ij, double dt, double dx, const int bc[6],
                         const rad_params_t *p, int dtype, void *stream)
{
    clear_error();
    RAD_TRY(check_grid_args(nx, ny, nz, dt, dx, bc, p, DIR_ANY));
    if (!x || !y || !dE || !rho || !kappa_R || !f_ij) return fail(RAD_EINVAL, "NULL data pointer");
    if (dtype != RAD_F64 && dtype != RAD_F32) return fail(RAD_EINVAL, "dtype must be RAD_F64 or RAD_F32");
    Grid g = make_grid(nx, ny, nz, bc, dt, dx, *p);
    hipStream_t st = (hipStream_t)stream;
    const bool c32 = p->coef_dtype == RAD_F32;
    if (dtype == RAD_F64) {
        if (c32)
            launch_apply_phys<double, float>(g, x, y, dE, rho, kappa_R, f_ij, p->c, st);
        else
            launch_apply_phys<double, double>(g, x, y, dE, rho, kappa_R, f_ij, p->c, st);
    } else {
        if (c32)
            launch_apply_phys<float, float>(g, x, y, dE, rho, kappa_R, f_ij, p->c, st);
        else
            launch_apply_phys<float, double>(g, x, y, dE, rho, kappa_R, f_ij, p->c, st);
    }
    HIP_TRY(hipGetLastError());
    return RAD_OK;
}

extern "C" int rad_exchange(long long n, const double *E, const double *T_n, double *T, const void *rho,
                            const void *kappa_P, double dt, const rad_params_t *p, void *stream)
{
    clear_error();
    if (!p) return fail(RAD_EINVAL, "params is NULL");
    RAD_TRY(check_params(p));
    if (n < 1) return fail(RAD_EINVAL, "n must be >= 1");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(RAD_EINVAL, "dt must be positive and finite");
    if (!E || !T_n || !T || !rho || !kappa_P) return fail(RAD_EINVAL, "NULL data pointer");
    Grid g;
    std::memset(&g, 0, sizeof(g));
    g.N = n;
    g.cdt = p->c * dt;
    g.aR = p->a_R;
    g.cv = p->c_v;
    g.c = p->c;
    g.cv_cubic = p->cv_cubic;
    const dim3 gc((unsigned)((n + kBlock - 1) / kBlock)), bl(kBlock);
    hipStream_t st = (hipStream_t)stream;
    if (p->coef_dtype == RAD_F64)
        hipLaunchKernelGGL((k_exchange_only<double>), gc, bl, 0, st, n, g, (const double *)rho,
                           (const double *)kappa_P, E, T_n, T);
    else
        hipLaunchKernelGGL((k_exchange_only<float>), gc, bl, 0, st, n, g, (const float *)rho, (const float *)kappa_P,
                           E, T_n, T);
    HIP_TRY(hipGetLastError());
    return RAD_OK;
}
