// rad_amr.h -- the two-level composite grid (one box refined by 2) on gfx950.
//
// Sec. 2.3.3 (eq. wavespeedtau, eq. interface_flux): each level runs the
// uniform-grid tile sweep unchanged -- the fine level with zero-gradient faces
// where its box ends inside the domain, the coarse level over all its cells --
// and k_amr_jump computes, per level-jump face, the HLL flux with the upstream
// optical depth.  The sweeps' epilogues then add, before the Jacobi scaling,
//   fine cell at a jump:     c dt / h_f (Phi_jump - Phi_self)   (replaces the zero-gradient face)
//   coarse cell at a jump:   c dt / H (mean of its 4 fine Phi_jump - Phi_coarse)
// and drop the transport of covered coarse cells (isolated-cell rows).  The
// Jacobi diagonal follows the composite operator too: a jump cell's diagonal
// gains the jump faces' diffusive coefficients in place of the sweep's
// (fifth correction plane); a covered cell's is its local diagonal.  The
// corrections are stored per cell in a level-blocked FP64 array (5 planes)
// that only jump cells write and read, so the sweeps' traffic grows with the
// box's surface, not its volume.
#pragma once

#include "rad_device.h"

#include <type_traits>

namespace vr {

// Refined box [lo, hi) in coarse cells; an axis that the box spans entirely
// (lo = 0, hi = n) has no level jumps and the fine level takes the domain's
// boundary there.  nf = 2 (hi - lo).
struct Amr {
    int lo[3], hi[3], nf[3], jump[3];
    int nc[3];
    long long Nc, Nf;
};

// Per-level view handed to a sweep: lev 0 coarse, 1 fine; corr points at this
// level's block of the correction array (5 planes of the level's cell count:
// the four transport corrections, then the change of the Jacobi diagonal), in
// the sweep's arithmetic precision.
struct AmrLv {
    Amr a;
    int lev;
    const void *corr;
};

enum { AMR_PLAIN = 0, AMR_COVERED = 1, AMR_JUMP = 2 };

__device__ __forceinline__ int amr_role(const AmrLv &L, int i, int j, int k)
{
    const int p[3] = {i, j, k};
    if (L.lev == 0) {
        int out = 0, od = -1;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (p[d] < L.a.lo[d] || p[d] >= L.a.hi[d]) {
                ++out;
                od = d;
            }
        if (out == 0) return AMR_COVERED;
        if (out == 1 && L.a.jump[od] && (p[od] == L.a.lo[od] - 1 || p[od] == L.a.hi[od])) return AMR_JUMP;
        return AMR_PLAIN;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (L.a.jump[d] && (p[d] == 0 || p[d] == L.a.nf[d] - 1)) return AMR_JUMP;
    return AMR_PLAIN;
}

// sqrt((1 - e^-tau) / tau) with its limits 1 (tau = 0) and 0 (tau = inf)
__device__ __forceinline__ double tau_factor(double tau)
{
    if (tau == 0.0) return 1.0;
    if (isinf(tau)) return 0.0;
    return sqrt(-expm1(-tau) / tau);
}

// One cell's state as seen by a face along axis d
struct JCell {
    double E, F[3], fr[3], tau;
};

// HLL flux (divided by c) with unequal speeds at a level jump: C^R from the
// left cell's tau, C^L from the right cell's (the upstream optical depths),
// sqrt(max f_dd) as at every face; with C^L + C^R = 0 the central flux.  g:
// the flux's diffusive coefficient C^L C^R / (C^L + C^R) (its diagonal part).
__device__ __forceinline__ void jump_flux(int d, const JCell &L, const JCell &R, double (&phi)[4], double &gd)
{
    const double root = sqrt(fmax(L.fr[d], R.fr[d]));
    const double CR = root * tau_factor(L.tau), CL = root * tau_factor(R.tau);
    const double S = CL + CR;
    double aL = 0.5, aR = 0.5, g = 0.0;
    if (S > 0) {
        aL = CR / S;
        aR = CL / S;
        g = CL * CR / S;
    }
    phi[0] = aL * L.F[d] + aR * R.F[d] - g * (R.E - L.E);
#pragma unroll
    for (int q = 0; q < 3; ++q) phi[1 + q] = aL * L.fr[q] * L.E + aR * R.fr[q] * R.E - g * (R.F[q] - L.F[q]);
    gd = g;
}

namespace {

// Corrections of every jump cell.  Threads [0, nshell) take the cells on the
// fine box's surface (each writes its own cell), the rest the coarse cells
// next to the box (each computes its four fine fluxes again, so no thread
// writes another's cell and no atomics are needed).  x is one state vector
// of either level block (E, Ft planes; FT the Krylov or the FP64 precision)
// scaled by *xs when given; Cc the coarse level's stored low-face speeds of
// the sweep whose coarse-coarse flux across a covered face is replaced.
template <class XT, class CT, class FT, class OT>
__global__ void __launch_bounds__(256)
    k_amr_jump(Amr a, Grid gc, Grid gf, long long nshell, long long ncoarse, const XT *__restrict__ x,
               const double *__restrict__ xs, const CT *__restrict__ f, const double *__restrict__ sR,
               const FT *__restrict__ Cc, OT *__restrict__ corr)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nshell + ncoarse) return;
    const double s = xs ? *xs : 1.0;
    const long long Nc = a.Nc, Nf = a.Nf;
    const XT *xc = x, *xf = x + 4 * Nc;   // state vectors: 4 planes per level
    const CT *fc = f, *ff = f + 6 * Nc;
    const double *sRc = sR, *sRf = sR + Nc;
    auto cidx = [&](int i, int j, int k) { return (long long)i + (long long)a.nc[0] * (j + (long long)a.nc[1] * k); };
    auto fidx = [&](int i, int j, int k) { return (long long)i + (long long)a.nf[0] * (j + (long long)a.nf[1] * k); };
    auto load = [&](const XT *xl, const CT *fl, const double *sl, long long N, long long c, int d, double tk,
                    JCell &u) {
        u.E = s * (double)xl[c];
#pragma unroll
        for (int q = 0; q < 3; ++q) u.F[q] = s * (double)xl[(1 + q) * N + c];
#pragma unroll
        for (int q = 0; q < 3; ++q) u.fr[q] = (double)fl[tens_row(d, q) * N + c];
        const double sr = sl[c], fdd = u.fr[d];
        u.tau = sr == 0.0 ? 0.0 : (fdd == 0.0 ? (double)INFINITY : tk * sr * sr / fdd);
    };
    if (t < nshell) {
        // fine surface cell: faces x-normal first, then y-normal (x interior), then z-normal
        const int A = a.nf[0], B = a.nf[1], C = a.nf[2];
        long long r = t;
        int p[3];
        if (r < 2LL * B * C) {
            const long long side = r / ((long long)B * C), q = r % ((long long)B * C);
            p[0] = side ? A - 1 : 0;
            p[1] = (int)(q % B);
            p[2] = (int)(q / B);
        } else if ((r -= 2LL * B * C) < 2LL * (A - 2) * C) {
            const long long side = r / ((long long)(A - 2) * C), q = r % ((long long)(A - 2) * C);
            p[1] = side ? B - 1 : 0;
            p[0] = 1 + (int)(q % (A - 2));
            p[2] = (int)(q / (A - 2));
        } else {
            r -= 2LL * (A - 2) * C;
            const long long side = r / ((long long)(A - 2) * (B - 2)), q = r % ((long long)(A - 2) * (B - 2));
            p[2] = side ? C - 1 : 0;
            p[0] = 1 + (int)(q % (A - 2));
            p[1] = 1 + (int)(q / (A - 2));
        }
        const long long cf = fidx(p[0], p[1], p[2]);
        double acc[5] = {0, 0, 0, 0, 0};
        bool any = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (!a.jump[d]) continue;
            const bool lo_side = p[d] == 0, hi_side = p[d] == a.nf[d] - 1;
            if (!lo_side && !hi_side) continue;
            any = true;
            int pc[3] = {a.lo[0] + p[0] / 2, a.lo[1] + p[1] / 2, a.lo[2] + p[2] / 2};
            pc[d] = hi_side ? a.hi[d] : a.lo[d] - 1;
            JCell uf, uc;
            load(xf, ff, sRf, Nf, cf, d, gf.tau_k, uf);
            load(xc, fc, sRc, Nc, cidx(pc[0], pc[1], pc[2]), d, gc.tau_k, uc);
            double phi[4], gd;
            if (hi_side)
                jump_flux(d, uf, uc, phi, gd);
            else
                jump_flux(d, uc, uf, phi, gd);
            acc[4] += gf.nu * gd;   // the sweep's zero-gradient face added nothing to the diagonal
            // the sweep's zero-gradient face carried the cell's own physical flux
            const double self[4] = {uf.F[d], uf.fr[0] * uf.E, uf.fr[1] * uf.E, uf.fr[2] * uf.E};
            const double sg = hi_side ? gf.nu : -gf.nu;
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += sg * (phi[q] - self[q]);
        }
        if (any) {
            OT *cr = corr + 5 * Nc;
#pragma unroll
            for (int q = 0; q < 5; ++q) cr[q * Nf + cf] = (OT)acc[q];
        }
        return;
    }
    // coarse cell next to the box across axis d: t enumerates, per jump axis, the low then the high layer
    long long r = t - nshell;
    int d = 0;
    long long layer = 0;
    for (d = 0; d < 3; ++d) {
        if (!a.jump[d]) continue;
        const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
        layer = (long long)(a.hi[e1] - a.lo[e1]) * (a.hi[e2] - a.lo[e2]);
        if (r < 2 * layer) break;
        r -= 2 * layer;
    }
    if (d == 3) return;
    // one body per axis, so that every index below is a compile-time constant (no stack arrays)
    auto coarse = [&](auto axis) {
        constexpr int D = decltype(axis)::value, e1 = D == 0 ? 1 : 0, e2 = D == 2 ? 1 : 2;
        const bool box_above = r < layer;  // the coarse cell sits below the box (its high face is covered)
        const long long q = box_above ? r : r - layer;
        const int w1 = a.hi[e1] - a.lo[e1];
        int pc[3];
        pc[e1] = a.lo[e1] + (int)(q % w1);
        pc[e2] = a.lo[e2] + (int)(q / w1);
        pc[D] = box_above ? a.lo[D] - 1 : a.hi[D];
        int pk[3] = {pc[0], pc[1], pc[2]};
        pk[D] = box_above ? a.lo[D] : a.hi[D] - 1;   // the covered neighbour
        const long long cc = cidx(pc[0], pc[1], pc[2]), ck = cidx(pk[0], pk[1], pk[2]);
        JCell uc, uk;
        load(xc, fc, sRc, Nc, cc, D, gc.tau_k, uc);
        load(xc, fc, sRc, Nc, ck, D, gc.tau_k, uk);
        double mean[4] = {0, 0, 0, 0}, gmean = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int p[3];
            p[e1] = 2 * (pc[e1] - a.lo[e1]) + (m & 1);
            p[e2] = 2 * (pc[e2] - a.lo[e2]) + (m >> 1);
            p[D] = box_above ? 0 : a.nf[D] - 1;
            JCell uf;
            load(xf, ff, sRf, Nf, fidx(p[0], p[1], p[2]), D, gf.tau_k, uf);
            double phi[4], gd;
            if (box_above)
                jump_flux(D, uc, uf, phi, gd);
            else
                jump_flux(D, uf, uc, phi, gd);
#pragma unroll
            for (int k = 0; k < 4; ++k) mean[k] += 0.25 * phi[k];
            gmean += 0.25 * gd;
        }
        // the coarse sweep's flux across the covered face: uniform HLLE with its stored speed
        const JCell &L = box_above ? uc : uk, &R = box_above ? uk : uc;
        const double Cu = (double)Cc[D * Nc + (box_above ? ck : cc)];
        double phic[4];
        phic[0] = 0.5 * (L.F[D] + R.F[D]) - 0.5 * Cu * (R.E - L.E);
#pragma unroll
        for (int k = 0; k < 3; ++k)
            phic[1 + k] = 0.5 * (L.fr[k] * L.E + R.fr[k] * R.E) - 0.5 * Cu * (R.F[k] - L.F[k]);
        const double sg = box_above ? gc.nu : -gc.nu;
#pragma unroll
        for (int k = 0; k < 4; ++k) corr[k * Nc + cc] = (OT)(sg * (mean[k] - phic[k]));
        corr[4 * Nc + cc] = (OT)(gc.nu * (gmean - 0.5 * Cu));
    };
    if (d == 0)
        coarse(std::integral_constant<int, 0>{});
    else if (d == 1)
        coarse(std::integral_constant<int, 1>{});
    else
        coarse(std::integral_constant<int, 2>{});
}

// Covered coarse cells := mean of their eight children (E, F, T), after the commit.
__global__ void __launch_bounds__(256)
    k_amr_restrict(Amr a, double *__restrict__ E, double *__restrict__ F, double *__restrict__ T)
{
    const int bx = a.hi[0] - a.lo[0], by = a.hi[1] - a.lo[1], bz = a.hi[2] - a.lo[2];
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)bx * by * bz) return;
    const int i = a.lo[0] + (int)(t % bx), j = a.lo[1] + (int)((t / bx) % by), k = a.lo[2] + (int)(t / ((long long)bx * by));
    const long long Nc = a.Nc, Nf = a.Nf;
    const long long cc = i + (long long)a.nc[0] * (j + (long long)a.nc[1] * k);
    double sE = 0, sF[3] = {0, 0, 0}, sT = 0;
    for (int m = 0; m < 8; ++m) {
        const int fi = 2 * (i - a.lo[0]) + (m & 1), fj = 2 * (j - a.lo[1]) + ((m >> 1) & 1),
                  fk = 2 * (k - a.lo[2]) + (m >> 2);
        const long long cf = Nc + fi + (long long)a.nf[0] * (fj + (long long)a.nf[1] * fk);
        sE += E[cf];
        sT += T[cf];
        for (int q = 0; q < 3; ++q) sF[q] += F[3 * Nc + q * Nf + (cf - Nc)];
    }
    E[cc] = 0.125 * sE;
    T[cc] = 0.125 * sT;
    for (int q = 0; q < 3; ++q) F[q * Nc + cc] = 0.125 * sF[q];
}

}  // namespace

}  // namespace vr
