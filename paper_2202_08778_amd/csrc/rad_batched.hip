// rad_batched.hip -- many independent blocks in one persistent launch (gfx950).
//
// Each block is an n^3 interior with ghost layers of fixed Dirichlet data (E,
// F and its own rho, kappa, f); the first ghost layer enters the first-order
// stencil.  A persistent grid of workgroups pops block indices from a queue
// ordered largest first (longest-processing-time first) and solves each
// block entirely inside one workgroup: FP64 residual of the Picard linear
// system, restarted GMRES(m) with workgroup-level reductions (Arnoldi in FP32
// or FP64; on the Jacobi-scaled operator times the Neumann polynomial 2I - B
// unless krylov_poly = 0), FP64 solution accumulation and refinement, per-cell FP64 exchange
// solve, and the same convergence test as the single-grid step.  Every loop is
// bounded (max_picard, max_krylov, m) and the queue ends every workgroup, so
// the grid always drains.  The launch (queue reset + persistent kernel) is a
// HIP graph rebuilt only when the plan changes; each step updates the kernel
// node's arguments and replays it.
#include "rad_host.h"
#include "rad_apply_tiled.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>


using namespace vr;

namespace {

struct BatchArgs {
    const rad_block_desc_t *desc;  // device copy of the caller's descriptors
    const int *order;              // block ids in processing order
    int nblocks;
    long long arena;               // elements per arena (stride between F / f component arenas)
    double *E, *F, *T;
    const void *rho, *kP, *kR, *f;
    rad_stats_t *stats;
    char *slots;
    long long slot_bytes;
    int *queue;
    double c, aR, cv, tol, eps_R;
    int max_picard, max_krylov, m, mode, poly;
    double clk_khz;                // rate of the device wall clock (per-block solve times; 0: not timed)
};

// per-slot scratch layout for a block of up to nmax^3 cells
struct SlotLayout {
    size_t X, X0, Tc, sR, dE, Cs, Cs64, V, W, total;
};

__host__ __device__ SlotLayout slot_layout(int nmax, int m, size_t kb)
{
    const size_t N = (size_t)nmax * nmax * nmax;
    SlotLayout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t at = o;
        o += align_up(b);
        return at;
    };
    L.X = take(4 * N * 8);
    L.X0 = take(4 * N * 8);
    L.Tc = take(N * 8);
    L.sR = take(N * kb);
    L.dE = take(N * kb);
    L.Cs = take(6 * N * kb);  // corrected speeds of the six faces of every interior cell
    L.Cs64 = take(kb == 8 ? 0 : 6 * N * 8);  // the same in FP64 for the residual (FP32 Krylov only)
    L.V = take((size_t)(m + 1) * 4 * N * kb);
    L.W = take(4 * N * kb);
    L.total = o;
    return L;
}

// geometry of one block
struct Blk {
    int n, ng, M, Nb;
    long long base;
    double nu, cdt, tau_k;
    __device__ long long p(int i, int j, int k) const
    {
        return base + (i + ng) + (long long)M * ((j + ng) + (long long)M * (k + ng));
    }
};

// Workgroup sum of NV values; every thread receives the sums.
template <int NT, int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double *red)
{
    constexpr int W = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) red[q * W + wid] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) t += red[q * W + w];
        v[q] = t;
    }
    __syncthreads();
}

// Transport part at interior cell (i,j,k) of a block, with the corrected face
// speeds given (cs(d, side) for face (d, side)); neighbours outside the interior
// are the first ghost layer.  Loaders take offsets (di, dj, dk).
template <class T, class LD, class FL, class CS>
__device__ __forceinline__ void transport_blk_pre(T nu, LD ld, FL fl, CS cs, T div[4], T &sumC)
{
    const T Ec = ld(0, 0, 0, 0);
    const T Fc[3] = {ld(1, 0, 0, 0), ld(2, 0, 0, 0), ld(3, 0, 0, 0)};
    T dE = 0, dF[3] = {0, 0, 0};
    sumC = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T fcr[3] = {fl(tens_row(d, 0), 0, 0, 0), fl(tens_row(d, 1), 0, 0, 0), fl(tens_row(d, 2), 0, 0, 0)};
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int o = side ? 1 : -1;
            const int di = d == 0 ? o : 0, dj = d == 1 ? o : 0, dk = d == 2 ? o : 0;
            const T En = ld(0, di, dj, dk);
            const T Fn[3] = {ld(1, di, dj, dk), ld(2, di, dj, dk), ld(3, di, dj, dk)};
            const T fnr[3] = {fl(tens_row(d, 0), di, dj, dk), fl(tens_row(d, 1), di, dj, dk),
                              fl(tens_row(d, 2), di, dj, dk)};
            const T C = cs(d, side);
            sumC += C;
            face_flux_acc<T>(d, side, C, Ec, Fc, fcr, En, Fn, fnr, dE, dF);
        }
    }
    div[0] = nu * dE;
    div[1] = nu * dF[0];
    div[2] = nu * dF[1];
    div[3] = nu * dF[2];
}

__device__ __forceinline__ void cell_of(int c, int n, int &i, int &j, int &k)
{
    const int q = c / n;
    i = c - q * n;
    k = q / n;
    j = q - k * n;
}

// Plane-marching form of the block apply (FP32, n <= 32), kept out of line so
// that it has its own register allocation: the thread owns plane positions
// q = tid, tid + NT; planes stream through three LDS slots (plane p in slot
// p % 3), the next-but-one plane is fetched into registers while the current
// one is computed, so each x and f value is read from memory once per apply and
// the lateral and vertical neighbours come from LDS.  Neighbours outside the
// block carry a zero correction (the ghosts are fixed data), so their tensor
// multiplies zero.  spl: 3 x 10 x 1024 floats of LDS.
template <class CT, int NT>
__device__ __noinline__ void apply_planes(Blk B, int n, int Nb, long long AR, const CT *__restrict__ f,
                                          const float *__restrict__ x, float s, const float *__restrict__ Cs,
                                          const float *__restrict__ sR, const float *__restrict__ dEv,
                                          float *__restrict__ y, float *spl_, float pg)
{
    using KT = float;
    auto spl = reinterpret_cast<float(*)[10][32 * 32]>(spl_);
    constexpr int QP = (32 * 32 + NT - 1) / NT;
    const int tid = threadIdx.x;
    const int n2 = n * n;
    const KT nu = (KT)B.nu, half = KT(0.5) * (KT)B.nu;
    KT R[QP][10];
    auto fetch = [&](int k) {
#pragma unroll
        for (int u = 0; u < QP; ++u) {
            const int q = tid + u * NT;
            if (q < n2) {
                const int c = q + n2 * k;
#pragma unroll
                for (int t = 0; t < 4; ++t) R[u][t] = s * x[t * Nb + c];
                const long long p = B.p(q % n, q / n, k);
#pragma unroll
                for (int t = 0; t < 6; ++t) R[u][4 + t] = (KT)f[t * AR + p];
            }
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int u = 0; u < QP; ++u) {
            const int q = tid + u * NT;
            if (q < n2)
#pragma unroll
                for (int t = 0; t < 10; ++t) spl[slot][t][q] = R[u][t];
        }
    };
    fetch(0);
    store(0);
    if (n > 1) {
        fetch(1);
        store(1);
    }
    lds_barrier();
    for (int k = 0; k < n; ++k) {
        if (k + 2 < n) fetch(k + 2);
        const int a = k % 3, lo = (k + 2) % 3, hi = (k + 1) % 3;
#pragma unroll 1
        for (int u = 0; u < QP; ++u) {
            const int q = tid + u * NT;
            if (q >= n2) continue;
            const int i = q % n, j = q / n, c = q + n2 * k;
            auto ld = [&](int t, int di, int dj, int dk) -> KT {
                if (dk) return (unsigned)(k + dk) < (unsigned)n ? spl[dk > 0 ? hi : lo][t][q] : KT(0);
                if ((unsigned)(i + di) >= (unsigned)n || (unsigned)(j + dj) >= (unsigned)n) return KT(0);
                return spl[a][t][q + di + n * dj];
            };
            auto fl = [&](int t, int di, int dj, int dk) -> KT {
                if (dk) return (unsigned)(k + dk) < (unsigned)n ? spl[dk > 0 ? hi : lo][4 + t][q] : spl[a][4 + t][q];
                if ((unsigned)(i + di) >= (unsigned)n || (unsigned)(j + dj) >= (unsigned)n) return spl[a][4 + t][q];
                return spl[a][4 + t][q + di + n * dj];
            };
            auto cs = [&](int d, int side) -> KT { return Cs[(2 * d + side) * Nb + c]; };
            KT div[4], sumC;
            transport_blk_pre<KT>(nu, ld, fl, cs, div, sumC);
            const KT sRc = sR[c], dEc = dEv[c];
            const KT xc = ld(0, 0, 0, 0);
            const KT yE = (dEc * xc + div[0]) / (dEc + half * sumC);
            y[c] = pg != KT(0) ? pg * xc - yE : yE;
            const KT DF = KT(1) + sRc + half * sumC;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const KT xq = ld(1 + t, 0, 0, 0);
                const KT yq = ((KT(1) + sRc) * xq + div[1 + t]) / DF;
                y[(1 + t) * Nb + c] = pg != KT(0) ? pg * xq - yq : yq;
            }
        }
        lds_barrier();
        if (k + 2 < n) store((k + 2) % 3);
        lds_barrier();
    }
}

template <class CT, class KT, int NT>
__global__ void __launch_bounds__(NT) k_batched(BatchArgs a)
{
    constexpr int W = NT / 64;
    constexpr int DC = 8;  // basis vectors per multi-dot pass
    __shared__ double red[16 * W];
    __shared__ double sh_dots[kMaxM + DC], sh_s[kMaxM + 2], sh_a[kMaxM + 1], sh_y[kMaxM];
    __shared__ double sh_H[(kMaxM + 1) * kMaxM], sh_cs[kMaxM], sh_sn[kMaxM], sh_g[kMaxM + 1];
    __shared__ int sh_flag, sh_b;
    // planes k-1, k, k+1 of the marching apply (FP32 blocks up to 32^3): x (4) and f (6)
    constexpr int PL = sizeof(KT) == 4 ? 32 * 32 : 1;
    __shared__ KT spl[3][10][PL];

    const CT *rho = (const CT *)a.rho, *kP = (const CT *)a.kP, *kR = (const CT *)a.kR, *f = (const CT *)a.f;
    const long long AR = a.arena;
    const int m = a.m;
    const int tid = threadIdx.x;
    char *slot = a.slots + (long long)blockIdx.x * a.slot_bytes;

    for (;;) {
        if (tid == 0) sh_b = atomicAdd(a.queue, 1);
        __syncthreads();
        // the same value in every lane: say so, so that block-derived sizes and
        // pointers live in scalar registers
        const int qi = __builtin_amdgcn_readfirstlane(sh_b);
        __syncthreads();
        if (qi >= a.nblocks) break;
        const int bid = a.order[qi];
        const long long t_start = wall_clock64();
        const rad_block_desc_t ds = a.desc[bid];
        Blk B;
        B.n = ds.n;
        B.ng = ds.ng;
        B.M = ds.n + 2 * ds.ng;
        B.Nb = ds.n * ds.n * ds.n;
        B.base = ds.off;
        B.cdt = a.c * ds.dt;
        B.nu = a.c * ds.dt / ds.dx;
        B.tau_k = 50.0 / (B.nu * B.nu);
        const int n = B.n, Nb = B.Nb, n4 = 4 * Nb;
        const double invc = 1.0 / a.c;

        SlotLayout L = slot_layout(n, m, sizeof(KT));
        double *X = (double *)(slot + L.X), *X0 = (double *)(slot + L.X0), *Tc = (double *)(slot + L.Tc);
        KT *sR = (KT *)(slot + L.sR), *dEv = (KT *)(slot + L.dE), *V = (KT *)(slot + L.V), *Wv = (KT *)(slot + L.W);
        KT *Cs = (KT *)(slot + L.Cs);
        double *Cs64 = sizeof(KT) == 8 ? (double *)Cs : (double *)(slot + L.Cs64);

        // ---- setup: state, sR, data check
        double bad[1] = {0};
        for (int c = tid; c < Nb; c += NT) {
            int i, j, k;
            cell_of(c, n, i, j, k);
            const long long p = B.p(i, j, k);
            const double r_ = (double)rho[p], pp = (double)kP[p], s_ = (double)kR[p];
            bool b = !(r_ >= 0) || !(pp >= 0) || !(s_ >= 0) || !isfinite(r_) || !isfinite(pp) || !isfinite(s_);
            for (int t = 0; t < 6; ++t) {
                const double ft = (double)f[t * AR + p];
                if (!isfinite(ft) || (t < 3 && ft < 0)) b = true;
            }
            bad[0] += b ? 1.0 : 0.0;
            sR[c] = (KT)(B.cdt * r_ * s_);
            X[c] = X0[c] = a.E[p];
            for (int q = 0; q < 3; ++q) X[(1 + q) * Nb + c] = X0[(1 + q) * Nb + c] = a.F[q * AR + p] * invc;
            Tc[c] = a.T[p];
        }
        // corrected face speeds, once per block solve: FP64 from the stored coefficients
        // (ghost neighbours carry their own rho, kappa_R, f), rounded to the Krylov precision
        for (int c = tid; c < Nb; c += NT) {
            int i, j, k;
            cell_of(c, n, i, j, k);
            auto sr64 = [&](int di, int dj, int dk) -> double {
                const long long p = B.p(i + di, j + dj, k + dk);
                return B.cdt * (double)rho[p] * (double)kR[p];
            };
            const double sRc = sr64(0, 0, 0);
            for (int d = 0; d < 3; ++d)
                for (int side = 0; side < 2; ++side) {
                    const int o = side ? 1 : -1;
                    const int di = d == 0 ? o : 0, dj = d == 1 ? o : 0, dk = d == 2 ? o : 0;
                    const double fc = (double)f[d * AR + B.p(i, j, k)];
                    const double fn = (double)f[d * AR + B.p(i + di, j + dj, k + dk)];
                    const double C = face_speed<double>(fc, fn, sRc, sr64(di, dj, dk), B.tau_k);
                    Cs[(2 * d + side) * Nb + c] = (KT)C;
                    Cs64[(2 * d + side) * Nb + c] = C;
                }
        }
        wg_sum<NT, 1>(bad, red);
        rad_stats_t st;
        memset(&st, 0, sizeof(st));
        st.bad_cells = (int)bad[0];
        int status = RAD_NOT_CONVERGED;
        if (st.bad_cells > 0) status = RAD_EDATA;

        // FP64 residual of the current linear system into V[0] (Jacobi-scaled);
        // returns [sum (rE/WE)^2, sum (rF/WF)^2, sum E^2, sum Ft^2, sum (D^-1 r)^2]
        auto residual = [&](double (&nr)[5]) {
            for (int q = 0; q < 5; ++q) nr[q] = 0;
            for (int c = tid; c < Nb; c += NT) {
                int i, j, k;
                cell_of(c, n, i, j, k);
                auto inside = [&](int di, int dj, int dk) {
                    return (unsigned)(i + di) < (unsigned)n && (unsigned)(j + dj) < (unsigned)n &&
                           (unsigned)(k + dk) < (unsigned)n;
                };
                auto ld = [&](int q, int di, int dj, int dk) -> double {
                    if (inside(di, dj, dk)) return X[q * Nb + c + di + n * (dj + n * dk)];
                    const long long p = B.p(i + di, j + dj, k + dk);
                    return q == 0 ? a.E[p] : a.F[(q - 1) * AR + p] * invc;
                };
                auto fl = [&](int t, int di, int dj, int dk) -> double {
                    return (double)f[t * AR + B.p(i + di, j + dj, k + dk)];
                };
                auto cs = [&](int d, int side) -> double { return Cs64[(2 * d + side) * Nb + c]; };
                double div[4], sumC;
                transport_blk_pre<double>(B.nu, ld, fl, cs, div, sumC);
                const long long p = B.p(i, j, k);
                const double r_ = (double)rho[p];
                const double sP = B.cdt * r_ * (double)kP[p], sRc = B.cdt * r_ * (double)kR[p], alpha = r_ * a.cv,
                             aR = a.aR;
                const double Ts = Tc[c], T3 = Ts * Ts * Ts, T4 = T3 * Ts;
                double dE, bE;
                if (a.mode == 0) {
                    dE = 1.0 + sP;
                    bE = a.E[p] + sP * aR * T4;
                } else {
                    const double den = alpha + 4.0 * sP * aR * T3;
                    const double eta = den > 0 ? 4.0 * sP * aR * T3 / den : 0.0;
                    dE = 1.0 + sP * (1.0 - eta);
                    bE = a.E[p] + eta * alpha * a.T[p] - 3.0 * (1.0 - eta) * sP * aR * T4;
                }
                const double E = X[c];
                const double rE = bE - (dE * E + div[0]);
                const double half = 0.5 * B.nu;
                const double DE = dE + half * sumC, DF = 1.0 + sRc + half * sumC;
                const double WE = 1.0 + sP + half * sumC, WF = 1.0 + sRc + half * sumC;
                const double zE = rE / DE;
                V[c] = (KT)zE;
                dEv[c] = (KT)dE;
                double zz = zE * zE, wf = 0, fn = 0;
                for (int q = 0; q < 3; ++q) {
                    const double Fq = X[(1 + q) * Nb + c];
                    const double rF = a.F[q * AR + p] * invc - ((1.0 + sRc) * Fq + div[1 + q]);
                    const double z = rF / DF;
                    V[(1 + q) * Nb + c] = (KT)z;
                    zz += z * z;
                    wf += (rF / WF) * (rF / WF);
                    fn += Fq * Fq;
                }
                nr[0] += (rE / WE) * (rE / WE);
                nr[1] += wf;
                nr[2] += E * E;
                nr[3] += fn;
                nr[4] += zz;
            }
            wg_sum<NT, 5>(nr, red);
        };

        // w = D^-1 A (s x): linear operator, ghost part of the correction is zero;
        // pg != 0: w = pg s x - D^-1 A (s x), the second factor of the polynomial step
        auto apply = [&](const KT *x, KT s, KT *y, KT pg = KT(0)) {
            if constexpr (sizeof(KT) == 4) {
                if (n <= 32) {
                    apply_planes<CT, NT>(B, n, Nb, AR, f, x, s, Cs, sR, dEv, y, &spl[0][0][0], pg);
                    return;
                }
            }
            for (int c = tid; c < Nb; c += NT) {
                int i, j, k;
                cell_of(c, n, i, j, k);
                auto inside = [&](int di, int dj, int dk) {
                    return (unsigned)(i + di) < (unsigned)n && (unsigned)(j + dj) < (unsigned)n &&
                           (unsigned)(k + dk) < (unsigned)n;
                };
                auto ld = [&](int q, int di, int dj, int dk) -> KT {
                    return inside(di, dj, dk) ? s * x[q * Nb + c + di + n * (dj + n * dk)] : KT(0);
                };
                auto fl = [&](int t, int di, int dj, int dk) -> KT {
                    return (KT)f[t * AR + B.p(i + di, j + dj, k + dk)];
                };
                auto cs = [&](int d, int side) -> KT { return Cs[(2 * d + side) * Nb + c]; };
                KT div[4], sumC;
                transport_blk_pre<KT>((KT)B.nu, ld, fl, cs, div, sumC);
                const KT sRc = sR[c], dEc = dEv[c], half = KT(0.5) * (KT)B.nu;
                const KT xc = ld(0, 0, 0, 0);
                const KT yE = (dEc * xc + div[0]) / (dEc + half * sumC);
                y[c] = pg != KT(0) ? pg * xc - yE : yE;
                const KT DF = KT(1) + sRc + half * sumC;
                for (int q = 0; q < 3; ++q) {
                    const KT xq = ld(1 + q, 0, 0, 0);
                    const KT yq = ((KT(1) + sRc) * xq + div[1 + q]) / DF;
                    y[(1 + q) * Nb + c] = pg != KT(0) ? pg * xq - yq : yq;
                }
            }
        };

        double resT = 0, best_res = INFINITY;
        int best_at = 0;
        double nr[5];
        for (int kp = 0; status != RAD_EDATA; ++kp) {
            residual(nr);
            st.refine_sweeps++;
            const double nE = sqrt(nr[2]), nF = sqrt(nr[3]);
            st.res_E = nE > 0 ? sqrt(nr[0]) / nE : sqrt(nr[0]);
            st.res_F = (nF + nE) > 0 ? sqrt(nr[1]) / (nF + nE) : sqrt(nr[1]);
            st.res_T = resT;
            const double res = fmax(fmax(st.res_E, st.res_F), resT);
            st.scaled_residual = res;
            if (kp > 0 && res <= a.tol) {
                status = RAD_OK;
                break;
            }
            if (kp >= a.max_picard) break;
            // stall: no new best residual within the last 5 Picard iterations
            if (res < best_res) {
                best_res = res;
                best_at = kp;
            } else if (kp - best_at >= 5) {
                break;
            }

            double beta = sqrt(nr[4]);
            const double rtol = fmin(1.0, fmax(fmin(a.eps_R, 1.0), 0.1 * a.tol / fmax(res, 1e-300)));
            const double target = beta * rtol;
            const double inner_floor = sizeof(KT) == 4 ? 1e-5 : 0.0;
            int its = 0;
            double beta_prev = INFINITY;
            while (beta > target && beta > 0 && its < a.max_krylov && beta < 0.999 * beta_prev) {
                beta_prev = beta;
                const double cyc_target = fmax(target, beta * inner_floor);
                if (tid == 0) {
                    sh_s[0] = 1.0 / beta;
                    for (int q = 0; q <= m; ++q) sh_g[q] = 0;
                    sh_g[0] = beta;
                }
                __syncthreads();
                int cols = 0;
                for (int j = 0; j < m && its < a.max_krylov; ++j) {
                    KT *vj = V + (long long)j * n4, *vn = V + (long long)(j + 1) * n4;
                    if (a.poly) {   // w = (2I - B) B (s_j V_j), B (s_j V_j) parked in the slot of V_j+1
                        apply(vj, (KT)sh_s[j], vn);
                        __syncthreads();
                        apply(vn, KT(1), Wv, KT(2));
                    } else {
                        apply(vj, (KT)sh_s[j], Wv);
                    }
                    ++its;
                    __syncthreads();
                    // dots <V_i, w>, i <= j, in chunks of DC, and <w, w>; indices past j are
                    // clamped to j so every load of a chunk is issued unconditionally
                    double ww = 0;
                    for (int i0 = 0; i0 <= j; i0 += DC) {
                        double acc[DC + 1];
#pragma unroll
                        for (int q = 0; q <= DC; ++q) acc[q] = 0;
                        const int cnt = min(DC, j + 1 - i0);
                        const KT *vq[DC];
#pragma unroll
                        for (int q = 0; q < DC; ++q) vq[q] = V + (long long)min(i0 + q, j) * n4;
                        for (int e = 4 * tid; e < n4; e += 4 * NT) {
                            double we[4];
                            Quad<KT>::load(Wv + e, we);
                            KT vv[DC][4];
#pragma unroll
                            for (int q = 0; q < DC; ++q) Quad<KT>::load_raw(vq[q] + e, vv[q]);
#pragma unroll
                            for (int q = 0; q < DC; ++q)
                                acc[q] += (double)vv[q][0] * we[0] + (double)vv[q][1] * we[1] + (double)vv[q][2] * we[2] +
                                          (double)vv[q][3] * we[3];
                            acc[DC] += we[0] * we[0] + we[1] * we[1] + we[2] * we[2] + we[3] * we[3];
                        }
                        wg_sum<NT, DC + 1>(acc, red);
                        if (tid == 0)
                            for (int q = 0; q < cnt; ++q) sh_dots[i0 + q] = acc[q];
                        ww = acc[DC];
                    }
                    __syncthreads();
                    if (tid <= j) sh_a[tid] = sh_s[tid] * sh_s[tid] * sh_dots[tid];
                    __syncthreads();
                    // v_{j+1} = w - sum_i s_i^2 d_i V_i
                    double nn[1] = {0};
                    // basis vectors in chunks of DC with indices past j clamped to j and a zero
                    // coefficient, so every load of a chunk is issued at once
                    for (int e = 4 * tid; e < n4; e += 4 * NT) {
                        double val[4];
                        Quad<KT>::load(Wv + e, val);
                        for (int i0 = 0; i0 <= j; i0 += DC) {
                            KT a8[DC][4];
#pragma unroll
                            for (int u = 0; u < DC; ++u) Quad<KT>::load_raw(V + (long long)min(i0 + u, j) * n4 + e, a8[u]);
#pragma unroll
                            for (int u = 0; u < DC; ++u) {
                                const double cu = i0 + u <= j ? sh_a[i0 + u] : 0.0;
#pragma unroll
                                for (int k = 0; k < 4; ++k) val[k] -= cu * (double)a8[u][k];
                            }
                        }
                        double r[4];
                        Quad<KT>::store(vn + e, val, r);
                        nn[0] += r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3];
                    }
                    wg_sum<NT, 1>(nn, red);
                    if (tid == 0) {
                        const double hn = sqrt(nn[0]);
                        for (int i = 0; i <= j; ++i) sh_H[i * m + j] = sh_s[i] * sh_dots[i];
                        sh_H[(j + 1) * m + j] = hn;
                        sh_s[j + 1] = hn > 0 ? 1.0 / hn : 0.0;
                        for (int i = 0; i < j; ++i) {
                            const double x = sh_H[i * m + j], y = sh_H[(i + 1) * m + j];
                            sh_H[i * m + j] = sh_cs[i] * x + sh_sn[i] * y;
                            sh_H[(i + 1) * m + j] = -sh_sn[i] * x + sh_cs[i] * y;
                        }
                        const double x = sh_H[j * m + j], y = sh_H[(j + 1) * m + j];
                        const double rr = hypot(x, y);
                        sh_cs[j] = rr > 0 ? x / rr : 1.0;
                        sh_sn[j] = rr > 0 ? y / rr : 0.0;
                        sh_H[j * m + j] = rr;
                        sh_H[(j + 1) * m + j] = 0.0;
                        sh_g[j + 1] = -sh_sn[j] * sh_g[j];
                        sh_g[j] = sh_cs[j] * sh_g[j];
                        sh_flag = (fabs(sh_g[j + 1]) <= cyc_target || hn <= 1e-14 * sqrt(ww)) ? 1 : 0;
                    }
                    __syncthreads();
                    cols = j + 1;
                    if (sh_flag) break;
                }
                // y = H^-1 g;  X += sum_i y_i s_i V_i
                if (tid == 0) {
                    for (int i = cols - 1; i >= 0; --i) {
                        double s = sh_g[i];
                        for (int l = i + 1; l < cols; ++l) s -= sh_H[i * m + l] * sh_y[l];
                        sh_y[i] = sh_H[i * m + i] != 0 ? s / sh_H[i * m + i] : 0.0;
                    }
                    for (int i = 0; i < cols; ++i) sh_a[i] = sh_y[i] * sh_s[i];
                }
                __syncthreads();
                if (a.poly) {
                    // X += (2I - B) z, z = sum_i a_i V_i formed in the slot of V_cols
                    KT *z = V + (long long)cols * n4;
                    for (int e = 4 * tid; e < n4; e += 4 * NT) {
                        double acc[4] = {0, 0, 0, 0}, r[4];
                        for (int i = 0; i < cols; ++i) {
                            double a1[4];
                            Quad<KT>::load(V + (long long)i * n4 + e, a1);
#pragma unroll
                            for (int k = 0; k < 4; ++k) acc[k] += sh_a[i] * a1[k];
                        }
                        Quad<KT>::store(z + e, acc, r);
                    }
                    __syncthreads();
                    apply(z, KT(1), Wv, KT(2));
                    __syncthreads();
                    for (int e = 4 * tid; e < n4; e += 4 * NT) {
                        double acc[4], w4[4], r[4];
                        Quad<double>::load(X + e, acc);
                        Quad<KT>::load(Wv + e, w4);
#pragma unroll
                        for (int k = 0; k < 4; ++k) acc[k] += w4[k];
                        Quad<double>::store(X + e, acc, r);
                    }
                } else {
                    for (int e = 4 * tid; e < n4; e += 4 * NT) {
                        double acc[4], r[4];
                        Quad<double>::load(X + e, acc);
                        for (int i = 0; i < cols; ++i) {
                            double a1[4];
                            Quad<KT>::load(V + (long long)i * n4 + e, a1);
#pragma unroll
                            for (int k = 0; k < 4; ++k) acc[k] += sh_a[i] * a1[k];
                        }
                        Quad<double>::store(X + e, acc, r);
                    }
                }
                __syncthreads();
                residual(nr);
                st.refine_sweeps++;
                beta = sqrt(nr[4]);
            }
            st.krylov_iters += its;

            // exchange and the iteration's diagnostics
            double ex[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int c = tid; c < Nb; c += NT) {
                int i, j, k;
                cell_of(c, n, i, j, k);
                const long long p = B.p(i, j, k);
                const double r_ = (double)rho[p];
                const double sP = B.cdt * r_ * (double)kP[p], alpha = r_ * a.cv, aR = a.aR, Tn = a.T[p];
                const double E = X[c];
                bool neg = false;
                const double T = exchange_T(alpha, Tn, sP, aR, E, neg);
                const double T3 = T * T * T;
                const double RT0 = alpha * (T - Tn) + sP * (aR * T3 * T - E);
                const double RT = (T == 0.0 && RT0 > 0.0) ? 0.0 : RT0;
                const double WT = alpha + 4.0 * sP * aR * T3;
                const double dT = T - Tc[c];
                Tc[c] = T;
                ex[0] += WT > 0 ? (RT / WT) * (RT / WT) : 0.0;
                ex[1] += T * T;
                ex[2] += dT * dT;
                const double dE = E - X0[c];
                ex[3] += dE * dE;
                ex[4] += E * E;
                X0[c] = E;
                for (int q = 1; q < 4; ++q) {
                    const double x = X[q * Nb + c], d = x - X0[q * Nb + c];
                    ex[5] += d * d;
                    ex[6] += x * x;
                    X0[q * Nb + c] = x;
                }
                ex[7] += neg ? 1.0 : 0.0;
            }
            wg_sum<NT, 8>(ex, red);
            resT = ex[1] > 0 ? sqrt(ex[0] / ex[1]) : sqrt(ex[0]);
            const double cE = ex[4] > 0 ? sqrt(ex[3] / ex[4]) : 0.0;
            const double cF = (ex[6] + ex[4]) > 0 ? sqrt(ex[5]) / (sqrt(ex[6]) + sqrt(ex[4])) : 0.0;
            const double cT = ex[1] > 0 ? sqrt(ex[2] / ex[1]) : 0.0;
            st.rel_change = fmax(cE, fmax(cF, cT));
            st.neg_cells = (int)ex[7];
            st.picard_iters = kp + 1;
        }

        // commit (not for invalid data: the state is left untouched)
        if (status != RAD_EDATA) {
            for (int c = tid; c < Nb; c += NT) {
                int i, j, k;
                cell_of(c, n, i, j, k);
                const long long p = B.p(i, j, k);
                a.E[p] = X[c];
                for (int q = 0; q < 3; ++q) a.F[q * AR + p] = X[(1 + q) * Nb + c] * a.c;
                a.T[p] = Tc[c];
            }
        }
        if (tid == 0) {
            st.status = status;
            st.t_total_ms = a.clk_khz > 0 ? (double)(wall_clock64() - t_start) / a.clk_khz : 0.0;
            a.stats[bid] = st;
        }
        __syncthreads();
    }
}

__global__ void k_queue_reset(int *q) { *q = 0; }

// ---------------------------------------------------------------- host side

using KernelFn = void (*)(BatchArgs);

KernelFn pick_kernel(int coef_dtype, int prec, int nt)
{
    const bool c32 = coef_dtype == RAD_F32, k32 = prec == RAD_MIXED;
    if (nt == 512) {
        if (c32) return k32 ? k_batched<float, float, 512> : k_batched<float, double, 512>;
        return k32 ? k_batched<double, float, 512> : k_batched<double, double, 512>;
    }
    if (c32) return k32 ? k_batched<float, float, 256> : k_batched<float, double, 256>;
    return k32 ? k_batched<double, float, 256> : k_batched<double, double, 256>;
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

constexpr int kMaxSlotsPerCU = 2;

struct Geometry {
    int nmax = 0;
    long long arena = 0;
    double work = 0;
};

int check_blocks(int nblocks, const rad_block_desc_t *desc, Geometry &G)
{
    if (nblocks < 1) return fail(RAD_EINVAL, "nblocks must be >= 1");
    if (!desc) return fail(RAD_EINVAL, "desc is NULL");
    std::vector<std::pair<long long, long long>> spans;
    for (int b = 0; b < nblocks; ++b) {
        const rad_block_desc_t &d = desc[b];
        if (d.n < 1 || d.n > 64) return fail(RAD_EINVAL, "block %d: n must be in [1, 64]", b);
        if (d.ng < 1) return fail(RAD_EINVAL, "block %d: ng must be >= 1", b);
        if (!(d.dx > 0) || !std::isfinite(d.dx)) return fail(RAD_EINVAL, "block %d: dx must be positive", b);
        if (!(d.dt > 0) || !std::isfinite(d.dt)) return fail(RAD_EINVAL, "block %d: dt must be positive", b);
        if (d.off < 0) return fail(RAD_EINVAL, "block %d: negative offset", b);
        const long long M = d.n + 2LL * d.ng, sz = M * M * M;
        spans.push_back({d.off, d.off + sz});
        G.nmax = std::max(G.nmax, d.n);
        G.arena = std::max(G.arena, d.off + sz);
        G.work += (double)d.n * d.n * d.n;
    }
    std::sort(spans.begin(), spans.end());
    for (size_t k = 1; k < spans.size(); ++k)
        if (spans[k].first < spans[k - 1].second) return fail(RAD_EINVAL, "block regions overlap in the arena");
    return RAD_OK;
}

struct WsLayout {
    size_t desc, order, queue, slots, total;
    long long slot_bytes;
    int nslots;
};

WsLayout ws_layout(int nblocks, int nmax, const rad_params_t &p)
{
    WsLayout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t at = o;
        o += align_up(b);
        return at;
    };
    L.desc = take(nblocks * sizeof(rad_block_desc_t));
    L.order = take(nblocks * sizeof(int));
    L.queue = take(256);
    L.slot_bytes = (long long)slot_layout(nmax, p.gmres_m, p.prec == RAD_MIXED ? 4 : 8).total;
    L.nslots = kMaxSlotsPerCU * device_cus();
    L.slots = take((size_t)L.slot_bytes * L.nslots);
    L.total = o;
    return L;
}

}  // namespace

struct rad_plan_s {
    int nblocks = 0;
    std::vector<rad_block_desc_t> desc;
    rad_params_t p;
    Geometry G;
    WsLayout L;
    char *ws = nullptr;
    int cus = 0;
    int nt = 512;
    int per_cu = 1;
    bool lpt = true;
    std::vector<double> cost;  // measured solve time per block (rad_plan_reorder), empty until then
    double clk_khz = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t knode = nullptr;
    BatchArgs args;
    void *argv[1];
    int *qptr = nullptr;     // argument storage of the queue-reset node
    void *rargv[1];
};

namespace {

int upload_order(rad_plan P, hipStream_t st)
{
    std::vector<int> order(P->nblocks);
    for (int b = 0; b < P->nblocks; ++b) order[b] = b;
    // longest processing time first: by the measured solve times of an earlier step when the caller
    // has supplied them, else estimated by interior cells
    if (P->lpt && (int)P->cost.size() == P->nblocks)
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return P->cost[x] > P->cost[y]; });
    else if (P->lpt)
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return P->desc[x].n > P->desc[y].n; });
    HIP_TRY(hipMemcpyAsync(P->ws + P->L.order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return RAD_OK;
}

int grid_of(rad_plan P) { return std::min(P->per_cu * P->cus, P->L.nslots); }

void fill_args(rad_plan P, double *E, double *F, double *T, const void *rho, const void *kP, const void *kR,
               const void *f, rad_stats_t *stats)
{
    BatchArgs &a = P->args;
    a.desc = (const rad_block_desc_t *)(P->ws + P->L.desc);
    a.order = (const int *)(P->ws + P->L.order);
    a.nblocks = P->nblocks;
    a.arena = P->G.arena;
    a.E = E;
    a.F = F;
    a.T = T;
    a.rho = rho;
    a.kP = kP;
    a.kR = kR;
    a.f = f;
    a.stats = stats;
    a.slots = P->ws + P->L.slots;
    a.slot_bytes = P->L.slot_bytes;
    a.queue = (int *)(P->ws + P->L.queue);
    a.c = P->p.c;
    a.aR = P->p.a_R;
    a.cv = P->p.c_v;
    a.tol = P->p.tol;
    a.eps_R = P->p.eps_R;
    a.max_picard = P->p.max_picard;
    a.max_krylov = P->p.max_krylov;
    a.m = P->p.gmres_m;
    a.poly = P->p.krylov_poly;
    a.mode = P->p.mode;
    a.clk_khz = P->clk_khz;
    P->argv[0] = &P->args;
}

hipKernelNodeParams kernel_params(rad_plan P)
{
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = (void *)pick_kernel(P->p.coef_dtype, P->p.prec, P->nt);
    kp.gridDim = dim3(grid_of(P));
    kp.blockDim = dim3(P->nt);
    kp.sharedMemBytes = 0;
    kp.kernelParams = P->argv;
    kp.extra = nullptr;
    return kp;
}

void destroy_graph(rad_plan P)
{
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    P->exec = nullptr;
    P->graph = nullptr;
    P->knode = nullptr;
}

// Graph: queue reset kernel -> persistent kernel (no memset nodes).
int build_graph(rad_plan P)
{
    destroy_graph(P);
    HIP_TRY(hipGraphCreate(&P->graph, 0));
    hipKernelNodeParams rp;
    std::memset(&rp, 0, sizeof(rp));
    P->qptr = (int *)(P->ws + P->L.queue);
    P->rargv[0] = &P->qptr;
    rp.func = (void *)k_queue_reset;
    rp.gridDim = dim3(1);
    rp.blockDim = dim3(1);
    rp.kernelParams = P->rargv;
    hipGraphNode_t rnode;
    HIP_TRY(hipGraphAddKernelNode(&rnode, P->graph, nullptr, 0, &rp));
    hipKernelNodeParams kp = kernel_params(P);
    HIP_TRY(hipGraphAddKernelNode(&P->knode, P->graph, &rnode, 1, &kp));
    HIP_TRY(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
    return RAD_OK;
}

// direct (non-graph) launch, used by the autotuner
int launch_direct(rad_plan P, hipStream_t st)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, st, P->args.queue);
    KernelFn fn = pick_kernel(P->p.coef_dtype, P->p.prec, P->nt);
    hipLaunchKernelGGL(fn, dim3(grid_of(P)), dim3(P->nt), 0, st, P->args);
    HIP_TRY(hipGetLastError());
    return RAD_OK;
}

std::string plan_key(rad_plan P)
{
    int hist[65] = {0};
    for (auto &d : P->desc) hist[d.n]++;
    std::ostringstream os;
    os << "batched|" << device_tag() << "|p" << P->p.prec << "|c" << P->p.coef_dtype << "|m" << P->p.gmres_m << "|k" << P->p.krylov_poly << "|";
    for (int k = 1; k <= 64; ++k)
        if (hist[k]) os << k << "x" << hist[k] << ",";
    return os.str();
}

bool cache_lookup(rad_plan P)
{
    std::string v;
    if (!cache_get(plan_key(P), v)) return false;
    int nt, pc, lpt;
    if (std::sscanf(v.c_str(), "%d %d %d", &nt, &pc, &lpt) == 3 && (nt == 256 || nt == 512) && pc >= 1 &&
        pc <= kMaxSlotsPerCU) {
        P->nt = nt;
        P->per_cu = pc;
        P->lpt = lpt != 0;
        return true;
    }
    return false;
}

void cache_store(rad_plan P)
{
    cache_put(plan_key(P), std::to_string(P->nt) + " " + std::to_string(P->per_cu) + " " + (P->lpt ? "1" : "0"));
}

}  // namespace

extern "C" size_t rad_batched_workspace_bytes(int nblocks, const rad_block_desc_t *desc, const rad_params_t *p)
{
    Geometry G;
    if (check_params(p) != RAD_OK || check_blocks(nblocks, desc, G) != RAD_OK) return 0;
    return ws_layout(nblocks, G.nmax, *p).total;
}

namespace {
int plan_batched(int nblocks, const rad_block_desc_t *desc, const rad_params_t *p, void *workspace, size_t ws_bytes,
                 void *stream, rad_plan *out)
{
    if (!out) return fail(RAD_EINVAL, "out is NULL");
    *out = nullptr;
    RAD_TRY(check_params(p));
    if (p->anderson_m != 0) return fail(RAD_EINVAL, "the batched path runs plain Picard: anderson_m must be 0");
    if (p->cv_cubic != 0) return fail(RAD_EINVAL, "the batched path requires cv_cubic = 0");
    if (p->krylov_poly == 2) return fail(RAD_EINVAL, "the batched path has no multigrid Krylov operator");
    if (p->energy_fix) return fail(RAD_EINVAL, "energy_fix: single-grid rad_step only");
    Geometry G;
    RAD_TRY(check_blocks(nblocks, desc, G));
    if (!workspace) return fail(RAD_EINVAL, "workspace is NULL");
    if (((uintptr_t)workspace) % 256) return fail(RAD_EINVAL, "workspace must be 256-byte aligned");
    WsLayout L = ws_layout(nblocks, G.nmax, *p);
    if (ws_bytes < L.total) return fail(RAD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    rad_plan P = new rad_plan_s();
    P->nblocks = nblocks;
    P->desc.assign(desc, desc + nblocks);
    P->p = *p;
    P->G = G;
    P->L = L;
    P->ws = (char *)workspace;
    P->cus = device_cus();
    P->nt = 512;  // one 8-wave workgroup per CU unless the autotune cache says otherwise
    P->per_cu = 1;
    P->lpt = true;
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            P->clk_khz = khz;
    }
    cache_lookup(P);
    int rc = RAD_OK;
    if (hipMemcpyAsync(P->ws + L.desc, desc, nblocks * sizeof(rad_block_desc_t), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        rc = fail(RAD_EHIP, "descriptor upload failed");
    if (rc == RAD_OK) rc = upload_order(P, st);
    if (rc == RAD_OK) {
        fill_args(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
        rc = build_graph(P);
    }
    if (rc != RAD_OK) {
        destroy_graph(P);
        delete P;
        return rc;
    }
    *out = P;
    return RAD_OK;
}
}  // namespace

extern "C" int rad_plan_batched(int nblocks, const rad_block_desc_t *desc, const rad_params_t *p, void *workspace,
                                size_t ws_bytes, void *stream, rad_plan *out)
{
    clear_error();
    if (out) *out = nullptr;
    try {  // the plan object and its descriptor copy live in host memory
        return plan_batched(nblocks, desc, p, workspace, ws_bytes, stream, out);
    } catch (const std::bad_alloc &) {
        return fail(RAD_ENOMEM, "host memory for the plan");
    }
}

extern "C" int rad_step_batched(rad_plan P, double *E, double *F, double *T_gas, const void *rho, const void *kappa_P,
                                const void *kappa_R, const void *f_ij, rad_stats_t *dev_stats, void *stream)
{
    clear_error();
    if (!P) return fail(RAD_EINVAL, "plan is NULL");
    if (!E || !F || !T_gas || !rho || !kappa_P || !kappa_R || !f_ij || !dev_stats)
        return fail(RAD_EINVAL, "NULL data pointer");
    fill_args(P, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, dev_stats);
    hipKernelNodeParams kp = kernel_params(P);
    HIP_TRY(hipGraphExecKernelNodeSetParams(P->exec, P->knode, &kp));
    const int tok = prof_begin(K_BATCHED, (hipStream_t)stream);
    HIP_TRY(hipGraphLaunch(P->exec, (hipStream_t)stream));
    // algorithmic bytes of one block step are iteration dependent; record the state traffic only
    prof_end(tok, (hipStream_t)stream, (double)P->G.work * (4 + 1) * 8 * 2);
    return RAD_OK;
}

extern "C" size_t rad_autotune_scratch_bytes(rad_plan P)
{
    if (!P) return 0;
    return align_up((size_t)P->G.arena * 5 * sizeof(double)) + align_up((size_t)P->nblocks * sizeof(rad_stats_t));
}

extern "C" int rad_autotune_batched(rad_plan P, double *E, double *F, double *T_gas, const void *rho,
                                    const void *kappa_P, const void *kappa_R, const void *f_ij, void *scratch,
                                    size_t scratch_bytes, void *stream)
{
    clear_error();
    if (!P) return fail(RAD_EINVAL, "plan is NULL");
    if (!E || !F || !T_gas || !rho || !kappa_P || !kappa_R || !f_ij || !scratch)
        return fail(RAD_EINVAL, "NULL data pointer");
    if (((uintptr_t)scratch) % 256) return fail(RAD_EINVAL, "scratch must be 256-byte aligned");
    if (scratch_bytes < rad_autotune_scratch_bytes(P)) return fail(RAD_ENOMEM, "autotune scratch too small");
    hipStream_t st = (hipStream_t)stream;
    const size_t A = (size_t)P->G.arena;
    double *saveE = (double *)scratch, *saveF = saveE + A, *saveT = saveF + 3 * A;
    rad_stats_t *tstats = (rad_stats_t *)((char *)scratch + align_up(A * 5 * sizeof(double)));
    HIP_TRY(hipMemcpyAsync(saveE, E, A * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(saveF, F, 3 * A * 8, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(saveT, T_gas, A * 8, hipMemcpyDeviceToDevice, st));
    auto restore = [&]() -> int {
        HIP_TRY(hipMemcpyAsync(E, saveE, A * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(F, saveF, 3 * A * 8, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(T_gas, saveT, A * 8, hipMemcpyDeviceToDevice, st));
        return RAD_OK;
    };
    struct Cand {
        int nt, per_cu;
        bool lpt;
    };
    const Cand cands[] = {{512, 1, true}, {512, 2, true}, {256, 2, true}, {256, 1, true}, {512, 1, false}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = INFINITY;
    Cand win = cands[0];
    int rc = RAD_OK;
    for (const Cand &c : cands) {
        P->nt = c.nt;
        P->per_cu = c.per_cu;
        P->lpt = c.lpt;
        if ((rc = upload_order(P, st)) != RAD_OK) break;
        fill_args(P, E, F, T_gas, rho, kappa_P, kappa_R, f_ij, tstats);
        // one timed trial per candidate: a trial is a whole batched step (seconds),
        // far longer than any cache or code warm-up
        float ms = 0;
        if ((rc = restore()) != RAD_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
        if (rc == RAD_OK) rc = launch_direct(P, st);
        if (rc == RAD_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(RAD_EHIP, "event record failed");
        if (rc == RAD_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(RAD_EHIP, "trial failed");
        if (rc == RAD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(RAD_EHIP, "timing failed");
        if (rc != RAD_OK) break;
        if (trace_enabled())
            std::fprintf(stderr, "[rad] autotune nt=%d per_cu=%d lpt=%d: %.3f ms\n", c.nt, c.per_cu, (int)c.lpt, ms);
        if (ms < best) {
            best = ms;
            win = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->nt = win.nt;
    P->per_cu = win.per_cu;
    P->lpt = win.lpt;
    const int rc2 = restore();
    if (rc != RAD_OK) return rc;
    RAD_TRY(rc2);
    RAD_TRY(upload_order(P, st));
    fill_args(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    RAD_TRY(build_graph(P));
    HIP_TRY(hipStreamSynchronize(st));
    cache_store(P);
    return RAD_OK;
}

extern "C" int rad_plan_launch_shape(rad_plan P, int *threads, int *per_cu, int *largest_first)
{
    clear_error();
    if (!P) return fail(RAD_EINVAL, "plan is NULL");
    if (threads) *threads = P->nt;
    if (per_cu) *per_cu = P->per_cu;
    if (largest_first) *largest_first = P->lpt ? 1 : 0;
    return RAD_OK;
}

extern "C" int rad_plan_reorder(rad_plan P, const rad_stats_t *dev_stats, void *stream)
{
    clear_error();
    if (!P) return fail(RAD_EINVAL, "plan is NULL");
    if (!dev_stats) return fail(RAD_EINVAL, "dev_stats is NULL");
    if (P->clk_khz <= 0) return fail(RAD_ENOTIMPL, "the device reports no wall-clock rate: blocks are not timed");
    hipStream_t st = (hipStream_t)stream;
    try {
        std::vector<rad_stats_t> h(P->nblocks);
        HIP_TRY(hipMemcpyAsync(h.data(), dev_stats, h.size() * sizeof(rad_stats_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::vector<double> cost(P->nblocks);
        for (int b = 0; b < P->nblocks; ++b) {
            const double t = h[b].t_total_ms;
            if (!(t >= 0) || !std::isfinite(t)) return fail(RAD_EINVAL, "block %d: no solve time in dev_stats", b);
            cost[b] = t;
        }
        P->cost.swap(cost);
    } catch (const std::bad_alloc &) {
        return fail(RAD_ENOMEM, "host memory for the block times");
    }
    P->lpt = true;
    return upload_order(P, st);
}

extern "C" void rad_plan_destroy(rad_plan P)
{
    if (!P) return;
    destroy_graph(P);
    delete P;
}
