// rad_apply_tiled.h -- the operator apply as a 2.5D z-marching stencil (gfx950).
//
// A workgroup of 256 threads (64 x 4) owns a 64 x 8 cell column of the grid
// over a range of z planes.  For the current plane k the tile and a one-cell
// x/y halo live in LDS (state, tensor, sR); the planes k-1 and k+1 of the
// thread's own cells live in registers, so every value is read from HBM once
// per z-range (the halo rows are read by the neighbouring tile too and hit in
// L2, since tiles are assigned to XCDs in contiguous ranges).  Every LDS slot
// and every z neighbour is first mapped through the boundary rule (periodic:
// wrap, outflow: the boundary cell itself), so boundary faces and ragged tile
// edges need no special cases: a face whose mapped neighbour is the cell
// itself carries the cell's physical flux and no dissipation.
#pragma once
#include "rad_device.h"

namespace vr {

constexpr int kTX = 64;          // tile width (x), one wave per row
constexpr int kTYT = 4;          // thread rows
constexpr int kCPT = 2;          // cells per thread along y
constexpr int kTY = kTYT * kCPT; // tile height (y)
constexpr int kLX = kTX + 2, kLY = kTY + 2;
constexpr int kHalo = 2 * kTX + 2 * kTY;

// Workgroup barrier that orders LDS only: global loads issued before it stay in
// flight (a full __syncthreads would wait for them as well).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int map_axis(int q, int n, int lo, int hi)
{
    if (q < 0) return lo == BC_PERIODIC ? ((q % n) + n) % n : 0;
    if (q >= n) return hi == BC_PERIODIC ? q % n : n - 1;
    return q;
}

struct TileGeom {
    int tiles_x, tiles_y, tiles_z, kz;
};

inline TileGeom tile_geom(const Grid &g)
{
    TileGeom t;
    t.tiles_x = (g.nx + kTX - 1) / kTX;
    t.tiles_y = (g.ny + kTY - 1) / kTY;
    // z-range per workgroup: enough workgroups to fill the chip several times over
    const long long cols = (long long)t.tiles_x * t.tiles_y;
    int kz = g.nz;
    while (kz > 8 && cols * ((g.nz + kz - 1) / kz) < 4096) kz = (kz + 1) / 2;
    t.kz = kz;
    t.tiles_z = (g.nz + kz - 1) / kz;
    return t;
}

// y = D^-1 A (s x) (prec = 1) or y = A x with flux rescaling xF/yF (prec = 0).
// sR: precomputed c dt rho kappa_R in AT, or nullptr to derive it from rho, kR.
// Cf: the corrected face speeds divided by c at the three low faces of every
// cell (planes x|y|z), precomputed once per step; nullptr derives them per face.
template <class AT, class ST>
__global__ void __launch_bounds__(256)
    k_apply_tiled(Grid g, TileGeom tg, const ST *__restrict__ f, const AT *__restrict__ sR,
                  const ST *__restrict__ rho, const ST *__restrict__ kR, const AT *__restrict__ Cf,
                  const AT *__restrict__ dE, const AT *__restrict__ x, const double *__restrict__ xs,
                  AT *__restrict__ y, int prec, AT xF, AT yF)
{
    __shared__ AT sx[4][kLY][kLX];
    __shared__ AT sf[6][kLY][kLX];
    __shared__ AT ss[kLY][kLX];
    __shared__ AT sc[2][kLY][kLX];

    const long long N = g.N;
    const long long plane = (long long)g.nx * g.ny;
    // XCD-aware tile order: consecutive workgroup ids go to different XCDs, so
    // give each XCD a contiguous range of tiles (neighbours share halo rows in L2)
    const int ntiles = gridDim.x;
    int tile = blockIdx.x;
    if (ntiles % 8 == 0) tile = (blockIdx.x % 8) * (ntiles / 8) + blockIdx.x / 8;
    const int bx = tile % tg.tiles_x;
    const int rest = tile / tg.tiles_x;
    const int by = rest % tg.tiles_y;
    const int bz = rest / tg.tiles_y;
    const int x0 = bx * kTX, y0 = by * kTY, z0 = bz * tg.kz;
    const int z1 = min(z0 + tg.kz, g.nz);
    const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;

    const AT s = xs ? (AT)(*xs) : AT(1);
    const AT sF = s * xF;
    const double cdt = g.cdt;
    auto sr_at = [&](long long idx) -> AT { return sR ? sR[idx] : (AT)(cdt * (double)rho[idx] * (double)kR[idx]); };

    // mapped coordinates of the thread's cells and of the LDS halo cell it loads
    const int gx = x0 + lx;
    const int mx = map_axis(gx, g.nx, g.bclo[0], g.bchi[0]);
    int my[kCPT];
    bool active[kCPT];
    for (int c = 0; c < kCPT; ++c) {
        const int gy = y0 + ly + kTYT * c;
        my[c] = map_axis(gy, g.ny, g.bclo[1], g.bchi[1]);
        active[c] = gx < g.nx && gy < g.ny;
    }
    // halo slot of this thread (if any): (hy, hx) in LDS coordinates and its mapped cell
    int hly = -1, hlx = -1, hmx = 0, hmy = 0;
    if (threadIdx.x < kHalo) {
        const int h = threadIdx.x;
        int gxh, gyh;
        if (h < kTX) { hlx = h + 1; hly = 0; gxh = x0 + h; gyh = y0 - 1; }
        else if (h < 2 * kTX) { hlx = h - kTX + 1; hly = kLY - 1; gxh = x0 + h - kTX; gyh = y0 + kTY; }
        else if (h < 2 * kTX + kTY) { hlx = 0; hly = h - 2 * kTX + 1; gxh = x0 - 1; gyh = y0 + h - 2 * kTX; }
        else { hlx = kLX - 1; hly = h - 2 * kTX - kTY + 1; gxh = x0 + kTX; gyh = y0 + h - 2 * kTX - kTY; }
        hmx = map_axis(gxh, g.nx, g.bclo[0], g.bchi[0]);
        hmy = map_axis(gyh, g.ny, g.bclo[1], g.bchi[1]);
    }
    // self-faces (mapped neighbour is the cell itself): excluded from the Jacobi diagonal
    const bool selfx_lo = map_axis(gx - 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    const bool selfx_hi = map_axis(gx + 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    bool selfy_lo[kCPT], selfy_hi[kCPT];
    for (int c = 0; c < kCPT; ++c) {
        const int gy = y0 + ly + kTYT * c;
        selfy_lo[c] = map_axis(gy - 1, g.ny, g.bclo[1], g.bchi[1]) == my[c];
        selfy_hi[c] = map_axis(gy + 1, g.ny, g.bclo[1], g.bchi[1]) == my[c];
    }

    const bool pre = Cf != nullptr;
    // full cell values: x (4, scaled), f (6), sR, low-face speeds (when precomputed)
    struct Full {
        AT x[4], f[6], s, c[3];
    };
    // z-neighbour subset: x (4), f row z (xz, yz, zz), sR
    struct ZRow {
        AT x[4], f[3], s;
    };
    auto load_full = [&](long long idx, Full &v) {
        v.x[0] = s * x[idx];
        for (int q = 1; q < 4; ++q) v.x[q] = sF * x[q * N + idx];
        for (int t = 0; t < 6; ++t) v.f[t] = (AT)f[t * N + idx];
        v.s = sr_at(idx);
        if (pre)
            for (int d = 0; d < 3; ++d) v.c[d] = Cf[d * N + idx];
        else
            v.c[0] = v.c[1] = v.c[2] = AT(0);
    };
    auto to_zrow = [&](const Full &v, ZRow &z) {
        for (int q = 0; q < 4; ++q) z.x[q] = v.x[q];
        z.f[0] = v.f[tens_row(2, 0)];
        z.f[1] = v.f[tens_row(2, 1)];
        z.f[2] = v.f[tens_row(2, 2)];
        z.s = v.s;
    };
    auto put = [&](int sy, int sxx, const Full &v) {
        for (int q = 0; q < 4; ++q) sx[q][sy][sxx] = v.x[q];
        for (int t = 0; t < 6; ++t) sf[t][sy][sxx] = v.f[t];
        ss[sy][sxx] = v.s;
        sc[0][sy][sxx] = v.c[0];
        sc[1][sy][sxx] = v.c[1];
    };

    const int mzlo0 = map_axis(z0 - 1, g.nz, g.bclo[2], g.bchi[2]);
    Full cur[kCPT], nxt[kCPT], hcur;
    ZRow prev[kCPT];
    if (hly >= 0) load_full(hmx + (long long)g.nx * hmy + plane * z0, hcur);
    for (int c = 0; c < kCPT; ++c) {
        Full t;
        load_full(mx + (long long)g.nx * my[c] + plane * mzlo0, t);
        to_zrow(t, prev[c]);
        load_full(mx + (long long)g.nx * my[c] + plane * z0, cur[c]);
    }
    const AT tk = (AT)g.tau_k, nu = (AT)g.nu, half = AT(0.5) * (AT)g.nu;

    for (int k = z0; k < z1; ++k) {
        const int mzhi = map_axis(k + 1, g.nz, g.bclo[2], g.bchi[2]);
        const bool selfz_lo = map_axis(k - 1, g.nz, g.bclo[2], g.bchi[2]) == k;
        const bool selfz_hi = mzhi == k;
        for (int c = 0; c < kCPT; ++c) put(ly + kTYT * c + 1, lx + 1, cur[c]);
        if (hly >= 0) {
            put(hly, hlx, hcur);
            // prefetch the halo of the next plane (consumed one plane later)
            if (k + 1 < z1) load_full(hmx + (long long)g.nx * hmy + plane * (k + 1), hcur);
        }
        for (int c = 0; c < kCPT; ++c) load_full(mx + (long long)g.nx * my[c] + plane * mzhi, nxt[c]);
        lds_barrier();

        for (int c = 0; c < kCPT; ++c) {
            if (!active[c]) continue;
            const int sy = ly + kTYT * c + 1, sxx = lx + 1;
            const Full &C0 = cur[c];
            const AT Ec = C0.x[0];
            const AT Fc[3] = {C0.x[1], C0.x[2], C0.x[3]};
            AT dEs = 0, dF[3] = {0, 0, 0}, sumC_nb = 0;
            // x and y faces from LDS
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const AT fcr[3] = {C0.f[tens_row(d, 0)], C0.f[tens_row(d, 1)], C0.f[tens_row(d, 2)]};
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int ny_ = d == 1 ? sy + (side ? 1 : -1) : sy;
                    const int nx_ = d == 0 ? sxx + (side ? 1 : -1) : sxx;
                    const AT En = sx[0][ny_][nx_];
                    const AT Fn[3] = {sx[1][ny_][nx_], sx[2][ny_][nx_], sx[3][ny_][nx_]};
                    const AT fnr[3] = {sf[tens_row(d, 0)][ny_][nx_], sf[tens_row(d, 1)][ny_][nx_],
                                       sf[tens_row(d, 2)][ny_][nx_]};
                    // low face: own value; high face: the neighbour's low face
                    const AT Cface = pre ? (side ? sc[d][ny_][nx_] : C0.c[d])
                                         : face_speed<AT>(fcr[d], fnr[d], C0.s, ss[ny_][nx_], tk);
                    const bool self = d == 0 ? (side ? selfx_hi : selfx_lo) : (side ? selfy_hi[c] : selfy_lo[c]);
                    if (!self) sumC_nb += Cface;
                    face_flux_acc<AT>(d, side, Cface, Ec, Fc, fcr, En, Fn, fnr, dEs, dF);
                }
            }
            // z faces from registers
            {
                const AT fcr[3] = {C0.f[tens_row(2, 0)], C0.f[tens_row(2, 1)], C0.f[tens_row(2, 2)]};
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    AT En, Fn[3], fnr[3], sRn;
                    if (side) {
                        En = nxt[c].x[0];
                        for (int q = 0; q < 3; ++q) Fn[q] = nxt[c].x[1 + q];
                        for (int q = 0; q < 3; ++q) fnr[q] = nxt[c].f[tens_row(2, q)];
                        sRn = nxt[c].s;
                    } else {
                        En = prev[c].x[0];
                        for (int q = 0; q < 3; ++q) Fn[q] = prev[c].x[1 + q];
                        for (int q = 0; q < 3; ++q) fnr[q] = prev[c].f[q];
                        sRn = prev[c].s;
                    }
                    const AT Cface = pre ? (side ? nxt[c].c[2] : C0.c[2]) : face_speed<AT>(fcr[2], fnr[2], C0.s, sRn, tk);
                    if (!(side ? selfz_hi : selfz_lo)) sumC_nb += Cface;
                    face_flux_acc<AT>(2, side, Cface, Ec, Fc, fcr, En, Fn, fnr, dEs, dF);
                }
            }
            const long long idx = gx + (long long)g.nx * (y0 + ly + kTYT * c) + plane * k;
            const AT dEc = dE[idx];
            AT yE = dEc * Ec + nu * dEs;
            AT yFq[3];
            for (int q = 0; q < 3; ++q) yFq[q] = (AT(1) + C0.s) * Fc[q] + nu * dF[q];
            if (prec) {
                yE /= dEc + half * sumC_nb;
                const AT DF = AT(1) + C0.s + half * sumC_nb;
                for (int q = 0; q < 3; ++q) yFq[q] /= DF;
            }
            y[idx] = yE;
            for (int q = 0; q < 3; ++q) y[(1 + q) * N + idx] = yFq[q] * yF;
        }
        lds_barrier();
        for (int c = 0; c < kCPT; ++c) {
            to_zrow(cur[c], prev[c]);
            cur[c] = nxt[c];
        }
    }
}

// Low-face corrected speeds (divided by c) of every cell, once per step, in
// FP64 from the stored coefficients, rounded to the apply precision.
template <class CT, class AT>
__global__ void __launch_bounds__(256) k_face_coef(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kR,
                                                   const CT *__restrict__ f, AT *__restrict__ Cf)
{
    const long long N = g.N;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= N) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const double sRc = g.cdt * (double)rho[c] * (double)kR[c];
    for (int d = 0; d < 3; ++d) {
        const long long nb = neighbour(g, i, j, k, c, d, 0);
        const double sRn = g.cdt * (double)rho[nb] * (double)kR[nb];
        Cf[d * N + c] = (AT)face_speed<double>((double)f[d * N + nb], (double)f[d * N + c], sRn, sRc, g.tau_k);
    }
}

}  // namespace vr
