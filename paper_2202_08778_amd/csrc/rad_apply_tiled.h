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

#include <type_traits>

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

// Element `off` of the array that starts at `base`: a 64-bit uniform base and a
// 32-bit per-lane byte offset.
template <class T>
__device__ __forceinline__ T ld_off(const T *base, unsigned off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (size_t)(off * (unsigned)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void st_off(T *base, unsigned off, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (size_t)(off * (unsigned)sizeof(T))) = v;
}

// y = D^-1 A (s x) (PRE: Jacobi-scaled Krylov operator) or y = A x with flux
// rescaling xF/yF (!PRE: the physical operator).
// PRE: sR (c dt rho kappa_R) and Cf (the corrected face speeds divided by c at
// the three low faces of every cell, planes x|y|z) are precomputed once per step.
// !PRE: both are derived per cell and face from rho, kR and f.
// Offsets inside one z plane are 32-bit: nx * ny * 8 < 2^31 is checked on the host.
template <class AT, class ST, bool PRE>
__global__ void __launch_bounds__(256)
    k_apply_tiled(Grid g, TileGeom tg, const ST *__restrict__ f, const AT *__restrict__ sR,
                  const ST *__restrict__ rho, const ST *__restrict__ kR, const AT *__restrict__ Cf,
                  const AT *__restrict__ dE, const AT *__restrict__ x, const double *__restrict__ xs,
                  AT *__restrict__ y, AT xF, AT yF)
{
    // LDS record of one cell: x (4, scaled), f (6), sR, low-face speeds (PRE: 3)
    constexpr int NC = PRE ? 3 : 0;
    constexpr int IX = 0, IF = 4, IS = 10, IC = 11, NL = 11 + NC;
    __shared__ AT lds[2][NL][kLY][kLX];  // planes k and k+1, slot = plane parity

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

    const AT s = (PRE && xs) ? (AT)(*xs) : AT(1);
    const AT sF = s * xF;
    const AT cdt = (AT)g.cdt;

    // in-plane offsets of the thread's (mapped) cells and of its LDS halo cell
    const int gx = x0 + lx;
    const int mx = map_axis(gx, g.nx, g.bclo[0], g.bchi[0]);
    unsigned off[kCPT];
    bool active[kCPT];
    for (int c = 0; c < kCPT; ++c) {
        const int gy = y0 + ly + kTYT * c;
        off[c] = (unsigned)mx + (unsigned)g.nx * (unsigned)map_axis(gy, g.ny, g.bclo[1], g.bchi[1]);
        active[c] = gx < g.nx && gy < g.ny;  // then off[c] is the cell's own offset
    }
    int hly = -1, hlx = -1;
    unsigned hoff = 0;
    if (threadIdx.x < kHalo) {
        const int h = threadIdx.x;
        int gxh, gyh;
        if (h < kTX) { hlx = h + 1; hly = 0; gxh = x0 + h; gyh = y0 - 1; }
        else if (h < 2 * kTX) { hlx = h - kTX + 1; hly = kLY - 1; gxh = x0 + h - kTX; gyh = y0 + kTY; }
        else if (h < 2 * kTX + kTY) { hlx = 0; hly = h - 2 * kTX + 1; gxh = x0 - 1; gyh = y0 + h - 2 * kTX; }
        else { hlx = kLX - 1; hly = h - 2 * kTX - kTY + 1; gxh = x0 + kTX; gyh = y0 + h - 2 * kTX - kTY; }
        hoff = (unsigned)map_axis(gxh, g.nx, g.bclo[0], g.bchi[0]) +
               (unsigned)g.nx * (unsigned)map_axis(gyh, g.ny, g.bclo[1], g.bchi[1]);
    }
    // self-faces (mapped neighbour is the cell itself): excluded from the Jacobi diagonal
    const bool selfx_lo = map_axis(gx - 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    const bool selfx_hi = map_axis(gx + 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    bool selfy_lo[kCPT], selfy_hi[kCPT];
    for (int c = 0; c < kCPT; ++c) {
        const int gy = y0 + ly + kTYT * c;
        const int my = map_axis(gy, g.ny, g.bclo[1], g.bchi[1]);
        selfy_lo[c] = map_axis(gy - 1, g.ny, g.bclo[1], g.bchi[1]) == my;
        selfy_hi[c] = map_axis(gy + 1, g.ny, g.bclo[1], g.bchi[1]) == my;
    }
    auto mapz = [&](int q) { return map_axis(q, g.nz, g.bclo[2], g.bchi[2]); };

    // one cell's record in registers (in flight from HBM), plus its dE
    struct Full {
        AT v[NL];
        AT d;
    };
    // z-neighbour subset below the current plane: x (4), f row z (xz, yz, zz), sR
    struct ZRow {
        AT x[4], f[3], s;
    };
    auto load_full = [&](int kp, unsigned o, Full &u, bool own) __attribute__((always_inline)) {
        const long long pb = plane * kp;
        u.v[IX] = s * ld_off(x + pb, o);
#pragma unroll
        for (int q = 1; q < 4; ++q) u.v[IX + q] = sF * ld_off(x + q * N + pb, o);
#pragma unroll
        for (int t = 0; t < 6; ++t) u.v[IF + t] = (AT)ld_off(f + t * N + pb, o);
        if constexpr (PRE) {
            u.v[IS] = ld_off(sR + pb, o);
#pragma unroll
            for (int d = 0; d < NC; ++d) u.v[IC + d] = ld_off(Cf + d * N + pb, o);
        } else {
            u.v[IS] = cdt * (AT)ld_off(rho + pb, o) * (AT)ld_off(kR + pb, o);
        }
        u.d = (PRE && own) ? ld_off(dE + pb, o) : AT(0);
    };
    auto put = [&](int sl, int sy, int sxx, const Full &u) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < NL; ++q) lds[sl][q][sy][sxx] = u.v[q];
    };

    ZRow prev[kCPT];
    AT dcur[kCPT], dnxt[kCPT];
    const AT tk = (AT)g.tau_k, nu = (AT)g.nu, half = AT(0.5) * (AT)g.nu;

    // Plane k of the tile from LDS slot a, its upper z neighbour from slot b,
    // the lower one from registers; writes y for the thread's cells.
    auto compute = [&](int k, int a, int b) __attribute__((always_inline)) {
        const long long pb = plane * k;
        const bool selfz_lo = mapz(k - 1) == k, selfz_hi = mapz(k + 1) == k;
#pragma unroll
        for (int c = 0; c < kCPT; ++c) {
            // ragged-edge cells are computed from their mapped (in-range) values
            // and not stored, so the arithmetic has no divergent branch
            const int sy = ly + kTYT * c + 1, sxx = lx + 1;
            const AT Ec = lds[a][IX][sy][sxx];
            const AT Fc[3] = {lds[a][IX + 1][sy][sxx], lds[a][IX + 2][sy][sxx], lds[a][IX + 3][sy][sxx]};
            const AT sc = lds[a][IS][sy][sxx];
            AT dEs = 0, dF[3] = {0, 0, 0}, sumC_nb = 0;
            // x and y faces
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const AT fcr[3] = {lds[a][IF + tens_row(d, 0)][sy][sxx], lds[a][IF + tens_row(d, 1)][sy][sxx],
                                   lds[a][IF + tens_row(d, 2)][sy][sxx]};
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int ny_ = d == 1 ? sy + (side ? 1 : -1) : sy;
                    const int nx_ = d == 0 ? sxx + (side ? 1 : -1) : sxx;
                    const AT En = lds[a][IX][ny_][nx_];
                    const AT Fn[3] = {lds[a][IX + 1][ny_][nx_], lds[a][IX + 2][ny_][nx_], lds[a][IX + 3][ny_][nx_]};
                    const AT fnr[3] = {lds[a][IF + tens_row(d, 0)][ny_][nx_], lds[a][IF + tens_row(d, 1)][ny_][nx_],
                                       lds[a][IF + tens_row(d, 2)][ny_][nx_]};
                    // low face: own value; high face: the neighbour's low face
                    AT Cface;
                    if constexpr (PRE)
                        Cface = side ? lds[a][IC + d][ny_][nx_] : lds[a][IC + d][sy][sxx];
                    else
                        Cface = face_speed<AT>(fcr[d], fnr[d], sc, lds[a][IS][ny_][nx_], tk);
                    const bool self = d == 0 ? (side ? selfx_hi : selfx_lo) : (side ? selfy_hi[c] : selfy_lo[c]);
                    sumC_nb += self ? AT(0) : Cface;
                    face_flux_acc<AT>(d, side, Cface, Ec, Fc, fcr, En, Fn, fnr, dEs, dF);
                }
            }
            // z faces
            const AT fcr[3] = {lds[a][IF + tens_row(2, 0)][sy][sxx], lds[a][IF + tens_row(2, 1)][sy][sxx],
                               lds[a][IF + tens_row(2, 2)][sy][sxx]};
            {
                const AT En = lds[b][IX][sy][sxx];
                const AT Fn[3] = {lds[b][IX + 1][sy][sxx], lds[b][IX + 2][sy][sxx], lds[b][IX + 3][sy][sxx]};
                const AT fnr[3] = {lds[b][IF + tens_row(2, 0)][sy][sxx], lds[b][IF + tens_row(2, 1)][sy][sxx],
                                   lds[b][IF + tens_row(2, 2)][sy][sxx]};
                AT Cface;
                if constexpr (PRE)
                    Cface = lds[b][IC + 2][sy][sxx];
                else
                    Cface = face_speed<AT>(fcr[2], fnr[2], sc, lds[b][IS][sy][sxx], tk);
                sumC_nb += selfz_hi ? AT(0) : Cface;
                face_flux_acc<AT>(2, 1, Cface, Ec, Fc, fcr, En, Fn, fnr, dEs, dF);
            }
            {
                const ZRow &P = prev[c];
                const AT Fn[3] = {P.x[1], P.x[2], P.x[3]};
                AT Cface;
                if constexpr (PRE)
                    Cface = lds[a][IC + 2][sy][sxx];
                else
                    Cface = face_speed<AT>(fcr[2], P.f[2], sc, P.s, tk);
                sumC_nb += selfz_lo ? AT(0) : Cface;
                face_flux_acc<AT>(2, 0, Cface, Ec, Fc, fcr, P.x[0], Fn, P.f, dEs, dF);
            }
            AT yE, yFq[3];
            if constexpr (PRE) {
                const AT dEc = dcur[c];
                yE = (dEc * Ec + nu * dEs) * (AT(1) / (dEc + half * sumC_nb));
                const AT iDF = AT(1) / (AT(1) + sc + half * sumC_nb);
                for (int q = 0; q < 3; ++q) yFq[q] = ((AT(1) + sc) * Fc[q] + nu * dF[q]) * iDF;
            } else {
                const AT dEc = ld_off(dE + pb, off[c]);
                yE = dEc * Ec + nu * dEs;
                for (int q = 0; q < 3; ++q) yFq[q] = (AT(1) + sc) * Fc[q] + nu * dF[q];
            }
            if (active[c]) {
                st_off(y + pb, off[c], yE);
                for (int q = 0; q < 3; ++q) st_off(y + (1 + q) * N + pb, off[c], yFq[q] * yF);
            }
            // this plane becomes the lower neighbour of the next one
            ZRow &P = prev[c];
            P.x[0] = Ec;
            for (int q = 0; q < 3; ++q) P.x[1 + q] = Fc[q];
            for (int q = 0; q < 3; ++q) P.f[q] = fcr[q];
            P.s = sc;
        }
    };

    // Pipeline: plane k is computed while planes k+2 and k+3 are in flight
    // (two register sets used alternately), so each load has two planes of
    // work to arrive before it is written to LDS.  Every load of the steady
    // state is unconditional (lanes without a halo cell re-read their own
    // cell, an L2 hit), so the compiler's wait counts stay two planes deep.
    const unsigned hsrc = hly >= 0 ? hoff : off[0];
    Full S0[kCPT], S1[kCPT], H0, H1;
    {
        Full t;
        for (int c = 0; c < kCPT; ++c) {
            load_full(mapz(z0 - 1), off[c], t, false);
            prev[c].x[0] = t.v[IX];
            for (int q = 0; q < 3; ++q) prev[c].x[1 + q] = t.v[IX + 1 + q];
            for (int q = 0; q < 3; ++q) prev[c].f[q] = t.v[IF + tens_row(2, q)];
            prev[c].s = t.v[IS];
        }
        for (int c = 0; c < kCPT; ++c) {
            load_full(z0, off[c], t, true);
            put(0, ly + kTYT * c + 1, lx + 1, t);
            dcur[c] = t.d;
        }
        load_full(z0, hsrc, t, false);
        if (hly >= 0) put(0, hly, hlx, t);
    }
    for (int c = 0; c < kCPT; ++c) load_full(mapz(z0 + 1), off[c], S0[c], true);
    load_full(mapz(z0 + 1), hsrc, H0, false);
    for (int c = 0; c < kCPT; ++c) load_full(mapz(min(z0 + 2, z1)), off[c], S1[c], true);
    load_full(mapz(min(z0 + 2, z1)), hsrc, H1, false);

    // one plane: LOAD issues plane k+3 (needed when k+3 <= z1)
    auto iter = [&](auto LOAD, int t, Full (&S)[kCPT], Full &H) __attribute__((always_inline)) {
        const int k = z0 + t;
        const int a = t & 1, b = a ^ 1;
        // plane k+1 (issued two planes ago) into the free slot
        for (int c = 0; c < kCPT; ++c) {
            put(b, ly + kTYT * c + 1, lx + 1, S[c]);
            dnxt[c] = S[c].d;
        }
        if (hly >= 0) put(b, hly, hlx, H);
        if constexpr (decltype(LOAD)::value) {
            const int kp = mapz(k + 3);
            for (int c = 0; c < kCPT; ++c) load_full(kp, off[c], S[c], true);
            load_full(kp, hsrc, H, false);
        }
        lds_barrier();
        compute(k, a, b);
        lds_barrier();
        for (int c = 0; c < kCPT; ++c) dcur[c] = dnxt[c];
    };
    constexpr std::true_type L1{};
    constexpr std::false_type L0{};
    const int nzr = z1 - z0;
    int t = 0;
    for (; t + 4 <= nzr; t += 2) {
        iter(L1, t, S0, H0);
        iter(L1, t + 1, S1, H1);
    }
    // the last one to three planes (t is even)
    const int r = nzr - t;
    if (r == 3) {
        iter(L1, t, S0, H0);
        iter(L0, t + 1, S1, H1);
        iter(L0, t + 2, S0, H0);
    } else if (r == 2) {
        iter(L0, t, S0, H0);
        iter(L0, t + 1, S1, H1);
    } else if (r == 1) {
        iter(L0, t, S0, H0);
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
