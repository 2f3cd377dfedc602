// rad_apply_tiled.h -- the transport stencil as a 2.5D z-marching tile sweep (gfx950).
//
// A workgroup owns a 64 x 8 cell column of the grid over a range of z planes
// (FP32: 256 threads, each with two cells adjacent along y; FP64: 512 threads,
// one cell each).  Two LDS slots hold the planes k and k+1 of the tile with a one-cell
// x/y halo (state, tensor, sR, low-face speeds); the plane k-1 of the thread's
// own cells lives in registers.  Planes k+2 and k+3 are in flight in two
// register sets used alternately, so every HBM value is read once per z-range
// and each load has two planes of work to arrive (the halo rows are read by the
// neighbouring tile too and hit in L2, since tiles are assigned to XCDs in
// contiguous ranges).  Every LDS slot and every z neighbour is first mapped
// through the boundary rule (periodic: wrap, any wall: the boundary cell
// itself), so boundary faces and ragged tile edges need no special cases: a
// zero-gradient wall's face carries the cell's physical flux and no
// dissipation.  A Dirichlet, open, Marshak or reflecting face adds the
// difference to the flux against its ghost, which is local to the cell (the
// HLLE flux is linear in the neighbour's state): tiles holding such cells
// compute it in uniform branches on every lane and keep it on the face's lanes,
// so the sweep carries no per-lane branch, and the Krylov operator no ghost data
// (the residual reads a Dirichlet face's data in those branches only).  The per-cell epilogue is a functor:
// the Krylov operator apply and the FP64 residual of one Picard iteration
// share the sweep.
#pragma once
#include "rad_device.h"
#include "rad_amr.h"

#include <algorithm>
#include <type_traits>

namespace vr {

constexpr int kTX = 64;  // tile width (x), one wave per row
constexpr int kLX = kTX + 2;

// thread rows of the tile, cells per thread along y and planes in flight
// (prefetch depth), by arithmetic type; every shape covers the same 64 x 8 cell
// tile.  One cell per thread and one plane in flight keep the FP32 sweep within
// 128 VGPRs: two 512-thread workgroups per CU (their 75-81 KB of LDS each) give 4
// waves per SIMD.  Measured at 256^3 against two cells per thread with two planes
// in flight (PAIR: 256 threads, 231-245 VGPRs, 2 waves per SIMD): 295 against 317
// us per Krylov apply, and 290 against 302 ms per multigrid step.  The two-level
// grid's sweeps, whose jump terms would spill at 128 VGPRs, keep PAIR (1255
// against 1305 ms per step).  FP64 records take twice the registers; its LDS
// allows one workgroup per CU.
template <class AT, bool PAIR = false>
struct TileShape {
    static constexpr int TYT = PAIR ? 4 : 8, CPT = PAIR ? 2 : 1, DEPTH = PAIR ? 2 : 1;
    static constexpr int TY = TYT * CPT, LY = TY + 2, HALO = 2 * kTX + 2 * TY;
};
template <bool PAIR>
struct TileShape<double, PAIR> {
    static constexpr int TYT = 8, CPT = 1, DEPTH = 1;
    static constexpr int TY = TYT * CPT, LY = TY + 2, HALO = 2 * kTX + 2 * TY;
};
template <class AT, bool PAIR = false>
constexpr int tile_threads()
{
    return 64 * TileShape<AT, PAIR>::TYT;
}

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

// kz_req > 0: that z-range (planes per workgroup, clipped to nz).  Otherwise
// the default rule: the longest range up to kz_cap planes (so the two extra
// planes a column reads stay a small fraction, while x/y neighbours progress
// together and their shared halo rows hit in L2) that still gives min_tiles
// workgroups to fill the chip.  Defaults measured at 256^3 and 512^3: the Krylov
// apply is fastest at 32 planes, and so is the FP64 residual (one 512-thread
// workgroup per CU; 2.94 / 3.08 / 3.16 / 3.10 TB/s at 128 / 64 / 32 / 16 planes at
// 256^3, 3.22 / 3.31 / 3.39 / 3.41 at 512^3).
template <class AT>
inline TileGeom tile_geom(const Grid &g, int kz_req = 0, int kz_cap = 32, long long min_tiles = 1024)
{
    constexpr int TY = TileShape<AT>::TY;
    TileGeom t;
    t.tiles_x = (g.nx + kTX - 1) / kTX;
    t.tiles_y = (g.ny + TY - 1) / TY;
    if (kz_req > 0) {
        t.kz = std::min(kz_req, g.nz);
        t.tiles_z = (g.nz + t.kz - 1) / t.kz;
        return t;
    }
    const long long cols = (long long)t.tiles_x * t.tiles_y;
    int kz = g.nz;
    while (kz > 8 && (kz > kz_cap || cols * ((g.nz + kz - 1) / kz) < min_tiles)) kz = (kz + 1) / 2;
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

// LDS record of one cell: x (4, scaled), f (6), sR, low-face speeds (PRE: 3)
template <bool PRE>
struct Rec {
    static constexpr int IX = 0, IF = 4, IS = 10, IC = 11, NL = 11 + (PRE ? 3 : 0);
};

// The coarse level of a multigrid pair, for sweeps fused with the transfers
// between the two levels (FP32 tiles, whose threads hold y-pairs of cells):
// restriction (the sweep's output t accumulates into the parents' right-hand
// side qc = Dc^-1 mean_children(D t), D the Jacobi diagonal) and injection (the
// sweep's operand is a x + ec(parent), the parents' coarse correction added as
// the operand is loaded).
template <class AT>
struct MgFuse {
    AT *qc = nullptr;         // restriction: the parents' right-hand side (4 planes)
    const AT *Dc = nullptr;   // restriction: the parents' Jacobi diagonal (E row, F rows)
    const AT *ec = nullptr;   // injection: the parents' correction (4 planes)
    AT a = AT(1);             // injection: the operand's factor
    long long Nc = 0;         // cells of the coarse level
    int ncx = 0, ncy = 0;     // its extents in x and y
};

// Transport sums of one cell: dEs = sum_faces +-PhiE, dF likewise (without the
// factor nu), the face speeds of the faces between two cells (Jacobi diagonal)
// and of all six faces (residual weights; a wall face takes the cell's own
// speed), and the walls' own shares of the Jacobi diagonal per row (wE, wF;
// zero away from Dirichlet, open, Marshak and reflecting faces).
template <class AT>
struct CellSums {
    AT Ec, Fc[3], sc, dEs, dF[3], sumC_nb, sumC_all, wE, wF[3];
};

// The workgroup's tile in XCD-aware order: consecutive workgroup ids go to different XCDs, so each
// XCD gets a contiguous range of tiles (neighbours share halo rows in L2).
__device__ __forceinline__ void tile_coords(const TileGeom &tg, int &bx, int &by, int &bz)
{
    const int ntiles = gridDim.x;
    int tile = blockIdx.x;
    if (ntiles % 8 == 0) tile = (blockIdx.x % 8) * (ntiles / 8) + blockIdx.x / 8;
    bx = tile % tg.tiles_x;
    const int rest = tile / tg.tiles_x;
    by = rest % tg.tiles_y;
    bz = rest / tg.tiles_y;
}

// The sweep.  PRE: sR is precomputed, otherwise derived from rho and kR.  CST
// (PRE only): the low-face speeds Cf (divided by c, planes x|y|z) are
// precomputed too; otherwise each face's speed is formed from f and sR.
// lex(k, pb, o, e) loads the NE per-cell extras of the epilogue (plane k, its
// base pb, in-plane offset o); epi(k, c, o, active, sums, e) consumes one cell;
// wall(kind, d, side, Ec, Fc, fcr, e, fi, Eg, Fg, fg) forms the ghost across a
// Dirichlet, open, Marshak or reflecting face from the cell's values (its extras e
// and its index fi on the face); WL: the grid has such faces (0: none, and no wall
// code at all; 1: open, Marshak and reflecting walls; 2: Dirichlet faces too -- a
// separate level, since a fourth specialised branch costs the other kinds registers).
// Offsets inside one z plane are 32-bit: nx * ny * 8 < 2^31 is checked on the host.
// beg(k) runs at the start of plane k's step, after the barrier that ended plane k - 1 and once the
// prefetched record has gone to LDS (its registers free), before the next plane's loads are issued.
struct NoPlaneHook {
    __device__ void operator()(int) const {}
};
template <class AT, class ST, bool PRE, bool CALL, int NE, bool CST = PRE, int WL = 0, bool INJ = false,
          bool PAIR = false, class LEX, class EPI, class WALL, class BEG = NoPlaneHook>
__device__ __forceinline__ void tile_sweep(const Grid &g, const TileGeom &tg, const ST *__restrict__ f,
                                           const AT *__restrict__ sR, const ST *__restrict__ rho,
                                           const ST *__restrict__ kR, const AT *__restrict__ Cf,
                                           const AT *__restrict__ x, AT s, AT sF,
                                           AT (&lds)[2][Rec<CST>::NL][TileShape<AT, PAIR>::LY][kLX], LEX lex, EPI epi,
                                           WALL wall, const MgFuse<AT> &mf = MgFuse<AT>{},
                                           const AT *__restrict__ cw = nullptr, BEG beg = BEG{})
{
    using TS = TileShape<AT, PAIR>;
    constexpr int CPT = TS::CPT;   // a thread's cells: rows CPT ly + c of the tile
    constexpr int kTY = TS::TY, kLY = TS::LY, kHalo = TS::HALO;
    static_assert(PRE || !CST, "stored face speeds come with stored sR");
    static_assert(!CALL || CST, "the nonlinear residual reads stored face speeds");
    constexpr int NC = CST ? 3 : 0;
    constexpr int IX = Rec<CST>::IX, IF = Rec<CST>::IF, IS = Rec<CST>::IS, IC = Rec<CST>::IC, NL = Rec<CST>::NL;

    const long long N = g.N;
    const long long plane = (long long)g.nx * g.ny;
    int bx, by, bz;
    tile_coords(tg, bx, by, bz);
    const int x0 = bx * kTX, y0 = by * kTY, z0 = bz * tg.kz;
    const int z1 = min(z0 + tg.kz, g.nz);
    const int lx = threadIdx.x % kTX, ly = threadIdx.x / kTX;
    const AT cdt = (AT)g.cdt;

    // in-plane offsets of the thread's (mapped) cells and of its LDS halo cell
    const int gx = x0 + lx;
    const int mx = map_axis(gx, g.nx, g.bclo[0], g.bchi[0]);
    unsigned off[CPT], poff[CPT];   // poff (injection): the parents' in-plane offsets
    bool active[CPT];
    for (int c = 0; c < CPT; ++c) {
        const int gy = y0 + CPT * ly + c;
        const int my = map_axis(gy, g.ny, g.bclo[1], g.bchi[1]);
        off[c] = (unsigned)mx + (unsigned)g.nx * (unsigned)my;
        // (a ragged row past the grid maps to the last row: its parent is in range, and it is not stored)
        poff[c] = INJ ? (unsigned)(mx >> 1) + (unsigned)mf.ncx * (unsigned)(my >> 1) : 0u;
        active[c] = gx < g.nx && gy < g.ny;  // then off[c] is the cell's own offset
    }
    int hly = -1, hlx = -1;
    unsigned hoff = 0, phoff = 0;
    int gxh = 0, gyh = 0;
    if (threadIdx.x < kHalo) {
        const int h = threadIdx.x;
        if (h < kTX) { hlx = h + 1; hly = 0; gxh = x0 + h; gyh = y0 - 1; }
        else if (h < 2 * kTX) { hlx = h - kTX + 1; hly = kLY - 1; gxh = x0 + h - kTX; gyh = y0 + kTY; }
        else if (h < 2 * kTX + kTY) { hlx = 0; hly = h - 2 * kTX + 1; gxh = x0 - 1; gyh = y0 + h - 2 * kTX; }
        else { hlx = kLX - 1; hly = h - 2 * kTX - kTY + 1; gxh = x0 + kTX; gyh = y0 + h - 2 * kTX - kTY; }
        const int mxh = map_axis(gxh, g.nx, g.bclo[0], g.bchi[0]), myh = map_axis(gyh, g.ny, g.bclo[1], g.bchi[1]);
        hoff = (unsigned)mxh + (unsigned)g.nx * (unsigned)myh;
        if (INJ) phoff = (unsigned)(mxh >> 1) + (unsigned)mf.ncx * (unsigned)(myh >> 1);
    }
    // self-faces (mapped neighbour is the cell itself): excluded from the Jacobi diagonal
    const bool selfx_lo = map_axis(gx - 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    const bool selfx_hi = map_axis(gx + 1, g.nx, g.bclo[0], g.bchi[0]) == mx;
    bool selfy_lo[CPT], selfy_hi[CPT];
    for (int c = 0; c < CPT; ++c) {
        const int gy = y0 + CPT * ly + c;
        const int my = map_axis(gy, g.ny, g.bclo[1], g.bchi[1]);
        selfy_lo[c] = map_axis(gy - 1, g.ny, g.bclo[1], g.bchi[1]) == my;
        selfy_hi[c] = map_axis(gy + 1, g.ny, g.bclo[1], g.bchi[1]) == my;
    }
    auto mapz = [&](int q) { return map_axis(q, g.nz, g.bclo[2], g.bchi[2]); };
    // the six faces' kinds packed 4 bits each (face 2 d + side), and the faces of the thread's cells on
    // Dirichlet, open, Marshak or reflecting faces (bits: x lo, x hi, y lo, y hi)
    unsigned kinds = 0;
    for (int fi = 0; fi < 6; ++fi) kinds |= (unsigned)((fi & 1) ? g.bchi[fi >> 1] : g.bclo[fi >> 1]) << (4 * fi);
    auto kind_of = [&](int d, int side) { return (int)((kinds >> (4 * (2 * d + side))) & 15u); };
    const bool zwall_lo = WL && ghost_face(kind_of(2, 0)), zwall_hi = WL && ghost_face(kind_of(2, 1));
    unsigned wmask[CPT];
    for (int c = 0; c < CPT; ++c)
        wmask[c] = !(WL && active[c]) ? 0u
                   : (selfx_lo && ghost_face(kind_of(0, 0)) ? 1u : 0u) | (selfx_hi && ghost_face(kind_of(0, 1)) ? 2u : 0u) |
                         (selfy_lo[c] && ghost_face(kind_of(1, 0)) ? 4u : 0u) |
                         (selfy_hi[c] && ghost_face(kind_of(1, 1)) ? 8u : 0u);
    // tiles holding cells on such walls (uniform; bits as wmask)
    const unsigned twall = !WL ? 0u
                           : (x0 == 0 && ghost_face(kind_of(0, 0)) ? 1u : 0u) |
                                 (x0 + kTX >= g.nx && ghost_face(kind_of(0, 1)) ? 2u : 0u) |
                                 (y0 == 0 && ghost_face(kind_of(1, 0)) ? 4u : 0u) |
                                 (y0 + kTY >= g.ny && ghost_face(kind_of(1, 1)) ? 8u : 0u);
    // A high wall's speed is the cell's own, which the stored low-face speeds do not hold.  Sweeps of
    // tiles on a high x wall (a quarter of the tiles at 256^3) read it from cw (per step: x walls [nz][ny],
    // then y walls [nz][nx], then z walls [ny][nx]), staged into LDS for the tile's z-range: FP32 Krylov
    // sweeps (1 KB, so that two workgroups still share a CU) and the FP64 residual (8 KB beside its 145 KB,
    // one workgroup per CU either way).  The rarer high y and z walls, and longer z-ranges, form it.
    constexpr int kWz = CALL ? 128 : 32;
    constexpr bool WST = WL && CST && (CALL || sizeof(AT) == 4);
    __shared__ std::conditional_t<WST, AT[kWz * kTY], AT[1]> wsp;
    const bool wlds = WST && cw != nullptr && tg.kz <= kWz && (twall & 2u);
    if constexpr (WST) {
        if (wlds)
            for (int t = threadIdx.x; t < (z1 - z0) * kTY; t += blockDim.x)
                wsp[t] = cw[(long long)(z0 + t / kTY) * g.ny + min(y0 + t % kTY, g.ny - 1)];
    }

    // one cell's record in registers (in flight from HBM)
    struct Full {
        AT v[NL];
    };
    // z-neighbour subset below the current plane: x (4), f row z (xz, yz, zz), sR
    struct ZRow {
        AT x[4], f[3], s;
    };
    // the operand's 4 values of the cell at plane kp, offset o (parent offset po)
    auto load_x = [&](int kp, unsigned o, unsigned po, AT *v) __attribute__((always_inline)) {
        const long long pb = plane * kp;
        if constexpr (INJ) {
            const long long pp = (long long)(kp >> 1) * mf.ncx * mf.ncy;
            v[0] = s * (mf.a * ld_off(x + pb, o) + ld_off(mf.ec + pp, po));
#pragma unroll
            for (int q = 1; q < 4; ++q) v[q] = sF * (mf.a * ld_off(x + q * N + pb, o) + ld_off(mf.ec + q * mf.Nc + pp, po));
        } else {
            v[0] = s * ld_off(x + pb, o);
#pragma unroll
            for (int q = 1; q < 4; ++q) v[q] = sF * ld_off(x + q * N + pb, o);
        }
    };
    auto load_full = [&](int kp, unsigned o, unsigned po, Full &u) __attribute__((always_inline)) {
        const long long pb = plane * kp;
        load_x(kp, o, po, u.v + IX);
#pragma unroll
        for (int t = 0; t < 6; ++t) u.v[IF + t] = (AT)ld_off(f + t * N + pb, o);
        if constexpr (PRE) {
            u.v[IS] = ld_off(sR + pb, o);
#pragma unroll
            for (int d = 0; d < NC; ++d) u.v[IC + d] = ld_off(Cf + d * N + pb, o);   // NC = 0 unless CST
        } else {
            u.v[IS] = cdt * (AT)ld_off(rho + pb, o) * (AT)ld_off(kR + pb, o);
        }
    };
    auto put = [&](int sl, int sy, int sxx, const Full &u) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < NL; ++q) lds[sl][q][sy][sxx] = u.v[q];
    };
    // A halo cell is read only as the neighbour across its own axis (x for the side
    // columns, y for the top and bottom rows): its state, that row of the tensor and
    // its low-face speed of that axis (PRE) or its sR.  Lanes without a halo cell
    // re-read their own cell along x (an L2 hit), so the loads stay unconditional.
    // The apply loads these 8 values; the residual (CALL), whose FP64 records leave
    // fewer registers, keeps the whole record (the lane-dependent planes cost it spills).
    constexpr bool SLIM = !CALL;
    const int hax = (threadIdx.x < 2 * kTX) ? 1 : 0;
    struct Halo {
        AT v[8];
    };
    auto load_halo = [&](int kp, unsigned o, unsigned po, Halo &u) __attribute__((always_inline)) {
        const long long pb = plane * kp;
        load_x(kp, o, po, u.v);
#pragma unroll
        for (int q = 0; q < 3; ++q) u.v[4 + q] = (AT)ld_off(f + tens_row(hax, q) * N + pb, o);
        if constexpr (CST)
            u.v[7] = ld_off(Cf + hax * N + pb, o);
        else if constexpr (PRE)
            u.v[7] = ld_off(sR + pb, o);
        else
            u.v[7] = cdt * (AT)ld_off(rho + pb, o) * (AT)ld_off(kR + pb, o);
    };
    auto put_halo = [&](int sl, const Halo &u) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) lds[sl][IX + q][hly][hlx] = u.v[q];
#pragma unroll
        for (int q = 0; q < 3; ++q) lds[sl][IF + tens_row(hax, q)][hly][hlx] = u.v[4 + q];
        if constexpr (CST)
            lds[sl][IC + hax][hly][hlx] = u.v[7];
        else
            lds[sl][IS][hly][hlx] = u.v[7];
    };

    const AT tk = (AT)g.tau_k;
    // The correction that turns the flux of ghost face (d, side) of a cell from the self-mapped one
    // the sweep computed (neighbour = the cell itself: the cell's physical flux, whatever the speed)
    // into the flux against the face's ghost, which the wall functor forms from the cell's state,
    // tensor row and (the nonlinear residual) the face's data at the cell's index fi on the face
    // (x faces [nz][ny], y faces [nz][nx], z faces [ny][nx], formed from the mapped coordinates:
    // in range on every lane); plus the face's shares of the Jacobi diagonal.  Cw: the face's speed
    // (the cell's own).  m: 1 for a cell on the face, else 0 -- the correction is computed by every
    // lane of a tile holding such cells (uniform branches, no per-lane ones) and kept by those on
    // the face.  (d is a constant once the face loops are unrolled)
    auto wall_fix_k = [&](auto K, int d, int side, AT m, AT Cw, const AT(&fr)[3], const AT(&e)[NE > 0 ? NE : 1],
                          int k, int c, CellSums<AT> &S) __attribute__((always_inline)) {
        constexpr int kind = decltype(K)::value;
        const unsigned my = (unsigned)map_axis(y0 + CPT * ly + c, g.ny, g.bclo[1], g.bchi[1]);
        const unsigned fi = d == 0 ? (unsigned)k * (unsigned)g.ny + my
                                   : (d == 1 ? (unsigned)k * (unsigned)g.nx + (unsigned)mx
                                             : my * (unsigned)g.nx + (unsigned)mx);
        AT Eg, Fg[3], fg[3];
        wall(kind, d, side, S.Ec, S.Fc, fr, e, fi, Eg, Fg, fg);
        const AT sg = side ? AT(1) : AT(-1), ms = m * sg, hc = AT(-0.5) * sg * Cw;
        S.dEs += ms * (AT(0.5) * (Fg[d] - S.Fc[d]) + hc * (Eg - S.Ec));
#pragma unroll
        for (int q = 0; q < 3; ++q) S.dF[q] += ms * (AT(0.5) * (fg[q] * Eg - fr[q] * S.Ec) + hc * (Fg[q] - S.Fc[q]));
        if constexpr (PRE) {
            AT qE, qF, qX;
            wall_diag_q<AT>(kind, d, fr, Cw, qE, qF, qX);
            S.wE += m * qE;
            if constexpr (kind == BC_DIRICHLET) {
#pragma unroll
                for (int q = 0; q < 3; ++q) S.wF[q] += m * (q == d ? qF : qX);
            } else {
                S.wF[d] += m * qF;
            }
        }
    };
    // the kind is uniform: a scalar branch to code specialised for it
    auto wall_fix = [&](int kind, int d, int side, AT m, AT Cw, const AT(&fr)[3], const AT(&e)[NE > 0 ? NE : 1],
                        int k, int c, CellSums<AT> &S) __attribute__((always_inline)) {
        if (kind == BC_OPEN)
            wall_fix_k(std::integral_constant<int, BC_OPEN>{}, d, side, m, Cw, fr, e, k, c, S);
        else if (kind == BC_MARSHAK)
            wall_fix_k(std::integral_constant<int, BC_MARSHAK>{}, d, side, m, Cw, fr, e, k, c, S);
        else if (WL == 2 && kind == BC_DIRICHLET) {
            if constexpr (WL == 2)
                wall_fix_k(std::integral_constant<int, BC_DIRICHLET>{}, d, side, m, Cw, fr, e, k, c, S);
        } else {
            wall_fix_k(std::integral_constant<int, BC_REFLECT>{}, d, side, m, Cw, fr, e, k, c, S);
        }
    };

    ZRow prev[CPT];
    AT ex[CPT][NE > 0 ? NE : 1];

    // Plane k of the tile from LDS slot a, its upper z neighbour from slot b,
    // the lower one from registers.
    auto compute = [&](int k, int a, int b) __attribute__((always_inline)) {
        const bool selfz_lo = mapz(k - 1) == k, selfz_hi = mapz(k + 1) == k;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            // ragged-edge cells are computed from their mapped (in-range) values
            // and not stored, so the arithmetic has no divergent branch
            const int sy = CPT * ly + c + 1, sxx = lx + 1;
            CellSums<AT> S;
            S.Ec = lds[a][IX][sy][sxx];
            for (int q = 0; q < 3; ++q) S.Fc[q] = lds[a][IX + 1 + q][sy][sxx];
            S.sc = lds[a][IS][sy][sxx];
            S.dEs = 0;
            S.dF[0] = S.dF[1] = S.dF[2] = 0;
            S.sumC_nb = 0;
            S.sumC_all = 0;
            S.wE = 0;
            S.wF[0] = S.wF[1] = S.wF[2] = 0;
            // a self face's speed for the residual weights: the cell with itself
            auto self_speed = [&](AT fdd) { return face_speed<AT>(fdd, fdd, S.sc, S.sc, tk); };
            // x and y faces
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const AT fcr[3] = {lds[a][IF + tens_row(d, 0)][sy][sxx], lds[a][IF + tens_row(d, 1)][sy][sxx],
                                   lds[a][IF + tens_row(d, 2)][sy][sxx]};
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int ny_ = d == 1 ? sy + (side ? 1 : -1) : sy;
                    const int nx_ = d == 0 ? sxx + (side ? 1 : -1) : sxx;
                    AT En = lds[a][IX][ny_][nx_];
                    AT Fn[3] = {lds[a][IX + 1][ny_][nx_], lds[a][IX + 2][ny_][nx_], lds[a][IX + 3][ny_][nx_]};
                    AT fnr[3] = {lds[a][IF + tens_row(d, 0)][ny_][nx_], lds[a][IF + tens_row(d, 1)][ny_][nx_],
                                 lds[a][IF + tens_row(d, 2)][ny_][nx_]};
                    // low face: own value; high face: the neighbour's low face
                    AT Cface;
                    if constexpr (CST)
                        Cface = side ? lds[a][IC + d][ny_][nx_] : lds[a][IC + d][sy][sxx];
                    else
                        Cface = face_speed<AT>(fcr[d], fnr[d], S.sc, lds[a][IS][ny_][nx_], tk);
                    const bool self = d == 0 ? (side ? selfx_hi : selfx_lo) : (side ? selfy_hi[c] : selfy_lo[c]);
                    S.sumC_nb += self ? AT(0) : Cface;
                    if constexpr (CALL) {
                        if (CST && side && self)
                            S.sumC_all += self_speed(fcr[d]);
                        else
                            S.sumC_all += Cface;
                    }
                    face_flux_acc<AT>(d, side, Cface, S.Ec, S.Fc, fcr, En, Fn, fnr, S.dEs, S.dF);
                    // a Dirichlet, open, Marshak or reflecting face (y: the lowest row only holds the first cell);
                    // its speed: a low face's stored speed is the cell's own, a high face's is formed
                    if (WL && (twall & (1u << (2 * d + side))) && !(d == 1 && side == 0 && c > 0)) {
                        const AT m = AT((wmask[c] >> (2 * d + side)) & 1u);
                        AT Cw = Cface;
                        if (CST && side) {
                            if constexpr (WST) {
                                if (d == 0 && wlds)
                                    Cw = wsp[(k - z0) * kTY + CPT * ly + c];
                                else
                                    Cw = self_face_speed<AT>(fcr[d], S.sc, tk);
                            } else {
                                Cw = self_face_speed<AT>(fcr[d], S.sc, tk);
                            }
                        }
                        wall_fix(kind_of(d, side), d, side, m, Cw, fcr, ex[c], k, c, S);
                    }
                }
            }
            // z faces: lower from registers, upper from slot b
            const AT fcr[3] = {lds[a][IF + tens_row(2, 0)][sy][sxx], lds[a][IF + tens_row(2, 1)][sy][sxx],
                               lds[a][IF + tens_row(2, 2)][sy][sxx]};
            {
                const ZRow &P = prev[c];
                AT En = P.x[0];
                AT Fn[3] = {P.x[1], P.x[2], P.x[3]};
                AT fnr[3] = {P.f[0], P.f[1], P.f[2]};
                AT Cface;
                if constexpr (CST)
                    Cface = lds[a][IC + 2][sy][sxx];
                else
                    Cface = face_speed<AT>(fcr[2], P.f[2], S.sc, P.s, tk);
                S.sumC_nb += selfz_lo ? AT(0) : Cface;
                if constexpr (CALL) S.sumC_all += Cface;
                face_flux_acc<AT>(2, 0, Cface, S.Ec, S.Fc, fcr, En, Fn, fnr, S.dEs, S.dF);
                if (WL && selfz_lo && zwall_lo)   // uniform: the grid's bottom plane
                    wall_fix(kind_of(2, 0), 2, 0, AT(1), Cface, fcr, ex[c], k, c, S);
            }
            {
                AT En = lds[b][IX][sy][sxx];
                AT Fn[3] = {lds[b][IX + 1][sy][sxx], lds[b][IX + 2][sy][sxx], lds[b][IX + 3][sy][sxx]};
                AT fnr[3] = {lds[b][IF + tens_row(2, 0)][sy][sxx], lds[b][IF + tens_row(2, 1)][sy][sxx],
                             lds[b][IF + tens_row(2, 2)][sy][sxx]};
                AT Cface;
                if constexpr (CST)
                    Cface = lds[b][IC + 2][sy][sxx];
                else
                    Cface = face_speed<AT>(fcr[2], fnr[2], S.sc, lds[b][IS][sy][sxx], tk);
                S.sumC_nb += selfz_hi ? AT(0) : Cface;
                if constexpr (CALL) {
                    if (CST && selfz_hi)
                        S.sumC_all += self_speed(fcr[2]);
                    else
                        S.sumC_all += Cface;
                }
                face_flux_acc<AT>(2, 1, Cface, S.Ec, S.Fc, fcr, En, Fn, fnr, S.dEs, S.dF);
                if (WL && selfz_hi && zwall_hi) {   // uniform: the grid's top plane
                    AT Cw = Cface;
                    if constexpr (CST) Cw = self_face_speed<AT>(fcr[2], S.sc, tk);
                    wall_fix(kind_of(2, 1), 2, 1, AT(1), Cw, fcr, ex[c], k, c, S);
                }
            }
            epi(k, c, off[c], active[c], S, ex[c]);
            // this plane becomes the lower neighbour of the next one
            ZRow &P = prev[c];
            P.x[0] = S.Ec;
            for (int q = 0; q < 3; ++q) P.x[1 + q] = S.Fc[q];
            for (int q = 0; q < 3; ++q) P.f[q] = fcr[q];
            P.s = S.sc;
        }
    };

    // Pipeline (DEPTH 2): plane k is computed while planes k+2 and k+3 are in
    // flight (two register sets used alternately), so each load has two planes
    // of work to arrive before it is written to LDS; DEPTH 1 keeps plane k+2 in
    // flight only.  Every load of the steady state is unconditional (lanes
    // without a halo cell re-read their own cell, an L2 hit), so the compiler's
    // wait counts stay a full set deep.  The epilogue's per-cell extras of plane
    // k are issued ahead of the prefetch, so waiting for them leaves it in flight.
    constexpr int DEPTH = TS::DEPTH;
    const unsigned hsrc = hly >= 0 ? hoff : off[0], phsrc = hly >= 0 ? phoff : poff[0];
    using HT = std::conditional_t<SLIM, Halo, Full>;
    auto load_h = [&](int kp, HT &u) __attribute__((always_inline)) {
        if constexpr (SLIM)
            load_halo(kp, hsrc, phsrc, u);
        else
            load_full(kp, hsrc, phsrc, u);
    };
    auto put_h = [&](int sl, const HT &u) __attribute__((always_inline)) {
        if constexpr (SLIM)
            put_halo(sl, u);
        else
            put(sl, hly, hlx, u);
    };
    Full S0[CPT], S1[DEPTH == 2 ? CPT : 1];
    HT H0, H1;
    {
        Full t;
        for (int c = 0; c < CPT; ++c) {
            load_full(mapz(z0 - 1), off[c], poff[c], t);
            prev[c].x[0] = t.v[IX];
            for (int q = 0; q < 3; ++q) prev[c].x[1 + q] = t.v[IX + 1 + q];
            for (int q = 0; q < 3; ++q) prev[c].f[q] = t.v[IF + tens_row(2, q)];
            prev[c].s = t.v[IS];
        }
        for (int c = 0; c < CPT; ++c) {
            load_full(z0, off[c], poff[c], t);
            put(0, CPT * ly + c + 1, lx + 1, t);
        }
        if constexpr (SLIM) {
            Halo th;
            load_halo(z0, hsrc, phsrc, th);
            if (hly >= 0) put_halo(0, th);
        } else {
            load_full(z0, hsrc, phsrc, t);
            if (hly >= 0) put(0, hly, hlx, t);
        }
    }
    for (int c = 0; c < CPT; ++c) load_full(mapz(z0 + 1), off[c], poff[c], S0[c]);
    load_h(mapz(z0 + 1), H0);
    if constexpr (DEPTH == 2) {
        for (int c = 0; c < CPT; ++c) load_full(mapz(min(z0 + 2, z1)), off[c], poff[c], S1[c]);
        load_h(mapz(min(z0 + 2, z1)), H1);
    }

    // one plane: LOAD issues plane k+1+DEPTH (needed when k+1+DEPTH <= z1)
    auto iter = [&](auto LOAD, int t, Full (&S)[CPT], HT &H) __attribute__((always_inline)) {
        const int k = z0 + t;
        const int a = t & 1, b = a ^ 1;
        // plane k+1 (issued DEPTH planes ago) into the free slot
        for (int c = 0; c < CPT; ++c) put(b, CPT * ly + c + 1, lx + 1, S[c]);
        if (hly >= 0) put_h(b, H);
        beg(k);
        if constexpr (NE > 0)
            for (int c = 0; c < CPT; ++c) lex(k, plane * k, off[c], ex[c]);
        if constexpr (decltype(LOAD)::value) {
            const int kp = mapz(k + 1 + DEPTH);
            for (int c = 0; c < CPT; ++c) load_full(kp, off[c], poff[c], S[c]);
            load_h(kp, H);
        }
        lds_barrier();
        compute(k, a, b);
        lds_barrier();
    };
    constexpr std::true_type L1{};
    constexpr std::false_type L0{};
    const int nzr = z1 - z0;
    if constexpr (DEPTH == 2) {
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
    } else {
        for (int t = 0; t + 1 < nzr; ++t) iter(L1, t, S0, H0);
        iter(L0, nzr - 1, S0, H0);
    }
}

// y = D^-1 A (s x) (PRE: Jacobi-scaled Krylov operator, dE the E diagonal of
// the Picard iteration) or y = A x with flux rescaling xF/yF (!PRE: the
// physical operator of one Picard iteration with E diagonal dE).
// AMR: one level of the two-level composite grid -- covered coarse cells keep
// only their local terms, jump cells add their level-jump corrections (5
// planes of the apply precision: transport of E and Ft, then the change of the
// Jacobi diagonal), loaded with the epilogue's other extras ahead of the
// plane's prefetch so that waiting for them leaves the prefetch in flight.
// VEL (moving medium): the O(v/c) couplings of the energy row to Ft (vb, 3
// planes) and of the flux rows to E (vc, 3 planes); the energy row's own
// O(v/c) term is part of dE.
// LC (PRE only): read the stored face speeds Cf (false: form them per face from
// f and sR, trading 3 loads per cell for two expm1/sqrt per face; an autotuner choice).
// pg != 0 (PRE, xF yF = 1): y = pg s x - D^-1 A (s x), the second factor of the
// Neumann polynomial step (2I - B) B at no extra traffic.  The operand's scale s
// is *xs times xm.  qv (PRE, pg = 0): y = s x + qm (qs qv - D^-1 A (s x)), a damped
// Jacobi sweep on B e = qs qv.  dout (PRE): also write the Jacobi diagonal D (E
// row, then the F rows' common value; two planes).  Used by the multigrid cycle.
// MGM (multigrid, FP32 tiles, even z-ranges): 1 fuses the restriction of the
// output into mf (y is not written), 2 the injection of mf's coarse correction
// into the operand (see MgFuse).
// Waves per SIMD the single-grid FP32 sweep is built for: 4, two workgroups per CU (<= 128 VGPRs).
// The multigrid transfer and moving-medium forms spill a few registers at that size (the
// injection form 18) and are still faster than at one workgroup per CU (measured at 256^3: 290
// against 298 ms per multigrid step).  The two-level grid's sweep (two cells per thread) is left
// to the compiler.
template <class AT, bool AMR, bool VEL, int MGM>
constexpr int apply_waves()
{
    return (sizeof(AT) == 4 && !AMR) ? 4 : 1;
}

template <class AT, class ST, bool PRE, bool AMR = false, bool VEL = false, bool LC = true, int WL = 0,
          int MGM = 0>
__global__ void __launch_bounds__((tile_threads<AT, AMR>()), (apply_waves<AT, AMR, VEL, MGM>()))
    k_apply_tiled(Grid g, TileGeom tg, const ST *__restrict__ f, const AT *__restrict__ sR,
                  const ST *__restrict__ rho, const ST *__restrict__ kR, const AT *__restrict__ Cf,
                  const AT *__restrict__ dE, const AT *__restrict__ x, const double *__restrict__ xs,
                  AT *__restrict__ y, AT xF, AT yF, AmrLv al = AmrLv{}, const AT *__restrict__ vb = nullptr,
                  const AT *__restrict__ vc = nullptr, AT pg = AT(0), AT xm = AT(1), const AT *__restrict__ qv = nullptr,
                  AT qm = AT(0), AT qs = AT(1), AT *__restrict__ dout = nullptr, MgFuse<AT> mf = MgFuse<AT>{},
                  const AT *__restrict__ cw = nullptr)
{
    static_assert(MGM == 0 || (PRE && !AMR && !VEL && sizeof(AT) == 4), "multigrid fusion: FP32 Krylov apply");
    using TS = TileShape<AT, AMR>;   // the two-level grid keeps two cells per thread
    constexpr int CPT = TS::CPT;
    static_assert(CPT == 1 || CPT == 2, "a restriction y-pair is a thread's two cells or two rows");
    constexpr bool CS = PRE && LC;
    __shared__ AT lds[2][Rec<CS>::NL][TS::LY][kLX];
    const long long N = g.N;
    const AT s = ((PRE && xs) ? (AT)(*xs) : AT(1)) * xm;
    const AT nu = (AT)g.nu, half = AT(0.5) * (AT)g.nu;
    constexpr int NEX = AMR ? 6 : (VEL ? 7 : 1);
    const AT *corr = (const AT *)al.corr;
    auto lex = [&](int k, long long pb, unsigned o, AT(&e)[NEX]) __attribute__((always_inline)) {
        e[0] = ld_off(dE + pb, o);
        if constexpr (AMR) {
            const int jj = (int)(o / (unsigned)g.nx), ii = (int)(o - (unsigned)jj * (unsigned)g.nx);
            if (amr_role(al, ii, jj, k) == AMR_JUMP) {
#pragma unroll
                for (int q = 0; q < 5; ++q) e[1 + q] = corr[q * N + pb + o];
            } else {
#pragma unroll
                for (int q = 0; q < 5; ++q) e[1 + q] = AT(0);
            }
        }
        if constexpr (VEL) {
#pragma unroll
            for (int q = 0; q < 3; ++q) e[1 + q] = ld_off(vb + q * N + pb, o);
#pragma unroll
            for (int q = 0; q < 3; ++q) e[4 + q] = ld_off(vc + q * N + pb, o);
        }
    };
    // restriction: the children's D t summed over the x-pair of lanes (a shuffle), the y-pair of rows
    // and a z-pair of planes.  Two cells per thread: the thread's own y-pair, summed in registers over
    // the z-pair (the parents' diagonal loaded on the pair's first plane).  One cell per thread (each
    // row a wave): no state in registers across planes -- every plane's x-pair sums go to LDS, and at
    // the start of the next plane (after the barrier that ends every plane) or after the range, 128
    // threads add each row pair, keep the z-pair's first half in LDS and store the parents on its
    // second (6 KB of LDS: two workgroups still share a CU).
    AT racc[4] = {AT(0), AT(0), AT(0), AT(0)}, rDc[2] = {AT(1), AT(1)};
    constexpr bool RL = MGM == 1 && CPT == 1;
    constexpr int RY = TS::TYT / 2, RX = kTX / 2;
    __shared__ std::conditional_t<RL, AT[2 * RY][RX][4], AT[1][1][1]> rsh;
    __shared__ std::conditional_t<RL, AT[RY][RX][4], AT[1][1][1]> rz;
    int rbx = 0, rby = 0, rbz = 0;
    if constexpr (RL) tile_coords(tg, rbx, rby, rbz);
    // plane kd's sums (in rsh): the first plane of a z-pair is kept, the second completes the parents
    auto rfold = [&](int kd) __attribute__((always_inline)) {
        if constexpr (RL) {
            const int t = (int)threadIdx.x;
            if (t < RY * RX) {
                const int r = t / RX, xp = t % RX;
                AT v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = rsh[2 * r][xp][q] + rsh[2 * r + 1][xp][q];
                if (!(kd & 1)) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) rz[r][xp][q] = v[q];
                } else {
                    const int gx = rbx * kTX + 2 * xp, gy = rby * TS::TY + 2 * r;
                    if (gx < g.nx && gy < g.ny) {
                        const long long pc = (long long)(kd >> 1) * mf.ncx * mf.ncy + (gx >> 1) +
                                             (long long)mf.ncx * (gy >> 1);
                        mf.qc[pc] = (rz[r][xp][0] + v[0]) * (AT(0.125) / mf.Dc[pc]);
                        const AT iF = AT(0.125) / mf.Dc[mf.Nc + pc];
                        for (int q = 1; q < 4; ++q) mf.qc[q * mf.Nc + pc] = (rz[r][xp][q] + v[q]) * iF;
                    }
                }
            }
        }
    };
    auto epi = [&](int k, int c, unsigned o, bool active, const CellSums<AT> &S, const AT(&e)[NEX])
                   __attribute__((always_inline)) {
        const long long pb = (long long)g.nx * g.ny * k;
        const AT dEc = e[0];
        AT yE = dEc * S.Ec + nu * S.dEs, yFq[3];
        for (int q = 0; q < 3; ++q) yFq[q] = (AT(1) + S.sc) * S.Fc[q] + nu * S.dF[q];
        AT dtr = half * S.sumC_nb;   // transport part of the Jacobi diagonal
        if constexpr (VEL) {
            for (int q = 0; q < 3; ++q) {
                yE += e[1 + q] * S.Fc[q];
                yFq[q] += e[4 + q] * S.Ec;
            }
        }
        if constexpr (AMR) {
            const int jj = (int)(o / (unsigned)g.nx), ii = (int)(o - (unsigned)jj * (unsigned)g.nx);
            const int role = amr_role(al, ii, jj, k);
            if (role == AMR_COVERED) {
                yE = dEc * S.Ec;
                for (int q = 0; q < 3; ++q) yFq[q] = (AT(1) + S.sc) * S.Fc[q];
                dtr = AT(0);
            } else {   // zero except at jump cells
                yE += e[1];
                for (int q = 0; q < 3; ++q) yFq[q] += e[2 + q];
                dtr += e[5];
            }
        }
        if constexpr (PRE) {
            AT DE = dEc + dtr, DF[3];
            DF[0] = DF[1] = DF[2] = AT(1) + S.sc + dtr;
            if constexpr (WL) {   // the walls' shares, per row
                DE += nu * S.wE;
                for (int q = 0; q < 3; ++q) DF[q] += nu * S.wF[q];
            }
            yE *= AT(1) / DE;
            if constexpr (WL) {
                for (int q = 0; q < 3; ++q) yFq[q] *= AT(1) / DF[q];
            } else {
                const AT iDF = AT(1) / DF[0];
                for (int q = 0; q < 3; ++q) yFq[q] *= iDF;
            }
            if (dout && active) {   // the Jacobi diagonal itself (E row, the F rows' mean)
                st_off(dout + pb, o, DE);
                st_off(dout + N + pb, o, (DF[0] + DF[1] + DF[2]) * AT(1.0 / 3.0));
            }
        }
        if (pg != AT(0)) {   // polynomial step: pg s x - B (s x), the centre of s x already in the sums
            yE = pg * S.Ec - yE;
            for (int q = 0; q < 3; ++q) yFq[q] = pg * S.Fc[q] - yFq[q];
        } else if (qv) {     // damped Jacobi sweep on B e = qs qv from e = s x
            yE = S.Ec + qm * (qs * ld_off(qv + pb, o) - yE);
            for (int q = 0; q < 3; ++q) yFq[q] = S.Fc[q] + qm * (qs * ld_off(qv + (1 + q) * N + pb, o) - yFq[q]);
        }
        if constexpr (MGM == 1) {
            // the diagonal of the restriction: E row, the F rows' mean (as dout holds it)
            AT DEr = dEc + dtr, DFr = AT(1) + S.sc + dtr;
            if constexpr (WL) {
                DEr += nu * S.wE;
                DFr += nu * (S.wF[0] + S.wF[1] + S.wF[2]) * AT(1.0 / 3.0);
            }
            if constexpr (RL) {   // this plane's x-pair sums into LDS, one row of the tile per wave
                AT v[4] = {DEr * yE, DFr * yFq[0], DFr * yFq[1], DFr * yFq[2]};
                for (int q = 0; q < 4; ++q) v[q] += __shfl_xor(v[q], 1);
                const int lx = (int)(threadIdx.x % kTX), ly = (int)(threadIdx.x / kTX);
                if (!(lx & 1))
                    for (int q = 0; q < 4; ++q) rsh[ly][lx >> 1][q] = v[q];
            } else {
                racc[0] += DEr * yE;
                for (int q = 0; q < 3; ++q) racc[1 + q] += DFr * yFq[q];
            }
            if (!RL && c == 1) {   // two cells per thread: the thread's y-pair is in
                const unsigned gxo = o % (unsigned)g.nx, gyo = o / (unsigned)g.nx;
                const long long pc = (long long)(k >> 1) * mf.ncx * mf.ncy + (gxo >> 1) + (long long)mf.ncx * (gyo >> 1);
                if (!(k & 1)) {   // first plane of the z-pair: the parents' diagonal
                    rDc[0] = mf.Dc[pc];
                    rDc[1] = mf.Dc[mf.Nc + pc];
                } else {          // the z-pair is in: add the x-pair's, store, start over
                    for (int q = 0; q < 4; ++q) racc[q] += __shfl_xor(racc[q], 1);
                    if (active && !(gxo & 1)) {
                        mf.qc[pc] = racc[0] * (AT(0.125) / rDc[0]);
                        const AT iF = AT(0.125) / rDc[1];
                        for (int q = 1; q < 4; ++q) mf.qc[q * mf.Nc + pc] = racc[q] * iF;
                    }
                    for (int q = 0; q < 4; ++q) racc[q] = AT(0);
                }
            }
        } else if (active) {
            st_off(y + pb, o, yE);
            for (int q = 0; q < 3; ++q) st_off(y + (1 + q) * N + pb, o, yFq[q] * yF);
        }
    };
    // the linear operator's ghost faces: ghosts without their data
    auto wall = [&](int kind, int d, int side, AT Ec, const AT(&Fc)[3], const AT(&fcr)[3], const AT(&)[NEX], unsigned,
                    AT &En, AT(&Fn)[3], AT(&fnr)[3]) __attribute__((always_inline)) {
        const AT z3[3] = {AT(0), AT(0), AT(0)};
        wall_ghost<AT>(kind, d, side, Ec, Fc, fcr, AT(0), z3, AT(0), En, Fn, fnr);
    };
    // the previous plane's restriction sums: at the start of each plane but the range's first, and
    // after the range (the sweep ends with a barrier)
    auto beg = [&](int k) __attribute__((always_inline)) {
        if constexpr (RL)
            if (k > rbz * tg.kz) rfold(k - 1);
    };
    tile_sweep<AT, ST, PRE, false, NEX, CS, WL, MGM == 2, AMR>(g, tg, f, sR, rho, kR, Cf, x, s, s * xF, lds, lex,
                                                              epi, wall, mf, cw, beg);
    if constexpr (RL) rfold(min(rbz * tg.kz + tg.kz, g.nz) - 1);
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

// The own corrected speed (divided by c) of every cell on a high Dirichlet, open, Marshak or
// reflecting face, once per step, in FP64 from the stored coefficients, rounded to the apply precision:
// x walls [nz][ny], then y walls [nz][nx], then z walls [ny][nx] (other faces' entries unused).
// SR: sR is given (coarse levels), else formed from rho and kR.
template <class CT, class AT, bool SR = false>
__global__ void __launch_bounds__(256) k_wall_speed(Grid g, const CT *__restrict__ rho, const CT *__restrict__ kR,
                                                    const AT *__restrict__ sR, const CT *__restrict__ f,
                                                    AT *__restrict__ cw)
{
    const long long ax = (long long)g.ny * g.nz, ay = (long long)g.nx * g.nz, az = (long long)g.nx * g.ny;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= ax + ay + az) return;
    int d, i, j, k;
    if (t < ax) {
        d = 0, i = g.nx - 1, j = (int)(t % g.ny), k = (int)(t / g.ny);
    } else if (t < ax + ay) {
        d = 1, i = (int)((t - ax) % g.nx), j = g.ny - 1, k = (int)((t - ax) / g.nx);
    } else {
        d = 2, i = (int)((t - ax - ay) % g.nx), j = (int)((t - ax - ay) / g.nx), k = g.nz - 1;
    }
    if (!ghost_face(wall_kind(g, d, 1))) return;
    const long long c = i + (long long)g.nx * (j + (long long)g.ny * k);
    const double s = SR ? (double)sR[c] : g.cdt * (double)rho[c] * (double)kR[c];
    const double fdd = (double)f[d * g.N + c];
    cw[t] = (AT)face_speed<double>(fdd, fdd, s, s, g.tau_k);
}

}  // namespace vr
