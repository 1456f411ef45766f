// janc_kernels.h -- gfx950 kernels of the JANC per-time-step update (templates over the
// model and the field count; instantiated by janc_kernels.hip and, for the detailed model,
// one species count per translation unit, by janc_species.hip).
//
// One RK stage is one launch over a list of tiles (a tile is up to 16x16,
// 32x8 or 64x4 cells of one block, or 256 cells of a one-dimensional block),
// one 256-thread workgroup per tile. Per tile:
//   phase 0  every cell of the tile plus 3 halo layers (cross-shaped; corners
//            are not needed by the dimension-by-dimension sweeps) is fetched
//            from its source -- the same block, a neighbouring block, the
//            coarser level for coarse-fine ring cells, or a boundary rule --
//            and its primitives are kept in registers;
//   phase 1  per conserved component: Lax-Friedrichs split fluxes F+/F- and
//            G+/G- (Eq. 4.11) go to LDS, WENO5 interface fluxes (Sec. 4.2)
//            are reconstructed from LDS, and each owned cell forms the
//            conservative difference (Eq. 4.10) and its Shu-Osher RK stage;
//   phase 2  T of the new state (Newton warm-started from the previous stage
//            for the NASA-7 model, Sec. 4.2), status checks, and the maxima of
//            |u|+c, |v|+c and the CFL bound for the next stage, reduced per
//            wavefront and published with one 64-bit atomic max per workgroup.
// Nothing here is a dense contraction, so there is no MFMA: the work is FP64
// VALU arithmetic on values staged through LDS.
#pragma once

#include "janc_device.h"

namespace janc {

// ------------------------------------------------------------------ the stage tile
// Conserved components reconstructed per pass between one pair of barriers: their
// split fluxes go to separate LDS sets, so each thread has STAGE_CPB independent
// WENO5 chains between the barriers and a stage has 2 ceil(NU / STAGE_CPB) barriers.
#ifndef STAGE_CPB
#define STAGE_CPB 2
#endif
// Points of a tile: the TX x TY owned positions first (point tid is thread tid's
// own cell), then the x halo (3 columns each side of every row) and, for 2-D
// tiles, the y halo (3 rows below and above every column).
template <int TX, int TY>
struct Geom {
    static constexpr bool TWO = TY > 1;
    static constexpr int NC = TX * TY;
    static constexpr int NHX = 6 * TY, NHY = TWO ? 6 * TX : 0;
    static constexpr int NP = NC + NHX + NHY, NPT = (NP + WG - 1) / WG;
    static constexpr int PW = TX + 6;
    static constexpr int NXS = PW * TY;                 // x split fluxes, row-major, 3 halo columns
    static constexpr int NYS = TWO ? TX * (TY + 6) : 0; // y split fluxes, 3 halo rows
    static constexpr int NIX = (TX + 1) * TY;           // x interfaces
    static constexpr int NIY = TWO ? TX * (TY + 1) : 0; // y interfaces
    static constexpr int NEXT = TY + (TWO ? TX : 0);  // right column / top row interfaces
    // LDS doubles of one set: F+/F- and G+/G-, then the numerical fluxes (sum of the
    // two one-sided reconstructions) at the x and y interfaces; one set per component
    // of a pass, then scratch
    static constexpr int SET = 2 * NXS + 2 * NYS + NIX + NIY;
    static constexpr int NSET = STAGE_CPB;
    static constexpr int LDS = NSET * SET + 16;
    static constexpr int oFPX = 0, oFMX = NXS, oFPY = 2 * NXS, oFMY = 2 * NXS + NYS;
    static constexpr int oHX = 2 * NXS + 2 * NYS, oHY = oHX + NIX;

    // tile-local position (li, lj) of point p
    __device__ static void point(int p, int& li, int& lj) {
        if (p < NC) {
            lj = p / TX;
            li = p - lj * TX;
        } else if (p < NC + NHX) {
            const int h = p - NC, side = h / (3 * TY), r = h - side * 3 * TY;
            lj = r / 3;
            li = side ? TX + (r - lj * 3) : (r - lj * 3) - 3;
        } else {
            const int h = p - NC - NHX, side = h / (3 * TX), r = h - side * 3 * TX;
            const int row = r / TX;
            li = r - row * TX;
            lj = side ? TY + row : row - 3;
        }
    }
};

// Point p of a tile of tw x th valid cells: its tile-local position and whether the x
// and the y sweep read it (the halo is cross-shaped).
template <int TX, int TY>
__device__ __forceinline__ void point_needs(int p, int tw, int th, int& li, int& lj, bool& nx,
                                            bool& ny) {
    Geom<TX, TY>::point(p, li, lj);
    nx = (lj >= 0 && lj < th) && (li >= -3 && li < tw + 3);
    ny = Geom<TX, TY>::TWO && (li >= 0 && li < tw) && (lj >= -3 && lj < th + 3);
}

// Block-local cell (bi, bj) is its own source: inside the block and not a ring cell.
__device__ __forceinline__ bool own_source(const DevBlock& B, int bi, int bj) {
    return bi >= 0 && bi < B.nx && bj >= 0 && bj < B.ny && !ring_at(B, bi, bj);
}

template <int M, int NU, int TX, int TY>
__device__ void stage_tile(const StageArgs& a, const int ti, const Tile tile, double* smem) {
    using G = Geom<TX, TY>;
    static_assert(TX * TY == WG, "one owned cell per thread");
    // set k at smem + k * SET: F+ / F- of x (fpx, fmx) and y (fpy, fmy), the WENO5 of
    // F+ and F- at x interfaces (hxp, hxm) and y interfaces (hyp, hym)
    double* scratch = smem + G::NSET * G::SET;

    const int tid = threadIdx.x;
    const DevBlock B = a.blk[tile.block];
    CDom& D = cdom(a.dom, B.domain);
    const int lev = B.level;
    const int stage = a.stage;
    const int bin = (stage == 1 && a.strang) ? 3 : stage - 1, bout = stage % 3;
    // crossover advance: dt_l = dt_0 / 2^l, dt_0 formed by the first launch of the step
    const double dt = a.cross ? ldexp((a.xfirst && stage == 1) ? step_dt(a, B.domain, 0)
                                                               : a.dt[B.domain], -lev)
                              : (stage == 1) ? step_dt(a, B.domain, 0) : a.dt[B.domain];
    if (!(dt > 0.0)) return;   // finished domain: state unchanged
    const double dxl = D.dx0 / (double)(1 << lev), dyl = D.dy0 / (double)(1 << lev);
    const double idx = 1.0 / dxl, idy = 1.0 / dyl;
    const int slot = D.slot0 + lev;
    const double ax = slot_get(a.red, bin, 2 * slot);
    const double ay = slot_get(a.red, bin, 2 * slot + 1);
    const int tw = min(TX, B.nx - tile.x0), th = min(TY, B.ny - tile.y0);

    // ---------------- phase 0: fetch the tile and its halo, primitives in registers
    double ur[G::NPT][NU];
    double vxr[G::NPT], vyr[G::NPT], pr[G::NPT];
    bool needx[G::NPT], needy[G::NPT];
    int xoff[G::NPT], yoff[G::NPT];
    double Town = 0.0;
#pragma unroll
    for (int q = 0; q < G::NPT; ++q) {
        const int p = tid + q * WG;
        needx[q] = needy[q] = false;
        xoff[q] = yoff[q] = 0;
        vxr[q] = vyr[q] = pr[q] = 0.0;
#pragma unroll
        for (int f = 0; f < NU; ++f) ur[q][f] = 0.0;
        // the table word is loaded for every point (one coalesced row per tile) ahead of
        // the test that decides whether it is used
        const int hv = (a.hsrc && p < G::NP) ? a.hsrc[(size_t)ti * a.hstride + p] : 0;
        if (p < G::NP) {
            int li, lj;
            point_needs<TX, TY>(p, tw, th, li, lj, needx[q], needy[q]);
            xoff[q] = lj * G::PW + li + 3;
            yoff[q] = (lj + 3) * TX + li;
            if (needx[q] || needy[q]) {
                const int bi = tile.x0 + li, bj = tile.y0 + lj;
                long long src;
                unsigned fl = 0u;
                if (own_source(B, bi, bj)) {
                    src = B.offset + (long long)bj * B.nx + bi;
                } else if (a.hsrc) {
                    src = (long long)(hv >> 3);
                    fl = (unsigned)(hv & 7);
                } else {
                    src = resolve(a, D, lev, B.i0 + bi, B.j0 + bj, fl);
                }
                double T;
                // crossover: coarser levels are read at their current state
                const bool base = a.cross && (fl & 4u);
                fetch<NU>(a, src, fl, base ? a.U0 : a.Uin, base ? a.Tbase : a.Tin, ur[q], T);
                halo_prims<M, NU>(ur[q], T, D, cmech(a.mech), vxr[q], vyr[q], pr[q]);
                if (q == 0) Town = T;
            }
        }
    }

    // owned cell: point tid, held in ur[0]
    const int oli = tid % TX, olj = tid / TX;
    const int obi = tile.x0 + oli, obj = tile.y0 + olj;
    const bool own = (oli < tw) && (olj < th) && !ring_at(B, obi, obj);
    const long long oc = B.offset + (long long)obj * B.nx + obi;
    double src_e = 0.0;   // explicit source of the one-step model (Sec. 4.3)
    if constexpr (M == ONESTEP) {
        if (own) {
            const double Tc = pr[0] / (ur[0][0] * D.R);
            src_e = -D.k * ur[0][4] * exp(-D.Ea / Tc);
        }
    }
    double unew[NU];

    // reconstruction tasks of this thread (see phase 1)
    const bool vxi = (olj < th) && (oli <= tw);
    const bool vyi = G::TWO && (oli < tw) && (olj <= th);
    const int bxi = olj * G::PW + oli, byi = olj * TX + oli;
    const int rxi = olj * (TX + 1) + oli, ryi = olj * TX + oli;
    bool ext_ok = false;
    int ext_str = 1, ext_p = 0, ext_m = 0, ext_out = 0;   // offsets within a set
    if (tid < G::NEXT) {
        const int e = tid;
        if (e < TY) {              // x interface TX of row e
            ext_ok = e < th && tw == TX;
            const int o = e * G::PW + TX;
            ext_p = G::oFPX + o;
            ext_m = G::oFMX + o;
            ext_str = 1;
            ext_out = G::oHX + e * (TX + 1) + TX;
        } else {                   // y interface TY of column e - TY
            const int col = e - TY;
            ext_ok = col < tw && th == TY;
            const int o = TY * TX + col;
            ext_p = G::oFPY + o;
            ext_m = G::oFMY + o;
            ext_str = TX;
            ext_out = G::oHY + TY * TX + col;
        }
    }

    // ---------------- phase 1: per component split fluxes, WENO5, RK update
    // U^(0) of the owned cell (stages 2 and 3) is loaded PF components ahead of
    // its use, so that its memory latency overlaps the reconstructions between.
    constexpr int PF = 3;
    const bool ld0 = own && stage != 1;
    double u0q[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) u0q[k] = (ld0 && k < NU) ? a.U0[(size_t)k * a.pool + oc] : 0.0;
    // split fluxes of component f (Eq. 4.11) into set S
    auto flux = [&](int f, double* S) {
#pragma unroll
        for (int q = 0; q < G::NPT; ++q) {
            const double uf = ur[q][f];
            if (needx[q]) {
                double F = uf * vxr[q];
                if (f == 1) F += pr[q];
                if (f == 3) F = (uf + pr[q]) * vxr[q];
                S[G::oFPX + xoff[q]] = 0.5 * (F + ax * uf);
                S[G::oFMX + xoff[q]] = 0.5 * (F - ax * uf);
            }
            if constexpr (G::TWO) {
                if (needy[q]) {
                    double Gf = uf * vyr[q];
                    if (f == 2) Gf += pr[q];
                    if (f == 3) Gf = (uf + pr[q]) * vyr[q];
                    S[G::oFPY + yoff[q]] = 0.5 * (Gf + ay * uf);
                    S[G::oFMY + yoff[q]] = 0.5 * (Gf - ay * uf);
                }
            }
        }
    };
    // WENO5 reconstructions from set S into set S: each thread takes the left x
    // interface and the lower y interface of its own position (both one-sided values,
    // summed: the numerical flux), at fixed LDS offsets; the right column and top row
    // of interfaces are the extra tasks of the first threads. F- reads its stencil
    // mirrored.
    auto recon = [&](double* S) {
        if (vxi) {
            const double* P = S + G::oFPX + bxi;
            const double* Mn = S + G::oFMX + bxi;
            S[G::oHX + rxi] = weno5(P[0], P[1], P[2], P[3], P[4]) +
                              weno5(Mn[5], Mn[4], Mn[3], Mn[2], Mn[1]);
        }
        if constexpr (G::TWO) {
            if (vyi) {
                const double* P = S + G::oFPY + byi;
                const double* Mn = S + G::oFMY + byi;
                S[G::oHY + ryi] = weno5(P[0], P[TX], P[2 * TX], P[3 * TX], P[4 * TX]) +
                                  weno5(Mn[5 * TX], Mn[4 * TX], Mn[3 * TX], Mn[2 * TX], Mn[TX]);
            }
        }
        if (ext_ok) {
            const double* P = S + ext_p;
            const double* Mn = S + ext_m;
            const int k = ext_str;
            S[ext_out] = weno5(P[0], P[k], P[2 * k], P[3 * k], P[4 * k]) +
                         weno5(Mn[5 * k], Mn[4 * k], Mn[3 * k], Mn[2 * k], Mn[k]);
        }
    };
    // flux difference (Eq. 4.10), source and RK stage of component f from set S
    auto update = [&](int f, const double* S, double u0) {
        if (own) {
            const double* hx = S + G::oHX;
            const int rx = olj * (TX + 1) + oli;
            double L = -(hx[rx + 1] - hx[rx]) * idx;
            if constexpr (G::TWO) {
                const double* hy = S + G::oHY;
                const int ry = olj * TX + oli;
                L -= (hy[ry + TX] - hy[ry]) * idy;
            }
            if constexpr (M == ONESTEP) {
                if (f == 4) L += src_e;
            }
            const double un = rk_combine(stage, u0, ur[0][f], L, dt);
            a.Uout[(size_t)f * a.pool + oc] = un;
            unew[f] = un;
        }
    };
    constexpr int CPB = G::NSET;
#pragma unroll
    for (int f0 = 0; f0 < NU; f0 += CPB) {
#pragma unroll
        for (int k = 0; k < CPB; ++k)
            if (f0 + k < NU) flux(f0 + k, smem + k * G::SET);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CPB; ++k)
            if (f0 + k < NU) recon(smem + k * G::SET);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < CPB; ++k) {
            const int f = f0 + k;
            if (f < NU) {
                const double u0 = (stage == 1) ? ur[0][f] : u0q[f % PF];
                if (f + PF < NU) u0q[f % PF] = ld0 ? a.U0[(size_t)(f + PF) * a.pool + oc] : 0.0;
                update(f, smem + k * G::SET, u0);
            }
        }
    }

    // ---------------- phase 2: T, checks, maxima for the next stage
    double sx = 0.0, sy = 0.0, sc = 0.0;
    if (own) {
        double T, c, vx, vy;
        const unsigned st = owner_state<M, NU>(unew, Town, D, cmech(a.mech), T, c, vx, vy);
        a.Tout[oc] = T;
        if (st) atomicOr(a.status, st);
        const bool skip = (stage == 3) && B.fine_child && (!a.cross || a.xskip_cov) &&
                          covered_by_finer(a, D, lev, B.i0 + obi, B.j0 + obj);
        if (a.reduce_out && !st && !skip) {
            sx = fabs(vx) + c;
            sy = fabs(vy) + c;
            sc = cfl_bound(a, D, lev, sx, sy, idx, idy);
        }
    }
    if (a.reduce_out)
        publish_max3(a.red, bout, 2 * slot, 2 * slot + 1, 2 * a.red.nunits + B.domain, sx, sy, sc,
                     scratch);
}

#ifndef STAGE_WAVES
#define STAGE_WAVES 1
#endif
template <int M, int NU, int TX, int TY, bool HAS1D, bool HAS2D>
__global__ __launch_bounds__(WG, STAGE_WAVES) void stage_kernel(StageArgs a, int first_tile, int owner_launch) {
    constexpr int L2 = Geom<TX, TY>::LDS, L1 = Geom<WG, 1>::LDS;
    __shared__ double smem[(L2 > L1) ? L2 : L1];
    if (blockIdx.x == 0) stage_bookkeeping(a, owner_launch);
    const int ti = first_tile + (a.linear_sched ? (int)blockIdx.x : xcd_chunk(blockIdx.x, gridDim.x));
    const Tile tile = a.tiles[ti];
    if (HAS1D && tile.kind == 1) {
        if constexpr (HAS1D) stage_tile<M, NU, WG, 1>(a, ti, tile, smem);
    } else {
        if constexpr (HAS2D) stage_tile<M, NU, TX, TY>(a, ti, tile, smem);
    }
    if (a.stage == 3 && (a.cross ? a.xlast : owner_launch) && blockIdx.x == 0) {
        // t and the step counter are read by the next step's first stage only
        if (M != DETAILED) step_finish(a);
    }
}

// ------------------------------------------------------------------ halo source table
// Workgroup t fills row t of the table: for each point of tile t that a sweep reads and
// that is not its own block's cell, 8 * resolve() + its flags (bit 0 / 1: mirrored x / y
// momentum, bit 2: a coarser level); 0 elsewhere (never read).
template <int TX, int TY>
__device__ void halo_table_tile(const StageArgs& a, int ti, const Tile& tile, int* row) {
    using G = Geom<TX, TY>;
    const DevBlock B = a.blk[tile.block];
    CDom& D = cdom(a.dom, B.domain);
    const int tw = min(TX, B.nx - tile.x0), th = min(TY, B.ny - tile.y0);
    for (int p = threadIdx.x; p < G::NP; p += WG) {
        int li, lj;
        bool nx, ny;
        point_needs<TX, TY>(p, tw, th, li, lj, nx, ny);
        int v = 0;
        const int bi = tile.x0 + li, bj = tile.y0 + lj;
        if ((nx || ny) && !own_source(B, bi, bj)) {
            unsigned fl = 0u;
            const long long src = resolve(a, D, B.level, B.i0 + bi, B.j0 + bj, fl);
            v = (int)(src * 8 + (long long)fl);
        }
        row[p] = v;
    }
}

template <int TX, int TY>
__global__ __launch_bounds__(WG) void halo_table_kernel(StageArgs a, int* out, int stride) {
    const int ti = blockIdx.x;
    const Tile tile = a.tiles[ti];
    int* row = out + (size_t)ti * stride;
    if (tile.kind == 1) halo_table_tile<WG, 1>(a, ti, tile, row);
    else halo_table_tile<TX, TY>(a, ti, tile, row);
}

// ------------------------------------------------------------------ per-cell kernels
// Cell of a tile owned by this thread (same mapping as the stage kernel).
struct CellRef {
    long long c;
    int I, J;     // level coordinates
    bool own;
};

__device__ __forceinline__ CellRef tile_cell(const StageArgs& a, const Tile& tile, const DevBlock& B) {
    (void)a;
    CellRef r;
    int tw, th, li, lj;
    if (tile.kind == 1) {
        li = threadIdx.x;
        lj = 0;
        tw = min(WG, B.nx - tile.x0);
        th = 1;
    } else {
        // 2-D tile shapes encode their width in kind >> 8
        const int TXs = tile.kind >> 8;
        li = threadIdx.x % TXs;
        lj = threadIdx.x / TXs;
        tw = min(TXs, B.nx - tile.x0);
        th = min(WG / TXs, B.ny - tile.y0);
    }
    const int bi = tile.x0 + li, bj = tile.y0 + lj;
    r.own = (li < tw) && (lj < th) && !ring_at(B, bi, bj);
    r.c = B.offset + (long long)bj * B.nx + bi;
    r.I = B.i0 + bi;
    r.J = B.j0 + bj;
    return r;
}

// Call entry: T re-solved from U (warm start = stored T) and the maxima for stage 1.
template <int M, int NU>
__global__ __launch_bounds__(WG) void init_kernel(StageArgs a) {
    __shared__ double scratch[16];
    const Tile tile = a.tiles[blockIdx.x];
    const DevBlock B = a.blk[tile.block];
    CDom& D = cdom(a.dom, B.domain);
    const CellRef r = tile_cell(a, tile, B);
    const int lev = B.level, slot = D.slot0 + lev;
    const double idx = (double)(1 << lev) / D.dx0, idy = (double)(1 << lev) / D.dy0;
    double sx = 0.0, sy = 0.0, sc = 0.0;
    if (r.own) {
        double u[NU];
#pragma unroll
        for (int f = 0; f < NU; ++f) u[f] = a.Uin[(size_t)f * a.pool + r.c];
        double T, c, vx, vy;
        const unsigned st = owner_state<M, NU>(u, a.Tin[r.c], D, cmech(a.mech), T, c, vx, vy);
        a.Tout[r.c] = T;
        if (st) atomicOr(a.status, st);
        else {
            sx = fabs(vx) + c;
            sy = fabs(vy) + c;
            sc = cfl_bound(a, D, lev, sx, sy, idx, idy);
        }
    }
    publish_max3(a.red, 0, 2 * slot, 2 * slot + 1, 2 * a.red.nunits + B.domain, sx, sy, sc, scratch);
}

// (I - dt J) dU = dt w of the point-implicit step (Eq. 4.12-4.13) for the Jacobian J of
// rho Y_1 .. rho Y_{Ns-1} and the production rates w: Gaussian elimination with partial
// pivoting in registers; w returns the increment.
template <int NS>
__device__ __forceinline__ void chem_solve(double (&J)[NS - 1][NS - 1], double (&w)[NS - 1],
                                           double dt, unsigned& st) {
    constexpr int NT = NS - 1;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
#pragma unroll
        for (int q = 0; q < NT; ++q) J[k][q] = (k == q ? 1.0 : 0.0) - dt * J[k][q];
        w[k] = w[k] * dt;
    }
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        // pivot row: the first row at or below c with the largest |entry| in column c;
        // rows are exchanged by selects so that the matrix stays in registers, and only
        // in wavefronts where some cell needs an exchange
        int p = c;
        double amax = fabs(J[c][c]);
#pragma unroll
        for (int r = c + 1; r < NT; ++r) {
            const double ar = fabs(J[r][c]);
            if (ar > amax) { amax = ar; p = r; }
        }
        if (__any(p != c)) {
#pragma unroll
            for (int r = c + 1; r < NT; ++r) {
                const bool sw = (r == p);
#pragma unroll
                for (int q = c; q < NT; ++q) {
                    const double top = J[c][q], row = J[r][q];
                    J[c][q] = sw ? row : top;
                    J[r][q] = sw ? top : row;
                }
                const double wt = w[c], wr = w[r];
                w[c] = sw ? wr : wt;
                w[r] = sw ? wt : wr;
            }
        }
        const double piv = J[c][c];
        if (!(fabs(piv) > 0.0) || !isfinite(piv)) st |= STB_NONFINITE;
        const double ip = 1.0 / piv;
#pragma unroll
        for (int r = c + 1; r < NT; ++r) {
            const double fct = J[r][c] * ip;
#pragma unroll
            for (int q = c + 1; q < NT; ++q) J[r][q] -= fct * J[c][q];
            w[r] -= fct * w[c];
        }
    }
#pragma unroll
    for (int r = NT - 1; r >= 0; --r) {
        double sacc = w[r];
#pragma unroll
        for (int q = r + 1; q < NT; ++q) sacc -= J[r][q] * w[q];
        w[r] = sacc / J[r][r];
    }
}


// Point-implicit chemistry (Eq. 4.12-4.13) on rho Y_1 .. rho Y_{Ns-1} of each
// solved cell, then Newton for the new T and the maxima for the next step.
// Mechanism tables are read as wave-uniform scalar loads. Per-thread columns in
// LDS hold X, the species Gibbs terms and the derivative row dq/dX of the
// current reaction (indexed by wave-uniform species numbers); the (Ns-1)^2
// Jacobian, the production rates and the LU factorization live in registers.
template <int NS, bool FULLJ>
__device__ __forceinline__ void chem_cell(CMech* m, double* Xs, double* gts, double* dqs,
                                          double rho, double T, const double (&rY)[NS - 1],
                                          double dt, double (&w)[NS - 1], unsigned& st) {
    constexpr int NT = NS - 1;
    const int tid = threadIdx.x;
    // LDS column per thread: X[0..NS-1], X[NS] = 1 (padding of the molecule lists)
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        Xs[j * WG + tid] = rY[j] * m->invM[j];
        s += rY[j];
    }
    Xs[NT * WG + tid] = (rho - s) * m->invM[NT];
    Xs[NS * WG + tid] = 1.0;
    const double lnT = log(T), invT = 1.0 / T;
    const double lnC = log(PATM / RU) - lnT;      // ln(p_atm / (R_u T))
#pragma unroll
    for (int j = 0; j < NS; ++j) {                 // h/(R T) - s/R per species
        const bool hi = m->two_range && T >= m->tmid[j];
        double a[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) a[q] = hi ? m->nasa_hi[j][q] : m->nasa[j][q];
        gts[j * WG + tid] = a[0] * (1.0 - lnT) -
                T * (0.5 * a[1] + T * (a[2] * (1.0 / 6.0) + T * (a[3] * (1.0 / 12.0) + T * (a[4] * 0.05)))) +
                a[5] * invT - a[6];
    }
    gts[NS * WG + tid] = 0.0;   // padding slot of the molecule lists
    // species + T Jacobian: T follows the composition at fixed rho and e, so
    // J += (dS/dT) (dT/d rho Y)^T with dT/d rho Y_m = -(e_m - e_last) / (rho c_v);
    // hm1[j] = h_j/(R_u T) - 1 = e_j / (R_u T) per mole, cvs = rho c_v / R_u
    double hm1[NS], dSdT[NT];
    double cvs = 0.0;
    if constexpr (FULLJ) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const bool hi = m->two_range && T >= m->tmid[j];
            double a[7];
#pragma unroll
            for (int q = 0; q < 7; ++q) a[q] = hi ? m->nasa_hi[j][q] : m->nasa[j][q];
            hm1[j] = a[0] + T * (0.5 * a[1] + T * (a[2] * (1.0 / 3.0) + T * (0.25 * a[3] + T * (0.2 * a[4])))) +
                     a[5] * invT - 1.0;
            cvs += Xs[j * WG + tid] * (a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4]))) - 1.0);
        }
#pragma unroll
        for (int k = 0; k < NT; ++k) dSdT[k] = 0.0;
    }
    double J[NT][NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        w[k] = 0.0;
#pragma unroll
        for (int q = 0; q < NT; ++q) J[k][q] = 0.0;
    }
    const int nr = m->nr;
    for (int i = 0; i < nr; ++i) {
        const double lnkf = m->lnA[i] + m->b[i] * lnT - m->EaR[i] * invT;
        const double kf = exp(lnkf);
        const int f0 = m->lf[i][0], f1 = m->lf[i][1], f2 = m->lf[i][2];
        const int r0 = m->lb[i][0], r1 = m->lb[i][1], r2 = m->lb[i][2];
        double kb = 0.0;
        if (m->rev[i]) {
            // sum_j dnu_j g_j, g = h/(RT) - s/R: products minus reactants, one entry per
            // molecule (the padding slot holds 0)
            const double sg = (gts[r0 * WG + tid] + gts[r1 * WG + tid] + gts[r2 * WG + tid]) -
                              (gts[f0 * WG + tid] + gts[f1 * WG + tid] + gts[f2 * WG + tid]);
            // K_eq = exp(-sum dnu g) (p_atm/(R_u T))^(sum dnu), Eq. 4.9
            kb = exp(lnkf + sg - (double)m->dnsum[i] * lnC);
        }
        const double xf0 = Xs[f0 * WG + tid], xf1 = Xs[f1 * WG + tid], xf2 = Xs[f2 * WG + tid];
        const double xb0 = Xs[r0 * WG + tid], xb1 = Xs[r1 * WG + tid], xb2 = Xs[r2 * WG + tid];
        const double Rf = kf * (xf0 * xf1 * xf2), Rb = kb * (xb0 * xb1 * xb2);
        const bool tbr = m->has_tb[i] != 0;
        double ctb = 1.0;
        if (tbr) {
            ctb = 0.0;
#pragma unroll
            for (int j = 0; j < NS; ++j) ctb += m->tb[i][j] * Xs[j * WG + tid];
        }
        const double net = Rf - Rb;
        const double q = ctb * net;
#pragma unroll
        for (int k = 0; k < NT; ++k) w[k] += m->Mdnu[i][k] * q;
        if constexpr (FULLJ) {
            // d ln kf/dT = (b + Ea/(R T))/T; d ln kb/dT = d ln kf/dT - sum_j dnu_j (H_j - 1)/T
            const double dlf = (m->b[i] + m->EaR[i] * invT) * invT;
            double dlb = dlf;
            if (m->rev[i]) {
                double sh = 0.0;
#pragma unroll
                for (int j = 0; j < NS; ++j) sh += (double)m->dnu[i][j] * hm1[j];
                dlb = dlf - sh * invT;
            }
            const double dqT = ctb * (Rf * dlf - Rb * dlb);
#pragma unroll
            for (int k = 0; k < NT; ++k) dSdT[k] += m->Mdnu[i][k] * dqT;
        }
        // dq/dX_j into LDS (padding slot NS absorbs the entries of missing molecules)
#pragma unroll
        for (int j = 0; j <= NS; ++j) dqs[j * WG + tid] = (tbr && j < NS) ? m->tb[i][j] * net : 0.0;
        const double cf = ctb * kf, cb = ctb * kb;
        dqs[f0 * WG + tid] += cf * (xf1 * xf2);
        dqs[f1 * WG + tid] += cf * (xf0 * xf2);
        dqs[f2 * WG + tid] += cf * (xf0 * xf1);
        dqs[r0 * WG + tid] -= cb * (xb1 * xb2);
        dqs[r1 * WG + tid] -= cb * (xb0 * xb2);
        dqs[r2 * WG + tid] -= cb * (xb0 * xb1);
        // d(rho Y_m): dX_j/d(rho Y_m) = delta_jm / M_m - delta_{j,last} / M_last
        const double dlast = dqs[NT * WG + tid] * m->invM[NT];
        double Dm[NT];
#pragma unroll
        for (int mm = 0; mm < NT; ++mm) Dm[mm] = dqs[mm * WG + tid] * m->invM[mm] - dlast;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            if (m->dnu[i][k] != 0) {
                const double ck = m->Mdnu[i][k];
#pragma unroll
                for (int mm = 0; mm < NT; ++mm) J[k][mm] += ck * Dm[mm];
            }
        }
    }
    if constexpr (FULLJ) {
        const double ilast = hm1[NT] * m->invM[NT];
#pragma unroll
        for (int mm = 0; mm < NT; ++mm) {
            const double dTm = -T * (hm1[mm] * m->invM[mm] - ilast) / cvs;
#pragma unroll
            for (int k = 0; k < NT; ++k) J[k][mm] += dSdT[k] * dTm;
        }
    }
    chem_solve<NS>(J, w, dt, st);
}

// One chemistry launch over the tiles (one cell per thread): the dt of the phase, the
// point-implicit step `cell(mech, rho, T, rho Y, dt, dY, status)` on each solved cell,
// Newton for the new T, and the maxima for the next stage. Shared by the generic kernel
// below and the kernel specialised at run time to a mechanism's structure.
template <int NS, class Cell>
__device__ __forceinline__ void chem_body(const StageArgs& a, double* scratch, Cell&& cell) {
    constexpr int NU = NS + 3;
    const Tile tile = a.tiles[blockIdx.x];
    const DevBlock B = a.blk[tile.block];
    CDom& D = cdom(a.dom, B.domain);
    CMech* mech = cmech(a.mech);
    const CellRef r = tile_cell(a, tile, B);
    const int lev = B.level, slot = D.slot0 + lev;
    // phase 0: the whole dt after the stages (Lie); phase 1: dt/2 before stage 1, this
    // launch forms the step's dt; phase 2: dt/2 after stage 3 (Strang, Sec. 4.2)
    const int phase = a.chem_phase;
    const double dstep = a.cross ? ldexp((phase == 1 && a.xfirst) ? step_dt(a, B.domain, 0)
                                                                   : a.dt[B.domain], -lev)
                                 : (phase == 1) ? step_dt(a, B.domain, 0) : a.dt[B.domain];
    const double dt = (phase == 0) ? dstep : 0.5 * dstep;
    const double idx = (double)(1 << lev) / D.dx0, idy = (double)(1 << lev) / D.dy0;
    if (blockIdx.x == 0) {
        if (phase == 1) {
            if (!a.cross || a.xfirst) record_dt(a);
        } else if (!a.cross || a.xlast) {
            step_finish(a);
        }
    }
    if (phase == 2)   // buffer 3 was read by stage 1; clean for the next step's first half
        for (int q = threadIdx.x; q < a.red.stride; q += WG) a.red.buf[slot_word(a.red.stride, 3, q)] = 0ull;
    if (!(dt > 0.0)) return;
    // A cell under a finer block is overwritten by the restriction that follows this
    // launch (the Lie step, or the second half of the Strang split; in the crossover
    // advance, the level's last step) and leaves the maxima (the restriction publishes
    // the restricted cell's instead). Where none of its four children is a ring cell,
    // the restriction does not read it either: its chemistry is dead work.
    const bool covered = r.own && phase != 1 && B.fine_child && (!a.cross || a.xskip_cov) &&
                         covered_by_finer(a, D, lev, r.I, r.J);
    const bool dead = covered && restricted_over(a, D, lev, r.I, r.J);
    const bool work = r.own && !dead;
    double sx = 0.0, sy = 0.0, sc = 0.0;
    unsigned st = 0u;
    double dY[NS - 1];
    double T = 1.0;
    {
        // inactive lanes run the same arithmetic on a harmless state
        double rho = 1.0;
        double rY[NS - 1];
#pragma unroll
        for (int k = 0; k < NS - 1; ++k) rY[k] = 0.0;
        if (work) {
            rho = a.Uout[r.c];
#pragma unroll
            for (int k = 0; k < NS - 1; ++k) rY[k] = a.Uout[(size_t)(4 + k) * a.pool + r.c];
            T = a.Tout[r.c];
        }
        if (__any(work)) cell(mech, rho, T, rY, dt, dY, st);   // wavefronts with no work skip it
    }
    if (work) {
        double u[NU];
#pragma unroll
        for (int f = 0; f < NU; ++f) u[f] = a.Uout[(size_t)f * a.pool + r.c];
#pragma unroll
        for (int k = 0; k < NS - 1; ++k) {
            u[4 + k] += dY[k];
            a.Uout[(size_t)(4 + k) * a.pool + r.c] = u[4 + k];
        }
        double Tn, c, vx, vy;
        st |= owner_state<DETAILED, NU>(u, T, D, mech, Tn, c, vx, vy);
        a.Tout[r.c] = Tn;
        if (st) atomicOr(a.status, st);
        // the first half's maxima are stage 1's alpha over all solved cells
        if (!st && !covered) {
            sx = fabs(vx) + c;
            sy = fabs(vy) + c;
            sc = cfl_bound(a, D, lev, sx, sy, idx, idy);
        }
    }
    publish_max3(a.red, (phase == 1) ? 3 : 0, 2 * slot, 2 * slot + 1, 2 * a.red.nunits + B.domain, sx,
                 sy, sc, scratch);
}

#ifndef CHEM_WAVES
#define CHEM_WAVES 1
#endif
template <int NS, bool FULLJ>
__global__ __launch_bounds__(WG, CHEM_WAVES) void chem_kernel(StageArgs a) {
    __shared__ double Xs[(NS + 1) * WG];
    __shared__ double gts[(NS + 1) * WG];
    __shared__ double dqs[(NS + 1) * WG];
    __shared__ double scratch[16];
    chem_body<NS>(a, scratch, [&](CMech* m, double rho, double T, const double (&rY)[NS - 1],
                                  double dt, double (&dY)[NS - 1], unsigned& st) {
        chem_cell<NS, FULLJ>(m, Xs, gts, dqs, rho, T, rY, dt, dY, st);
    });
}

// Four-to-one restriction (Sec. 3.1.4 coarsening): each coarse cell under a
// valid block of this level becomes the mean of its four children (ring
// children count with their effective value, the coarse cell itself); T is
// re-solved; the coarse cell enters the maxima of the next step. Workgroup
// (b, y) takes coarse cells y*WG, y*WG + gridDim.y*WG, ... of fine block b.
template <int M, int NU>
__global__ __launch_bounds__(WG) void restrict_kernel(StageArgs a, const int* fine_blocks) {
    __shared__ double scratch[16];
    const DevBlock B = a.blk[fine_blocks[blockIdx.x]];
    CDom& D = cdom(a.dom, B.domain);
    const int lev = B.level;
    const double dt = a.dt[B.domain];
    const int cw = B.nx / 2, ch = B.ny / 2;
    if (!(dt > 0.0) || (int)blockIdx.y * WG >= cw * ch) return;
    const int cslot = D.slot0 + lev - 1;
    const double idx = (double)(1 << (lev - 1)) / D.dx0, idy = (double)(1 << (lev - 1)) / D.dy0;
    double sx = 0.0, sy = 0.0, sc = 0.0;
    for (int cc = blockIdx.y * WG + threadIdx.x; cc < cw * ch; cc += gridDim.y * WG) {
        const int cj = cc / cw, ci = cc - cj * cw;
        unsigned fl = 0u;
        const long long cpar = resolve(a, D, lev - 1, (B.i0 >> 1) + ci, (B.j0 >> 1) + cj, fl);
        double mean[NU];
        double ch4[4][NU];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int li = 2 * ci + (q & 1), lj = 2 * cj + (q >> 1);
            long long s;
            unsigned f2 = 0u;
            if (!ring_at(B, li, lj)) s = B.offset + (long long)lj * B.nx + li;
            else s = resolve(a, D, lev - 1, (B.i0 + li) >> 1, (B.j0 + lj) >> 1, f2);
            double Tq;
            fetch<NU>(a, s, f2, a.Uout, a.Tout, ch4[q], Tq);
        }
#pragma unroll
        for (int f = 0; f < NU; ++f) mean[f] = ((ch4[0][f] + ch4[1][f]) + (ch4[2][f] + ch4[3][f])) * 0.25;
        // all children are read before any coarse value changes: a ring child of this
        // coarse cell resolves to the cell itself, which only this thread writes
#pragma unroll
        for (int f = 0; f < NU; ++f) a.Uout[(size_t)f * a.pool + cpar] = mean[f];
        double T, c, vx, vy;
        const unsigned st = owner_state<M, NU>(mean, a.Tout[cpar], D, cmech(a.mech), T, c, vx, vy);
        a.Tout[cpar] = T;
        if (st) atomicOr(a.status, st);
        else {
            sx = fmax(sx, fabs(vx) + c);
            sy = fmax(sy, fabs(vy) + c);
            sc = fmax(sc, cfl_bound(a, D, lev - 1, fabs(vx) + c, fabs(vy) + c, idx, idy));
        }
    }
    publish_max3(a.red, 0, 2 * cslot, 2 * cslot + 1, 2 * a.red.nunits + B.domain, sx, sy, sc,
                 scratch);
}

// Ring cells take the injection (one-to-four) of the coarser level after restriction.
// Only the 3-cell bands along the four sides can hold ring cells: workgroup (b, y)
// walks the band cells y*WG, y*WG + gridDim.y*WG, ... of block b (W, E, S, N bands;
// a corner cell lies in two bands and is written twice with the same value).
template <int NU>
__global__ __launch_bounds__(WG) void ring_fill_kernel(StageArgs a, const int* ring_blocks) {
    const DevBlock B = a.blk[ring_blocks[blockIdx.x]];
    CDom& D = cdom(a.dom, B.domain);
    const int nband = 6 * B.ny + 6 * B.nx;
    if (!(a.dt[B.domain] > 0.0) || (int)blockIdx.y * WG >= nband) return;
    for (int q = blockIdx.y * WG + threadIdx.x; q < nband; q += gridDim.y * WG) {
        int li, lj;
        if (q < 6 * B.ny) {
            const int r = (q < 3 * B.ny) ? q : q - 3 * B.ny;
            lj = r / 3;
            li = (q < 3 * B.ny) ? r - 3 * lj : B.nx - 3 + (r - 3 * lj);
        } else {
            const int h = q - 6 * B.ny, r = (h < 3 * B.nx) ? h : h - 3 * B.nx;
            const int row = r / B.nx;
            li = r - row * B.nx;
            lj = (h < 3 * B.nx) ? row : B.ny - 3 + row;
        }
        if (!ring_at(B, li, lj)) continue;
        unsigned fl = 0u;
        const long long s = resolve(a, D, B.level - 1, (B.i0 + li) >> 1, (B.j0 + lj) >> 1, fl);
        double u[NU], T;
        fetch<NU>(a, s, fl, a.Uout, a.Tout, u, T);
        const long long c = B.offset + (long long)lj * B.nx + li;
#pragma unroll
        for (int f = 0; f < NU; ++f) a.Uout[(size_t)f * a.pool + c] = u[f];
        a.Tout[c] = T;
    }
}

// Conserved state from primitives (Eq. 4.2), one thread per cell.
template <int M, int NU>
__global__ void prim_to_cons_kernel(const DevMech* mech, double gamma, double R, double Q,
                                    long long n, const double* W, double* U, double* T,
                                    long long sin, long long sout) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double w[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) w[f] = W[(size_t)f * sin + c];
    if constexpr (M == DETAILED) {
        constexpr int NS = NU - 3;
        const double p = w[0], u = w[1], v = w[2], Tt = w[3];
        double Y[NS], s = 0.0;
#pragma unroll
        for (int k = 0; k < NS - 1; ++k) {
            Y[k] = w[4 + k];
            s += Y[k];
        }
        Y[NS - 1] = 1.0 - s;
        double Rm = 0.0, e = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double* a = (mech->two_range && Tt >= mech->tmid[k]) ? mech->nasa_hi[k] : mech->nasa[k];
            const double h = Tt * (a[0] + Tt * (0.5 * a[1] + Tt * (a[2] * (1.0 / 3.0) +
                             Tt * (0.25 * a[3] + Tt * (0.2 * a[4]))))) + a[5];
            Rm += Y[k] * mech->Rk[k];
            e += Y[k] * mech->Rk[k] * (h - Tt);
        }
        const double rho = p / (Rm * Tt);
        U[c] = rho;
        U[(size_t)sout + c] = rho * u;
        U[(size_t)2 * sout + c] = rho * v;
        U[(size_t)3 * sout + c] = rho * e + 0.5 * rho * (u * u + v * v);
#pragma unroll
        for (int k = 0; k < NS - 1; ++k) U[(size_t)(4 + k) * sout + c] = rho * Y[k];
        T[c] = Tt;
    } else {
        const double rho = w[0], u = w[1], v = w[2], p = w[3];
        U[c] = rho;
        U[(size_t)sout + c] = rho * u;
        U[(size_t)2 * sout + c] = rho * v;
        double E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v);
        if constexpr (M == ONESTEP) {
            E += rho * w[4] * Q;
            U[(size_t)4 * sout + c] = rho * w[4];
        }
        U[(size_t)3 * sout + c] = E;
        T[c] = p / (rho * R);
    }
}

// ------------------------------------------------------------------ launch shapes
// Workgroups per block of the restriction and ring-fill launches (a 64 x 64 fine
// block has 1024 coarse cells and 768 band cells: four workgroups of 256 threads).
constexpr int RESTRICT_SPLIT = 4;

}  // namespace janc
