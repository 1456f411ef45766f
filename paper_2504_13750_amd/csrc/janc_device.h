// janc_device.h -- device helpers shared by the forward and adjoint kernels:
// reduction slots, coarse-fine ring tests, source resolution, primitives,
// Newton for T, WENO5 and the RK combination. Included by .hip files only.
#pragma once

#include "janc_internal.h"

namespace janc {

constexpr double WENO_EPS = 1e-6;

// Read-only tables (domains, mechanism) viewed through the constant address
// space: the compiler may then serve workgroup-uniform reads from scalar loads,
// also after the kernel's own global stores.
typedef __attribute__((address_space(4))) const DevMech CMech;
typedef __attribute__((address_space(4))) const DevDomain CDom;
__device__ __forceinline__ CMech* cmech(const DevMech* p) { return (CMech*)p; }
__device__ __forceinline__ CDom& cdom(const DevDomain* p, int d) { return ((CDom*)p)[d]; }

// ------------------------------------------------------------------ small helpers
__device__ __forceinline__ double sq(double x) { return x * x; }

// Word of slot idx of buffer buf (each slot alone in a 128-byte line).
__device__ __forceinline__ size_t slot_word(int stride, int buf, int idx) {
    return ((size_t)buf * stride + idx) * SLOT_WORDS;
}

__device__ __forceinline__ double slot_get(const Reduce& r, int buf, int idx) {
    return __longlong_as_double((long long)r.buf[slot_word(r.stride, buf, idx)]);
}

__device__ __forceinline__ void slot_max(const Reduce& r, int buf, int idx, double v) {
    // v >= 0: the bit pattern orders like the value
    atomicMax(&r.buf[slot_word(r.stride, buf, idx)], (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Workgroup max of three values; thread 0 publishes them.
__device__ __forceinline__ void publish_max3(const Reduce& r, int buf, int i0, int i1, int i2,
                                             double v0, double v1, double v2, double* scratch) {
    v0 = wave_max(v0);
    v1 = wave_max(v1);
    v2 = wave_max(v2);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        scratch[3 * w + 0] = v0;
        scratch[3 * w + 1] = v1;
        scratch[3 * w + 2] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m0 = scratch[0], m1 = scratch[1], m2 = scratch[2];
        for (int q = 1; q < WG / 64; ++q) {
            m0 = fmax(m0, scratch[3 * q]);
            m1 = fmax(m1, scratch[3 * q + 1]);
            m2 = fmax(m2, scratch[3 * q + 2]);
        }
        if (m0 > 0.0) slot_max(r, buf, i0, m0);
        if (m1 > 0.0) slot_max(r, buf, i1, m1);
        if (m2 > 0.0) slot_max(r, buf, i2, m2);
    }
}

// Coarse-fine ring test for block-local cell (li, lj) (segment masks per side).
__device__ __forceinline__ bool ring_at(const DevBlock& B, int li, int lj) {
    const unsigned sx = (unsigned)(lj >> 3) & 31u, sy = (unsigned)(li >> 3) & 31u;
    return (li < 3 && ((B.ring[0] >> sx) & 1u)) || (li >= B.nx - 3 && ((B.ring[1] >> sx) & 1u)) ||
           (lj < 3 && ((B.ring[2] >> sy) & 1u)) || (lj >= B.ny - 3 && ((B.ring[3] >> sy) & 1u));
}

// Effective source of level-`lev` cell (I, J) of domain D: boundary rule first,
// then the covering block of that level, or the coarser level where the cell is
// uncovered or a ring cell. Returns a pool cell (>= 0) or -(1 + Dirichlet row);
// fl gets bit 0 / bit 1 when x / y momentum must be mirrored.
__device__ long long resolve(const StageArgs& a, CDom& D, int lev, int I, int J,
                             unsigned& fl) {
    const int W = D.nx0 << lev, H = D.twod ? (D.ny0 << lev) : 1;
    if (I < 0 || I >= W) {
        const int side = (I < 0) ? 0 : 1;
        switch (D.bc[side]) {
            case BC_PERIODIC: I = (I < 0) ? I + W : I - W; break;
            case BC_ZEROGRAD: I = (I < 0) ? 0 : W - 1; break;
            case BC_SLIPWALL: I = (I < 0) ? -I - 1 : 2 * W - 1 - I; fl ^= 1u; break;
            default: return -(1ll + D.dir[side]);
        }
    }
    if (J < 0 || J >= H) {
        const int side = (J < 0) ? 2 : 3;
        switch (D.bc[side]) {
            case BC_PERIODIC: J = (J < 0) ? J + H : J - H; break;
            case BC_ZEROGRAD: J = (J < 0) ? 0 : H - 1; break;
            case BC_SLIPWALL: J = (J < 0) ? -J - 1 : 2 * H - 1 - J; fl ^= 2u; break;
            default: return -(1ll + D.dir[side]);
        }
    }
    for (;;) {
        const int b = a.maps[D.map_off[lev] + (J >> 3) * D.map_w[lev] + (I >> 3)];
        if (b >= 0) {
            const DevBlock& B = a.blk[b];
            const int li = I - B.i0, lj = J - B.j0;
            if (!ring_at(B, li, lj)) return B.offset + (long long)lj * B.nx + li;
        }
        // level 0 tiles the domain and has no ring cells, so this ends; bit 2 of fl
        // marks a source on a coarser level than the one asked for
        --lev;
        I >>= 1;
        J >>= 1;
        fl |= 4u;
    }
}

template <int NU>
__device__ __forceinline__ void fetch(const StageArgs& a, long long src, unsigned fl,
                                      const double* Uarr, const double* Tarr, double (&u)[NU],
                                      double& T) {
    if (src >= 0) {
#pragma unroll
        for (int f = 0; f < NU; ++f) u[f] = Uarr[(size_t)f * a.pool + src];
        T = Tarr[src];
    } else {
        const double* r = a.dirU + (size_t)(-src - 1) * (MAXF + 1);
#pragma unroll
        for (int f = 0; f < NU; ++f) u[f] = r[f];
        T = r[MAXF];
    }
    if (fl & 1u) u[1] = -u[1];
    if (fl & 2u) u[2] = -u[2];
}

// Velocities and pressure of a stencil cell (Eq. 4.2; T from storage for NASA-7).
template <int M, int NU, class Dom, class Mech>
__device__ __forceinline__ void halo_prims(const double (&u)[NU], double T, const Dom& D,
                                           Mech mech, double& vx, double& vy,
                                           double& p) {
    const double ir = 1.0 / u[0];
    vx = u[1] * ir;
    vy = u[2] * ir;
    if constexpr (M == DETAILED) {
        double s = 0.0, r = 0.0;
#pragma unroll
        for (int k = 0; k < NU - 4; ++k) {
            s += u[4 + k];
            r += u[4 + k] * mech->invM[k];
        }
        r += (u[0] - s) * mech->invM[NU - 4];
        p = RU * r * T;
    } else {
        double e = u[3] * ir - 0.5 * (vx * vx + vy * vy);
        if constexpr (M == ONESTEP) e -= u[4] * ir * D.Q;
        p = (D.gamma - 1.0) * u[0] * e;
    }
}

// Mixture NASA-7 coefficients (Y fixed, so the species sums are formed once): per mass,
// sum_k Y_k R_k a_q of each range, and R_mix. With two NASA-7 ranges (one t_mid for all
// species) both sets are formed and an evaluation uses the set of its temperature.
struct MixNasa {
    double b[6], h[6];
    double Rmix, tm;
    bool two;
};

template <int NS>
__device__ __forceinline__ void mix_nasa(const double (&Y)[NS], CMech* m, MixNasa& x) {
    double b0 = 0.0, b1 = 0.0, b2 = 0.0, b3 = 0.0, b4 = 0.0, b5 = 0.0;
    double h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0, h4 = 0.0, h5 = 0.0;
    x.two = m->two_range != 0;
    x.tm = m->tmid[0];
    x.Rmix = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const double w = Y[k] * m->Rk[k];
        x.Rmix += w;
        b0 += w * m->nasa[k][0];
        b1 += w * m->nasa[k][1];
        b2 += w * m->nasa[k][2];
        b3 += w * m->nasa[k][3];
        b4 += w * m->nasa[k][4];
        b5 += w * m->nasa[k][5];
        if (x.two) {
            h0 += w * m->nasa_hi[k][0];
            h1 += w * m->nasa_hi[k][1];
            h2 += w * m->nasa_hi[k][2];
            h3 += w * m->nasa_hi[k][3];
            h4 += w * m->nasa_hi[k][4];
            h5 += w * m->nasa_hi[k][5];
        }
    }
    x.b[0] = b0; x.b[1] = b1; x.b[2] = b2; x.b[3] = b3; x.b[4] = b4; x.b[5] = b5;
    x.h[0] = h0; x.h[1] = h1; x.h[2] = h2; x.h[3] = h3; x.h[4] = h4; x.h[5] = h5;
}

// e(T) and cv(T) of the mixture (per mass).
__device__ __forceinline__ void mix_eval(const MixNasa& x, double Tc, double& ec, double& cvv) {
    const bool hi = x.two && Tc >= x.tm;
    const double B0 = hi ? x.h[0] : x.b[0], B1 = hi ? x.h[1] : x.b[1], B2 = hi ? x.h[2] : x.b[2],
                 B3 = hi ? x.h[3] : x.b[3], B4 = hi ? x.h[4] : x.b[4], B5 = hi ? x.h[5] : x.b[5];
    const double c0 = B0 - x.Rmix, c1 = 0.5 * B1, c2 = B2 * (1.0 / 3.0), c3 = 0.25 * B3,
                 c4 = 0.2 * B4;
    ec = Tc * (c0 + Tc * (c1 + Tc * (c2 + Tc * (c3 + Tc * c4)))) + B5;
    cvv = c0 + Tc * (B1 + Tc * (B2 + Tc * (B3 + Tc * B4)));
}

// Newton for T from the internal energy on the mixture coefficients (Sec. 4.2).
template <int NS>
__device__ __forceinline__ unsigned newton_T(const double (&Y)[NS], double e, CMech* m,
                                             double& T, double& cv, double& Rmix) {
    MixNasa x;
    mix_nasa<NS>(Y, m, x);
    Rmix = x.Rmix;
    unsigned st = STB_NEWTON;
    for (int it = 0; it < 50; ++it) {
        double ec, cvv;
        mix_eval(x, T, ec, cvv);
        const double dT = (ec - e) / cvv;
        T -= dT;
        if (!(fabs(dT) <= 1e-12 * fabs(T))) {
            if (!isfinite(T)) { st = STB_NONFINITE; break; }
            continue;
        }
        st = 0u;
        break;
    }
    double ec;
    mix_eval(x, T, ec, cv);
    return st;
}

// State of an owned cell after an update: T (closed form or Newton from Tprev),
// sound speed and velocities; returns status bits.
template <int M, int NU, class Dom, class Mech>
__device__ __forceinline__ unsigned owner_state(const double (&u)[NU], double Tprev,
                                                const Dom& D, Mech mech,
                                                double& T, double& c, double& vx, double& vy) {
    const double rho = u[0];
    if (!isfinite(rho)) return STB_NONFINITE;
    if (!(rho > 0.0)) return STB_NEGATIVE;
    const double ir = 1.0 / rho;
    vx = u[1] * ir;
    vy = u[2] * ir;
    const double e = u[3] * ir - 0.5 * (vx * vx + vy * vy);
    double p, gam;
    unsigned st = 0u;
    if constexpr (M == DETAILED) {
        constexpr int NS = NU - 3;
        double Y[NS];
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NS - 1; ++k) {
            Y[k] = u[4 + k] * ir;
            s += Y[k];
        }
        Y[NS - 1] = 1.0 - s;
        T = Tprev;
        double cv, Rmix;
        st = newton_T<NS>(Y, e, mech, T, cv, Rmix);
        p = rho * Rmix * T;
        gam = (cv + Rmix) / cv;
    } else {
        double ee = e;
        if constexpr (M == ONESTEP) ee -= u[4] * ir * D.Q;
        p = (D.gamma - 1.0) * rho * ee;
        T = p / (rho * D.R);
        gam = D.gamma;
    }
    if (!isfinite(p) || !isfinite(T)) return st | STB_NONFINITE;
    if (!(p > 0.0) || !(T > 0.0)) return st | STB_NEGATIVE;
    c = sqrt(gam * p * ir);
    return st;
}

// WENO5-JS at i+1/2 from f_{i-2..i+2} (a..e), written in first differences
// d1..d4: the candidate values are c + r_k / 6, the smoothness indicators times 12
// are 13 (second difference)^2 + 3 (one-sided slope)^2 (the common factor 144 of
// the squared (eps + beta) cancels in the normalized weights), and the weighted
// average is c + sum w_k r_k / (6 sum w_k) with the weights in common-denominator
// form (one division). Algebraically the textbook form; fewer operations.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e) {
    const double d1 = b - a, d2 = c - b, d3 = d - c, d4 = e - d;
    const double r0 = 5.0 * d2 - 2.0 * d1, r1 = d2 + 2.0 * d3, r2 = 4.0 * d3 - d4;
    const double t0 = d2 - d1, t1 = d3 - d2, t2 = d4 - d3;
    const double u0 = 3.0 * d2 - d1, u1 = d2 + d3, u2 = d4 - 3.0 * d3;
    const double s0 = sq((12.0 * WENO_EPS + 13.0 * t0 * t0) + 3.0 * u0 * u0);
    const double s1 = sq((12.0 * WENO_EPS + 13.0 * t1 * t1) + 3.0 * u1 * u1);
    const double s2 = sq((12.0 * WENO_EPS + 13.0 * t2 * t2) + 3.0 * u2 * u2);
    const double w0 = 0.1 * (s1 * s2), w1 = 0.6 * (s0 * s2), w2 = 0.3 * (s0 * s1);
    return c + (w0 * r0 + w1 * r1 + w2 * r2) / (6.0 * (w0 + w1 + w2));
}

__device__ __forceinline__ double rk_combine(int stage, double u0, double us, double L, double dt) {
    if (stage == 1) return u0 + dt * L;
    if (stage == 2) return 0.75 * u0 + 0.25 * (us + dt * L);
    return (1.0 / 3.0) * u0 + (2.0 / 3.0) * (us + dt * L);
}

// dt of domain d for this step from the CFL slot of buffer `bin`; in the crossover
// advance dt_0, from the largest bound over every level's slot triple.
__device__ __forceinline__ double step_dt(const StageArgs& a, int d, int bin) {
    double dt;
    if (a.tm.dt_fixed > 0.0) {
        dt = a.tm.dt_fixed;
    } else if (a.cross) {
        double m = 0.0;
        for (int l = 0; l < a.xlevels; ++l)
            m = fmax(m, __longlong_as_double((long long)a.xred[slot_word(a.red.stride, l * RED_BUFS + bin,
                                                                         2 * a.red.nunits + d)]));
        dt = a.tm.cfl / m;
    } else {
        dt = a.tm.cfl / slot_get(a.red, bin, 2 * a.red.nunits + d);
    }
    if (a.tm.t_end > 0.0) {
        const double rem = a.tm.t_end - a.t[d];
        if (!(rem > 0.0)) dt = 0.0;
        else if (dt > rem) dt = rem;
    }
    return dt;
}

// Is level-`lev` cell (I, J) of D under a valid block of level lev+1?
__device__ __forceinline__ bool covered_by_finer(const StageArgs& a, CDom& D, int lev,
                                                 int I, int J) {
    if (lev + 1 >= D.nlevels) return false;
    const int I2 = 2 * I, J2 = 2 * J;
    return a.maps[D.map_off[lev + 1] + (J2 >> 3) * D.map_w[lev + 1] + (I2 >> 3)] >= 0;
}

// Level-lev cell (I, J) lies under a finer valid block and none of its four children is
// a coarse-fine ring cell of that block: the restriction replaces it by the mean of its
// children without reading it. (Fine blocks sit on even cells, so the 2 x 2 children
// belong to one block.)
__device__ __forceinline__ bool restricted_over(const StageArgs& a, CDom& D, int lev, int I, int J) {
    if (lev + 1 >= D.nlevels || !D.twod) return false;
    const int I2 = 2 * I, J2 = 2 * J;
    const int b = a.maps[D.map_off[lev + 1] + (J2 >> 3) * D.map_w[lev + 1] + (I2 >> 3)];
    if (b < 0) return false;
    const DevBlock& F = a.blk[b];
    const int li = I2 - F.i0, lj = J2 - F.j0;
    return !ring_at(F, li, lj) && !ring_at(F, li + 1, lj) && !ring_at(F, li, lj + 1) &&
           !ring_at(F, li + 1, lj + 1);
}

// The dispatcher deals the workgroups of a launch round-robin over the 8 XCDs,
// each with its own L2. Workgroup b of n is given tile chunk(b) so that each XCD
// walks one contiguous run of tiles: neighbouring tiles, whose halos overlap,
// then read them through the same L2. The map is a bijection of [0, n).
__device__ __forceinline__ int xcd_chunk(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7;
    return x * q + min(x, r) + (b >> 3);
}

// CFL bound of a cell with wave speeds sx, sy at the spacing of its level (1/dx, 1/dy);
// in the crossover advance at the spacing of level 0, so that dt_0 bounds every level.
__device__ __forceinline__ double cfl_bound(const StageArgs& a, CDom& D, int lev, double sx,
                                            double sy, double idx, double idy) {
    if (a.cross) {
        idx = ldexp(idx, -lev);
        idy = ldexp(idy, -lev);
    }
    return sx * idx + (D.twod ? sy * idy : 0.0);
}

// Per-launch bookkeeping done by workgroup 0: rotate reduction buffers, dt and t.
// This step's dt per domain (from buffer 0's CFL slots) into a.dt and the dt log.
__device__ void record_dt(const StageArgs& a) {
    const int step = *a.step;
    for (int d = threadIdx.x; d < a.ndom; d += WG) {
        const double dt = step_dt(a, d, 0);
        a.dt[d] = dt;
        if (a.dt_log && step < a.dt_log_cap) a.dt_log[(size_t)step * a.ndom + d] = dt;
    }
}

__device__ void stage_bookkeeping(const StageArgs& a, int owner_launch) {
    const int s = a.stage;
    const int bclear = (s + 1) % 3;
    for (int q = threadIdx.x; q < a.red.stride; q += WG) a.red.buf[slot_word(a.red.stride, bclear, q)] = 0ull;
    if (a.cross) owner_launch = a.xfirst;
    if (!owner_launch) return;
    if (s == 1 && !a.strang) record_dt(a);   // under Strang splitting the first chemistry launch does
}

__device__ void step_finish(const StageArgs& a) {
    for (int d = threadIdx.x; d < a.ndom; d += WG) a.t[d] = a.t[d] + a.dt[d];
    if (threadIdx.x == 0) *a.step = *a.step + 1;
}


}  // namespace janc
