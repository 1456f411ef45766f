// janc_adjoint.h -- hand-written discrete adjoint of SSP-RK3 steps on a uniform
// grid (the adjoint method of paper Sec. 6.1, Eq. 6.1-6.5, applied to the discrete
// trajectory: the result is the exact gradient of the discrete forward map), for the
// one-step model and for the detailed model (NASA-7 thermodynamics with the
// temperature Newton, Eq. 4.2-4.5; point-implicit chemistry, Eq. 4.6-4.13).
//
// A stage W = a U^n + b (V + dt L(V)) is reversed as
//   lambda_V  = b lambda_W + (dL/dV)^T mu,   mu = b dt lambda_W,
//   lambda_Un += a lambda_W,  theta-gradient += (dL/dtheta)^T mu,
// with L(V) = -dF/dx - dG/dy + S. The vector-Jacobian product (dL/dV)^T mu is
// formed in gather form, without atomics on floating-point values:
//   A  (once per checkpoint segment, every stage input of the segment)
//      alpha_x = max(|u|+c), alpha_y = max(|v|+c) and their argmax (lowest
//      linear index among equal maxima): block maxima, then one workgroup per
//      stage input;
//   B  per interface and component: mu_Fhat = b dt (mu_right - mu_left)/dx and
//      the reverse of both WENO5 reconstructions (5 + 5 weights), the six
//      stencil states and their split fluxes formed in place;
//   C  per interior cell (x and y sweeps on two threads): gather of the
//      split-flux adjoints of its own strip positions and of the ghost positions
//      that copy or mirror it from the 5 + 5 interfaces that read them, reverse
//      of the split (flux Jacobian and the alpha term), the explicit Arrhenius
//      source (one-step model), the RK bookkeeping, block partials of d/dalpha,
//      d/dQ, d/dEa;
//   D  one workgroup: the partials summed in a fixed order, the alpha adjoints
//      applied at the argmax cells, theta, and the loss seed of the step start.
// The temperature of the detailed model is the Newton root of e(T, Y) = e; it is
// differentiated by the implicit-function theorem: dT = (de - sum_k (e_k - e_last)
// dY_k) / c_v. Its point-implicit chemistry step (I - dt J) dU = dt S, J = dS/d(rho Y)
// at frozen T and rho, is reversed per cell: mu = (I - dt J)^-T lambda, and the inputs
// (rho Y, rho, T) receive dt d/dx [mu . S(x) + mu . J(x) dU], the second term through
// the directional derivative of the rates along dU (a Hessian-vector product written
// out per reaction).
// Every thread issues its loads together (clamped indices, masked afterwards):
// the small grids of an adjoint run are bound by memory latency, not bandwidth.
#pragma once

#include "janc_device.h"

namespace janc {

// Source of grid position (i, j) (one coordinate may lie in the 3 ghost layers).
__device__ inline long long usrc(const AdjGrid& g, int i, int j, unsigned& fl) {
    fl = 0u;
    if (i < 0 || i >= g.nx) {
        const int side = (i < 0) ? 0 : 1;
        switch (g.bc[side]) {
            case BC_PERIODIC: i = ((i % g.nx) + g.nx) % g.nx; break;
            case BC_ZEROGRAD: i = (i < 0) ? 0 : g.nx - 1; break;
            case BC_SLIPWALL: i = (i < 0) ? -i - 1 : 2 * g.nx - 1 - i; fl ^= 1u; break;
            default: return -(1ll + g.dir[side]);
        }
    }
    if (j < 0 || j >= g.ny) {
        const int side = (j < 0) ? 2 : 3;
        switch (g.bc[side]) {
            case BC_PERIODIC: j = ((j % g.ny) + g.ny) % g.ny; break;
            case BC_ZEROGRAD: j = (j < 0) ? 0 : g.ny - 1; break;
            case BC_SLIPWALL: j = (j < 0) ? -j - 1 : 2 * g.ny - 1 - j; fl ^= 2u; break;
            default: return -(1ll + g.dir[side]);
        }
    }
    return (long long)j * g.nx + i;
}

// The cell loads are issued unconditionally (index clamped) so that the loads of
// several points are in flight together; a Dirichlet row replaces them.
template <int M, int NU>
__device__ __forceinline__ void load_src(const AdjArgs& A, long long s, unsigned fl, double (&u)[NU],
                                         double& T) {
    const long long sc = s >= 0 ? s : 0;
#pragma unroll
    for (int f = 0; f < NU; ++f) u[f] = A.V[(size_t)f * A.n + sc];
    T = (M == DETAILED) ? A.VT[sc] : 0.0;
    if (s < 0) {
        const double* r = A.g.dirU + (size_t)(-s - 1) * (MAXF + 1);
#pragma unroll
        for (int f = 0; f < NU; ++f) u[f] = r[f];
        T = r[MAXF];
    }
    if (fl & 1u) u[1] = -u[1];
    if (fl & 2u) u[2] = -u[2];
}

// ------------------------------------------------------------------ thermodynamics
// Per-species NASA-7 data at T (per mass): internal energy e_k = R_k (h_k/R - T),
// c_v,k = R_k (c_p,k/R - 1) and d c_v,k / dT; mixture R, c_v and d c_v/dT.
template <int NS>
struct SpeciesAt {
    double Rm, cv, dcv;
    double ek[NS], cvk[NS];
};

template <int NS>
__device__ __forceinline__ void species_at(CMech* m, const double (&Y)[NS], double T, SpeciesAt<NS>& s) {
    s.Rm = 0.0;
    s.cv = 0.0;
    s.dcv = 0.0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const bool hi = m->two_range && T >= m->tmid[k];
        double a[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) a[q] = hi ? m->nasa_hi[k][q] : m->nasa[k][q];
        const double Rk = m->Rk[k];
        const double cpt = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
        const double ht = T * (a[0] + T * (0.5 * a[1] + T * (a[2] * (1.0 / 3.0) + T * (0.25 * a[3] + T * (0.2 * a[4]))))) + a[5];
        const double dcp = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * (4.0 * a[4])));
        s.ek[k] = Rk * (ht - T);
        s.cvk[k] = Rk * (cpt - 1.0);
        s.Rm += Y[k] * Rk;
        s.cv += Y[k] * s.cvk[k];
        s.dcv += Y[k] * Rk * dcp;
    }
}

// Mass fractions of all species from a conserved state (last = complement).
template <int NU>
__device__ __forceinline__ void mass_fractions(const double (&V)[NU], double ir, double (&Y)[NU - 3]) {
    constexpr int NS = NU - 3;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NS - 1; ++k) {
        Y[k] = V[4 + k] * ir;
        s += Y[k];
    }
    Y[NS - 1] = 1.0 - s;
}

// dT/dU of the Newton temperature (implicit-function theorem on e(T, Y) = e).
template <int NU>
__device__ __forceinline__ void temperature_grad(const double (&V)[NU], const double (&Y)[NU - 3],
                                                 const SpeciesAt<NU - 3>& s, double (&dT)[NU]) {
    constexpr int NS = NU - 3, NT = NS - 1;
    const double rho = V[0], ir = 1.0 / rho;
    const double u = V[1] * ir, v = V[2] * ir;
    const double iC = ir / s.cv;
    double sy = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) sy += (s.ek[k] - s.ek[NT]) * Y[k];
    dT[0] = iC * (-V[3] * ir + (u * u + v * v) + sy);
    dT[1] = -iC * u;
    dT[2] = -iC * v;
    dT[3] = iC;
#pragma unroll
    for (int k = 0; k < NT; ++k) dT[4 + k] = -iC * (s.ek[k] - s.ek[NT]);
}

// Pressure, velocities and dp/dU of a state (detailed model: at its stored Newton T),
// optionally the sound speed and dc/dU, and dp/dQ (one-step model).
template <int NU>
struct PState {
    double u, v, p, c, dpQ;
    double dp[NU], dc[NU];
};

template <int M, int NU, bool SOUND>
__device__ __forceinline__ void pstate(const AdjGrid& g, CMech* m, const double (&V)[NU], double T,
                                       PState<NU>& P) {
    DevDomain D{};
    D.gamma = g.gamma;
    D.Q = g.Q;
    halo_prims<M, NU>(V, T, D, m, P.u, P.v, P.p);   // the forward's own formula
    const double rho = V[0], ir = 1.0 / rho;
    if constexpr (M == ONESTEP) {
        const double gm = g.gamma - 1.0;
        P.dp[0] = gm * 0.5 * (P.u * P.u + P.v * P.v);
        P.dp[1] = -gm * P.u;
        P.dp[2] = -gm * P.v;
        P.dp[3] = gm;
        P.dp[4] = -gm * g.Q;
        P.dpQ = -gm * V[4];
        if constexpr (SOUND) {
            P.c = sqrt(g.gamma * P.p * ir);
            const double kc = g.gamma / (2.0 * P.c * rho);
#pragma unroll
            for (int f = 0; f < NU; ++f) P.dc[f] = kc * P.dp[f];
            P.dc[0] -= kc * P.p * ir;
        }
    } else {
        constexpr int NS = NU - 3, NT = NS - 1;
        double Y[NS];
        mass_fractions<NU>(V, ir, Y);
        SpeciesAt<NS> s;
        species_at<NS>(m, Y, T, s);
        double dT[NU];
        temperature_grad<NU>(V, Y, s, dT);
        // p = T (sum_k<NT rho Y_k (R_k - R_last) + rho R_last) = T Rs
        const double Rl = m->Rk[NT];
        double Rs = V[0] * Rl;
#pragma unroll
        for (int k = 0; k < NT; ++k) Rs += V[4 + k] * (m->Rk[k] - Rl);
#pragma unroll
        for (int f = 0; f < NU; ++f) P.dp[f] = Rs * dT[f];
        P.dp[0] += T * Rl;
#pragma unroll
        for (int k = 0; k < NT; ++k) P.dp[4 + k] += T * (m->Rk[k] - Rl);
        P.dpQ = 0.0;
        if constexpr (SOUND) {
            // c^2 = gamma R T with gamma = 1 + R/c_v (R, c_v per mass)
            const double gam = 1.0 + s.Rm / s.cv;
            P.c = sqrt(gam * s.Rm * T);
            double dRm[NU], dcv[NU];
#pragma unroll
            for (int f = 0; f < NU; ++f) dRm[f] = dcv[f] = 0.0;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                // dY_k/d rho = -Y_k / rho, dY_k / d(rho Y_k) = 1 / rho
                const double dr = m->Rk[k] - Rl, dc = s.cvk[k] - s.cvk[NT];
                dRm[0] -= dr * Y[k] * ir;
                dcv[0] -= dc * Y[k] * ir;
                dRm[4 + k] = dr * ir;
                dcv[4 + k] = dc * ir;
            }
            const double i2c = 0.5 / P.c;
#pragma unroll
            for (int f = 0; f < NU; ++f) {
                const double dcvf = dcv[f] + s.dcv * dT[f];
                const double dgam = (dRm[f] * s.cv - s.Rm * dcvf) / (s.cv * s.cv);
                P.dc[f] = i2c * (dgam * s.Rm * T + gam * (dRm[f] * T + s.Rm * dT[f]));
            }
        }
    }
}

// Sound speed of a stored state as the forward's reductions formed it (detailed model:
// from the Newton T stored with the state, the forward's own mixture sums).
template <int M, int NU>
__device__ __forceinline__ void cell_speeds_of(const AdjGrid& g, CMech* m, const double* V, const double* VT,
                                               long long n, long long c, double& sx, double& sy) {
    double u[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) u[f] = V[(size_t)f * n + c];
    if constexpr (M == ONESTEP) {
        DevDomain D{};
        D.gamma = g.gamma;
        D.R = g.R;
        D.Q = g.Q;
        double T, cs, vx, vy;
        owner_state<ONESTEP, NU>(u, 0.0, D, nullptr, T, cs, vx, vy);
        sx = fabs(vx) + cs;
        sy = fabs(vy) + cs;
    } else {
        constexpr int NS = NU - 3;
        const double rho = u[0], ir = 1.0 / rho;
        const double vx = u[1] * ir, vy = u[2] * ir;
        double Y[NS];
        mass_fractions<NU>(u, ir, Y);
        MixNasa x;
        mix_nasa<NS>(Y, m, x);
        const double T = VT[c];
        double ec, cv;
        mix_eval(x, T, ec, cv);
        const double p = rho * x.Rmix * T;
        const double gam = (cv + x.Rmix) / cv;
        const double cs = sqrt(gam * p * ir);
        sx = fabs(vx) + cs;
        sy = fabs(vy) + cs;
    }
}

// Reverse of WENO5 (Jiang-Shu, eps = 1e-6) at output adjoint fb: adds dfhat/dv * fb.
__device__ __forceinline__ void weno5_adj(double a, double b, double c, double d, double e, double fb,
                                          double (&gr)[5]) {
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
    const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
    const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
    const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, u1 = b - d;
    const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
    const double s0 = WENO_EPS + ((13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0);
    const double s1 = WENO_EPS + ((13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1);
    const double s2 = WENO_EPS + ((13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2);
    const double al0 = 0.1 / (s0 * s0), al1 = 0.6 / (s1 * s1), al2 = 0.3 / (s2 * s2);
    const double S = al0 + al1 + al2;
    const double w0 = al0 / S, w1 = al1 / S, w2 = al2 / S;
    const double f = w0 * q0 + w1 * q1 + w2 * q2;
    const double qb0 = fb * w0, qb1 = fb * w1, qb2 = fb * w2;
    const double fs = fb / S;
    const double ab0 = fs * (q0 - f), ab1 = fs * (q1 - f), ab2 = fs * (q2 - f);
    const double bb0 = -2.0 * ab0 * al0 / s0, bb1 = -2.0 * ab1 * al1 / s1, bb2 = -2.0 * ab2 * al2 / s2;
    const double tb0 = bb0 * (13.0 / 6.0) * t0, ub0 = bb0 * 0.5 * u0;
    const double tb1 = bb1 * (13.0 / 6.0) * t1, ub1 = bb1 * 0.5 * u1;
    const double tb2 = bb2 * (13.0 / 6.0) * t2, ub2 = bb2 * 0.5 * u2;
    gr[0] = qb0 * (2.0 / 6.0) + tb0 + ub0;
    gr[1] = qb0 * (-7.0 / 6.0) - qb1 * (1.0 / 6.0) - 2.0 * tb0 - 4.0 * ub0 + tb1 + ub1;
    gr[2] = qb0 * (11.0 / 6.0) + qb1 * (5.0 / 6.0) + qb2 * (2.0 / 6.0) + tb0 + 3.0 * ub0 - 2.0 * tb1 +
            tb2 + 3.0 * ub2;
    gr[3] = qb1 * (2.0 / 6.0) + qb2 * (5.0 / 6.0) + tb1 - ub1 - 2.0 * tb2 - 4.0 * ub2;
    gr[4] = -qb2 * (1.0 / 6.0) + tb2 + ub2;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < AWG / 64; ++q) s += sh[q];
    return s;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double r = sh[0];
    for (int q = 1; q < AWG / 64; ++q) r = fmax(r, sh[q]);
    return r;
}

__device__ __forceinline__ int block_min(int v, int* sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    int r = sh[0];
    for (int q = 1; q < AWG / 64; ++q) r = min(r, sh[q]);
    return r;
}

// A: alpha_x, alpha_y of every stage input of a run of steps and the lowest
// cell attaining each: block maxima here, one workgroup per slice below.
template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_alpha(AlphaArgs P) {
    __shared__ double sh[8];
    __shared__ int ish[8];
    const int z = blockIdx.y;
    const double* V = P.base[z % 3] + (size_t)(z / 3) * P.step_stride;
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    double sx = -1.0, sy = -1.0;
    if (c < P.n) cell_speeds_of<M, NU>(P.g, cmech(P.mech), V, V + (size_t)NU * P.n, P.n, c, sx, sy);
    const double mx = block_max(sx, sh), my = block_max(sy, sh);
    const int ix = block_min((c < P.n && sx == mx) ? (int)c : 0x7fffffff, ish);
    const int iy = block_min((c < P.n && sy == my) ? (int)c : 0x7fffffff, ish);
    if (threadIdx.x == 0) {
        double* part = P.part + ((size_t)z * P.nbd + blockIdx.x) * 4;
        part[0] = mx;
        part[1] = my;
        part[2] = (double)ix;
        part[3] = (double)iy;
    }
}

// Split flux of component f at a stencil point (the forward's own formula).
template <int NU>
__device__ __forceinline__ void split_flux(const double (&V)[NU], double vn, double p, int f,
                                           bool xdir, double al, double& Fp, double& Fm) {
    double F = V[f] * vn;
    if (f == (xdir ? 1 : 2)) F += p;
    if (f == 3) F = (V[f] + p) * vn;
    Fp = 0.5 * (F + al * V[f]);
    Fm = 0.5 * (F - al * V[f]);
}

// B: per interface and component, mu_Fhat = b dt (mu_right - mu_left)/dx and
// the reverse of both WENO5 reconstructions; the six stencil states and their
// split fluxes are formed here from the stage input (component F = blockIdx.y). F is
// a run-time value, uniform over the workgroup: one body serves every component (a
// body per component made the kernel of the 12-field model copy its arguments to
// scratch memory, 304 bytes per lane, written by every thread at entry).
template <int M, int NU>
__device__ __forceinline__ void iface_component(const AdjArgs& A, int q, const int F) {
    const AdjGrid& g = A.g;
    const int nix = (g.nx + 1) * g.ny, niy = g.twod ? g.nx * (g.ny + 1) : 0;
    if (q >= nix + niy) return;
    const bool xdir = q < nix;
    int r, i0, j0, k, len, lidx;
    if (xdir) {
        r = q;
        j0 = q / (g.nx + 1);
        k = q - j0 * (g.nx + 1);
        i0 = k - 3;
        len = g.nx;
        lidx = j0 * g.nx + k;
    } else {
        r = q - nix;
        k = r / g.nx;
        i0 = r - k * g.nx;
        j0 = k - 3;
        len = g.ny;
        lidx = k * g.nx + i0;
    }
    const long long lstep = xdir ? 1 : g.nx;
    const double al = A.alpha[xdir ? 0 : 1];
    const double ih = xdir ? g.idx : g.idy;
    const double lr = A.lamW[(size_t)F * A.n + ((k < len) ? lidx : 0)];
    const double ll = A.lamW[(size_t)F * A.n + ((k > 0) ? lidx - lstep : 0)];
    const double mr = (k < len) ? lr : 0.0;
    const double ml = (k > 0) ? ll : 0.0;
    const double fb = A.b * A.dt * (mr - ml) * ih;
    // stencil points t = 0..5 at positions k-3 .. k+2 along the sweep
    DevDomain D{};
    D.gamma = g.gamma;
    D.Q = g.Q;
    double Fp[6], Fm[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        unsigned fl;
        const long long src = xdir ? usrc(g, i0 + t, j0, fl) : usrc(g, i0, j0 + t, fl);
        double V[NU], T, vx, vy, p;
        load_src<M, NU>(A, src, fl, V, T);
        halo_prims<M, NU>(V, T, D, cmech(A.mech), vx, vy, p);
        split_flux<NU>(V, xdir ? vx : vy, p, F, xdir, al, Fp[t], Fm[t]);
    }
    double gp[5], gm[5];
    weno5_adj(Fp[0], Fp[1], Fp[2], Fp[3], Fp[4], fb, gp);
    weno5_adj(Fm[5], Fm[4], Fm[3], Fm[2], Fm[1], fb, gm);
    const int ni = xdir ? nix : niy;
    double* out = (xdir ? A.cx : A.cy) + (size_t)F * 10 * ni;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        out[(size_t)m * ni + r] = gp[m];
        out[(size_t)(5 + m) * ni + r] = gm[4 - m];
    }
}

template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_iface(AdjArgs A) {
    const int q = blockIdx.x * AWG + threadIdx.x;
    iface_component<M, NU>(A, q, (int)blockIdx.y);
}

// Gather of the split-flux adjoints of strip position xi (x sweep: row j, xi in
// 0..nx+5) or yj (y sweep: column i, yj in 0..ny+5) from the 5 + 5 interfaces
// whose stencils read it.
template <int NU>
__device__ __forceinline__ void gather_strip(const AdjArgs& A, bool xdir, int i, int j, int xi,
                                             double (&mp)[NU], double (&mm)[NU]) {
    const AdjGrid& g = A.g;
    const int len = xdir ? g.nx : g.ny;
    const int ni = xdir ? (g.nx + 1) * g.ny : g.nx * (g.ny + 1);
#pragma unroll
    for (int f = 0; f < NU; ++f) {
        const double* cf = (xdir ? A.cx : A.cy) + (size_t)f * 10 * ni;
        double ap = 0.0, am = 0.0;
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            // loads at clamped interfaces, then a select: all ten are in flight together
            const int Ip = xi - m, Im = xi - 1 - m;
            const bool okp = Ip >= 0 && Ip <= len, okm = Im >= 0 && Im <= len;
            const int Ipc = okp ? Ip : 0, Imc = okm ? Im : 0;
            const int rp = xdir ? j * (g.nx + 1) + Ipc : Ipc * g.nx + i;
            const int rm = xdir ? j * (g.nx + 1) + Imc : Imc * g.nx + i;
            const double vp = cf[(size_t)m * ni + rp], vm = cf[(size_t)(5 + m) * ni + rm];
            ap += okp ? vp : 0.0;
            am += okm ? vm : 0.0;
        }
        mp[f] = ap;
        mm[f] = am;
    }
}

// Reverse of the split at one strip state V: flux Jacobian (rows: mass, normal and
// tangential momentum, energy, species) and the alpha term.
// out = adjoint of V; pal = d/dalpha part; pQ = d/dQ part.
template <int NU>
__device__ __forceinline__ void split_vjp(const double (&V)[NU], const PState<NU>& P, bool xdir,
                                          double al, const double (&mp)[NU], const double (&mm)[NU],
                                          double (&out)[NU], double& pal, double& pQ) {
    double a[NU], bq[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) {
        a[f] = 0.5 * (mp[f] + mm[f]);
        bq[f] = 0.5 * (mp[f] - mm[f]);
    }
    const double ir = 1.0 / V[0];
    const int nm = xdir ? 1 : 2, tm = xdir ? 2 : 1;
    // normal velocity w, tangential t
    const double w = xdir ? P.u : P.v, t = xdir ? P.v : P.u;
    const double a_nm = a[nm], a_tm = a[tm], a_E = a[3];
    double sr = 0.0;   // sum over the species rows of a_k (rho Y_k)
#pragma unroll
    for (int k = 4; k < NU; ++k) sr += a[k] * V[k];
    const double Ep = (V[3] + P.p) * ir;
    const double kp = a_nm + a_E * w;   // weight of dp/dV: normal momentum and energy rows
#pragma unroll
    for (int f = 0; f < NU; ++f) out[f] = kp * P.dp[f];
    out[0] += -a_nm * w * w - a_tm * w * t - a_E * Ep * w - sr * w * ir;
    out[nm] += a[0] + 2.0 * a_nm * w + a_tm * t + a_E * Ep + sr * ir;
    out[tm] += a_tm * w;
    out[3] += a_E * w;
#pragma unroll
    for (int k = 4; k < NU; ++k) out[k] += a[k] * w;
    pal = 0.0;
#pragma unroll
    for (int f = 0; f < NU; ++f) {
        out[f] += al * bq[f];
        pal += V[f] * bq[f];
    }
    pQ = kp * P.dpQ;
}

// The split-flux adjoints mp, mm gathered at a strip position, applied to the state
// there (the cell src, mirrored by fl, or a Dirichlet row): out (if add), the alpha
// and Q parts.
template <int M, int NU>
__device__ __forceinline__ void strip_apply(const AdjArgs& A, bool xdir, long long src, unsigned fl,
                                            const double (&Vc)[NU], double Tc, const double (&mp)[NU],
                                            const double (&mm)[NU], double (&out)[NU], bool add,
                                            double& pal, double& pQ) {
    const AdjGrid& g = A.g;
    double Vs[NU], Ts = Tc;
    if (src >= 0) {
#pragma unroll
        for (int f = 0; f < NU; ++f) Vs[f] = Vc[f];
        if (fl & 1u) Vs[1] = -Vs[1];
        if (fl & 2u) Vs[2] = -Vs[2];
    } else {
        const double* row = g.dirU + (size_t)(-src - 1) * (MAXF + 1);
#pragma unroll
        for (int f = 0; f < NU; ++f) Vs[f] = row[f];
        Ts = row[MAXF];
    }
    double o[NU], pa, pq;
    PState<NU> P;
    pstate<M, NU, false>(g, cmech(A.mech), Vs, Ts, P);
    split_vjp<NU>(Vs, P, xdir, A.alpha[xdir ? 0 : 1], mp, mm, o, pa, pq);
    if (M == ONESTEP && src < 0) {
        // Dirichlet ghost: its energy depends on Q through the chemical energy rho Y Q
        const double* row = g.dirU + (size_t)(-src - 1) * (MAXF + 1);
        pq += o[3] * row[4];
    }
    pal += pa;
    pQ += pq;
    if (add) {
#pragma unroll
        for (int f = 0; f < NU; ++f) {
            double v = o[f];
            if ((f == 1 && (fl & 1u)) || (f == 2 && (fl & 2u))) v = -v;
            out[f] += v;
        }
    }
}

// Adjoint of the cell's own strip position and its contributions.
template <int M, int NU>
__device__ __forceinline__ void strip_adjoint(const AdjArgs& A, bool xdir, int i, int j, int pos,
                                              long long src, unsigned fl, const double (&Vc)[NU],
                                              double Tc, double (&out)[NU], bool add, double& pal,
                                              double& pQ) {
    double mp[NU], mm[NU];
    gather_strip<NU>(A, xdir, i, j, pos, mp, mm);
    strip_apply<M, NU>(A, xdir, src, fl, Vc, Tc, mp, mm, out, add, pal, pQ);
}

// The ghost positions on one side (0: low, 1: high) of the cell's row (x sweep) or
// column (y sweep) that this cell owns: those whose source is the cell, or, on the first
// or last cell, the side's Dirichlet row. All of them have the same state (the same
// source and mirror flags, or the same row), and the reverse of the split is linear in
// the gathered adjoints, so their gathers are summed (in position order) and applied
// once: one state evaluation per side instead of one per position.
template <int M, int NU>
__device__ __forceinline__ void ghost_side(const AdjArgs& A, bool xdir, int i, int j, int side,
                                           long long c, const double (&Vc)[NU], double Tc,
                                           double (&out)[NU], double& pal, double& pQ) {
    const AdjGrid& g = A.g;
    const int len = xdir ? g.nx : g.ny;
    const int own = xdir ? i : j;
    double mp[NU], mm[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) mp[f] = mm[f] = 0.0;
    bool any = false;
    long long s0 = 0;
    unsigned f0 = 0u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int gp = (side == 0) ? -1 - k : len + k;
        unsigned fl;
        const long long s = xdir ? usrc(g, gp, j, fl) : usrc(g, i, gp, fl);
        const bool owner = (s == c) || (s < 0 && own == ((side == 0) ? 0 : len - 1));
        if (owner) {
            double ap[NU], am[NU];
            gather_strip<NU>(A, xdir, xdir ? gp : i, xdir ? j : gp, gp + 3, ap, am);
#pragma unroll
            for (int f = 0; f < NU; ++f) {
                mp[f] += ap[f];
                mm[f] += am[f];
            }
            any = true;
            s0 = s;
            f0 = fl;
        }
    }
    if (any) strip_apply<M, NU>(A, xdir, s0, f0, Vc, Tc, mp, mm, out, s0 == c, pal, pQ);
}

// C: per interior cell, the adjoint of the stage input: its own x and y strip
// positions, the ghost positions that copy or mirror it (and, on the first or
// last cell of a row or column, the Dirichlet ghosts of that side), the
// explicit Arrhenius source (one-step model) and the RK bookkeeping; per-block
// partials of the alpha, Q and Ea adjoints. Two threads per cell: the first half of
// the workgroup takes the x sweep, the second half the y sweep, and the y part
// reaches the cell's thread through LDS.
constexpr int CPB = AWG / 2;

template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_cell(AdjArgs A) {
    __shared__ double sh[8];
    __shared__ double ysum[NU][CPB];
    const int lc = threadIdx.x % CPB;
    const bool ydir = threadIdx.x >= CPB;
    const long long c = (long long)blockIdx.x * CPB + lc;
    const AdjGrid& g = A.g;
    double pax = 0.0, pay = 0.0, pQ = 0.0, pEa = 0.0;
    double V[NU], out[NU], Tc = 0.0;
#pragma unroll
    for (int f = 0; f < NU; ++f) out[f] = 0.0;
    const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
    if (c < A.n) {
#pragma unroll
        for (int f = 0; f < NU; ++f) V[f] = A.V[(size_t)f * A.n + c];
        if (M == DETAILED) Tc = A.VT[c];
        if (!ydir) {
#pragma unroll
            for (int f = 0; f < NU; ++f) out[f] = A.b * A.lamW[(size_t)f * A.n + c];
            strip_adjoint<M, NU>(A, true, i, j, i + 3, c, 0u, V, Tc, out, true, pax, pQ);
            if (i < 3 || i >= g.nx - 3) {
                ghost_side<M, NU>(A, true, i, j, 0, c, V, Tc, out, pax, pQ);
                ghost_side<M, NU>(A, true, i, j, 1, c, V, Tc, out, pax, pQ);
            }
        } else if (g.twod) {
            strip_adjoint<M, NU>(A, false, i, j, j + 3, c, 0u, V, Tc, out, true, pay, pQ);
            if (j < 3 || j >= g.ny - 3) {
                ghost_side<M, NU>(A, false, i, j, 0, c, V, Tc, out, pay, pQ);
                ghost_side<M, NU>(A, false, i, j, 1, c, V, Tc, out, pay, pQ);
            }
        }
    }
    if (ydir) {
#pragma unroll
        for (int f = 0; f < NU; ++f) ysum[f][lc] = out[f];
    }
    __syncthreads();
    if (!ydir && c < A.n) {
#pragma unroll
        for (int f = 0; f < NU; ++f) out[f] += ysum[f][lc];
        if constexpr (M == ONESTEP) {
            // explicit source S4 = -k r exp(-Ea/T), T = p/(rho R)
            PState<NU> P;
            pstate<M, NU, false>(g, nullptr, V, 0.0, P);
            const double mu4 = A.b * A.dt * A.lamW[(size_t)4 * A.n + c];
            const double T = P.p / (V[0] * g.R);
            const double ex = exp(-g.Ea / T);
            const double S = -g.k * V[4] * ex;
            const double dSdT = S * g.Ea / (T * T);
            const double iRr = 1.0 / (V[0] * g.R);
            double dT[NU];
#pragma unroll
            for (int f = 0; f < NU; ++f) dT[f] = P.dp[f] * iRr;
            dT[0] -= P.p / V[0] * iRr;
#pragma unroll
            for (int f = 0; f < NU; ++f) out[f] += mu4 * dSdT * dT[f];
            out[4] += mu4 * (-g.k * ex);
            pQ += mu4 * dSdT * (P.dpQ * iRr);
            pEa = mu4 * (-S / T);
        }
#pragma unroll
        for (int f = 0; f < NU; ++f) {
            A.lamOut[(size_t)f * A.n + c] = out[f];
            const double lw = A.a * A.lamW[(size_t)f * A.n + c];
            double acc = A.init_acc ? lw : A.acc[(size_t)f * A.n + c] + lw;
            if (A.add_out) acc += out[f];
            A.acc[(size_t)f * A.n + c] = acc;
        }
    }
    const double s0 = block_sum(pax, sh);
    const double s1 = block_sum(pay, sh);
    const double s2 = block_sum(pQ, sh);
    const double s3 = block_sum(pEa, sh);
    if (threadIdx.x == 0) {
        A.part[(size_t)blockIdx.x * 4 + 0] = s0;
        A.part[(size_t)blockIdx.x * 4 + 1] = s1;
        A.part[(size_t)blockIdx.x * 4 + 2] = s2;
        A.part[(size_t)blockIdx.x * 4 + 3] = s3;
    }
}

// D: one workgroup; the block partials summed in a fixed order, then the alpha
// adjoints at the argmax cells and, if asked, the loss seed of a state at the
// probes. Targets that share a cell are summed in target order and applied by
// one thread, so the result does not depend on thread timing.
constexpr int MAXT = 2 + MAXP;

template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_finish(AdjArgs A) {
    __shared__ double sh[4][AWG / 64];
    __shared__ double red[4];
    __shared__ double dlam[MAXT][NU], dacc[MAXT][NU], dth[MAXT];
    __shared__ long long tc[MAXT];
    __shared__ int uselam[MAXT];
    const AdjGrid& g = A.g;
    const int nal = g.twod ? 2 : 1;
    const int nsd = A.seedU ? A.np : 0;
    const int T = nal + nsd;
    const int k = threadIdx.x;
    // The state at the cell of this thread's task (an alpha term at its argmax cell, or a
    // probe's loss seed) does not depend on the block partials, and neither do the
    // adjoints there that the task adds to, nor theta: they are loaded first, so that
    // their latency overlaps the reduction. (Only this kernel writes them meanwhile, each
    // cell from one thread: the one whose own task cell it is.)
    long long cell = -1;
    double Vc[NU], lo[NU], ao[NU];
    double Tc = 0.0;
#pragma unroll
    for (int f = 0; f < NU; ++f) Vc[f] = lo[f] = ao[f] = 0.0;
    double th0 = 0.0, th1 = 0.0;
    if (k == 0) {
        th0 = A.theta[0];
        th1 = A.theta[1];
    }
    if (k < T) {
        if (k < nal) {
            const long long ca = A.argm[k];
            if (ca >= 0 && ca < A.n) cell = ca;   // (no cell attains the maximum only for non-finite data)
        } else {
            cell = A.pc[k - nal];
        }
        if (cell >= 0) {
            const double* src = (k < nal) ? A.V : A.seedU;
#pragma unroll
            for (int f = 0; f < NU; ++f) {
                Vc[f] = src[(size_t)f * A.n + cell];
                lo[f] = A.lamOut[(size_t)f * A.n + cell];
                ao[f] = A.acc[(size_t)f * A.n + cell];
            }
            if (M == DETAILED) Tc = (k < nal) ? A.VT[cell] : A.seedT[cell];
        }
    }
    // the four sums of the block partials in one pass: per wavefront by shuffles, then
    // the wavefronts' sums in order
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < A.nbd; q += AWG) {
#pragma unroll
        for (int j = 0; j < 4; ++j) s4[j] += A.part[(size_t)q * 4 + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s4[j] += __shfl_xor(s4[j], o, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int j = 0; j < 4; ++j) sh[j][threadIdx.x >> 6] = s4[j];
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int q = 0; q < AWG / 64; ++q) t += sh[threadIdx.x][q];
        red[threadIdx.x] = t;
    }
    __syncthreads();
    if (k < T) {
        double dl[NU], da[NU], th = 0.0;
        int ul = 0;
#pragma unroll
        for (int f = 0; f < NU; ++f) dl[f] = da[f] = 0.0;
        if (k < nal) {
            const int d = k;
            const double mua = red[d];
            if (cell >= 0) {
                PState<NU> P;
                pstate<M, NU, true>(g, cmech(A.mech), Vc, Tc, P);
                const double rho = Vc[0];
                const double w = d == 0 ? P.u : P.v;
                const double sg = (w > 0.0) ? 1.0 : ((w < 0.0) ? -1.0 : 0.0);
                double gr[NU];
#pragma unroll
                for (int f = 0; f < NU; ++f) gr[f] = P.dc[f];
                gr[0] -= sg * w / rho;
                gr[1 + d] += sg / rho;
#pragma unroll
                for (int f = 0; f < NU; ++f) {
                    dl[f] = mua * gr[f];
                    da[f] = A.add_out ? mua * gr[f] : 0.0;
                }
                ul = 1;
                if (M == ONESTEP) {
                    const double kc = g.gamma / (2.0 * P.c * rho);
                    th = mua * kc * P.dpQ;
                }
            }
        } else {
            // loss seed of the step start state: acc += dt w_q dp/dU at probe q
            const int q = k - nal;
            PState<NU> P;
            pstate<M, NU, false>(g, cmech(A.mech), Vc, Tc, P);
            const double s = A.dt * A.pw[q];
#pragma unroll
            for (int f = 0; f < NU; ++f) da[f] = s * P.dp[f];
            th = s * P.dpQ;
        }
        tc[k] = cell;
        uselam[k] = ul;
        dth[k] = th;
#pragma unroll
        for (int f = 0; f < NU; ++f) {
            dlam[k][f] = dl[f];
            dacc[k][f] = da[f];
        }
    }
    __syncthreads();
    if (k < T && tc[k] >= 0) {
        bool first = true;
        for (int q = 0; q < k; ++q) first = first && (tc[q] != tc[k]);
        if (first) {
            double sl[NU], sa[NU];
            int ul = 0;
#pragma unroll
            for (int f = 0; f < NU; ++f) sl[f] = sa[f] = 0.0;
            for (int q = k; q < T; ++q) {
                if (tc[q] != tc[k]) continue;
                ul |= uselam[q];
#pragma unroll
                for (int f = 0; f < NU; ++f) {
                    sl[f] += dlam[q][f];
                    sa[f] += dacc[q][f];
                }
            }
            const long long cc = tc[k];   // = cell, whose adjoints this thread loaded
#pragma unroll
            for (int f = 0; f < NU; ++f) {
                if (ul) A.lamOut[(size_t)f * A.n + cc] = lo[f] + sl[f];
                A.acc[(size_t)f * A.n + cc] = ao[f] + sa[f];
            }
        }
    }
    if (threadIdx.x == 0) {
        double sQ = red[2];
        for (int q = 0; q < T; ++q) sQ += dth[q];
        A.theta[0] = th0 + sQ;
        A.theta[1] = th1 + red[3];
    }
}

// ------------------------------------------------------------------ chemistry in reverse
// The reaction loops of the reversed chemistry step, the mechanism's structure read from
// its table: the rates, S and J = dS/d(rho Y) of the forward step (rates), and the
// reverse sweep that accumulates G = d/dX and GT = d/dT of mu . (dt S + dt J dU) (sweep).
// The run-time specialised kernel supplies the same two loops with the structure
// compiled in, the arithmetic unchanged.
template <int NS>
struct AdjReactions {
    static constexpr int NT = NS - 1;
    __device__ __forceinline__ void rates(CMech* m, const double (&X)[NS + 1], double lnT, double invT,
                                          double lnC, const double (&gts)[NS + 1], double (&S)[NT],
                                          double (&J)[NT][NT]) const {
        const int nr = m->nr;
        for (int i = 0; i < nr; ++i) {
            const double lnkf = m->lnA[i] + m->b[i] * lnT - m->EaR[i] * invT;
            const double kf = exp(lnkf);
            double kb = 0.0;
            if (m->rev[i]) {
                double sg = 0.0;
                for (int q = 0; q < MAXLIST; ++q) sg += gts[m->lb[i][q]] - gts[m->lf[i][q]];
                kb = exp(lnkf + sg - (double)m->dnsum[i] * lnC);
            }
            const int f0 = m->lf[i][0], f1 = m->lf[i][1], f2 = m->lf[i][2];
            const int r0 = m->lb[i][0], r1 = m->lb[i][1], r2 = m->lb[i][2];
            const double Rf = kf * (X[f0] * X[f1] * X[f2]), Rb = kb * (X[r0] * X[r1] * X[r2]);
            const bool tbr = m->has_tb[i] != 0;
            double ctb = 1.0;
            if (tbr) {
                ctb = 0.0;
#pragma unroll
                for (int j = 0; j < NS; ++j) ctb += m->tb[i][j] * X[j];
            }
            const double q = ctb * (Rf - Rb);
#pragma unroll
            for (int k = 0; k < NT; ++k) S[k] += m->Mdnu[i][k] * q;
            double dq[NS + 1];
#pragma unroll
            for (int j = 0; j <= NS; ++j) dq[j] = (tbr && j < NS) ? m->tb[i][j] * (Rf - Rb) : 0.0;
            dq[f0] += ctb * kf * (X[f1] * X[f2]);
            dq[f1] += ctb * kf * (X[f0] * X[f2]);
            dq[f2] += ctb * kf * (X[f0] * X[f1]);
            dq[r0] -= ctb * kb * (X[r1] * X[r2]);
            dq[r1] -= ctb * kb * (X[r0] * X[r2]);
            dq[r2] -= ctb * kb * (X[r0] * X[r1]);
            const double dl = dq[NT] * m->invM[NT];
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                const double ck = m->Mdnu[i][k];
                if (ck != 0.0) {
#pragma unroll
                    for (int q2 = 0; q2 < NT; ++q2) J[k][q2] += ck * (dq[q2] * m->invM[q2] - dl);
                }
            }
        }
    }
    __device__ __forceinline__ void sweep(CMech* m, const double (&X)[NS + 1], const double (&dX)[NS + 1],
                                          const double (&mu)[NT], double lnT, double invT, double lnC,
                                          const double (&gts)[NS + 1], const double (&hm1)[NS + 1],
                                          double (&G)[NS + 1], double& GT) const {
        const int nr = m->nr;
        for (int i = 0; i < nr; ++i) {
            double ci = 0.0;
#pragma unroll
            for (int k = 0; k < NT; ++k) ci += mu[k] * m->Mdnu[i][k];
            if (ci == 0.0) continue;
            const double lnkf = m->lnA[i] + m->b[i] * lnT - m->EaR[i] * invT;
            const double kf = exp(lnkf);
            double kb = 0.0, dlb = 0.0;
            const double dlf = (m->b[i] + m->EaR[i] * invT) * invT;   // d ln kf / dT
            if (m->rev[i]) {
                double sg = 0.0, sh = 0.0;
                for (int q = 0; q < MAXLIST; ++q) {
                    sg += gts[m->lb[i][q]] - gts[m->lf[i][q]];
                    sh += hm1[m->lb[i][q]] - hm1[m->lf[i][q]];
                }
                kb = exp(lnkf + sg - (double)m->dnsum[i] * lnC);
                dlb = dlf - sh * invT;                                  // d ln kb / dT
            }
            const int fs[3] = {m->lf[i][0], m->lf[i][1], m->lf[i][2]};
            const int bs[3] = {m->lb[i][0], m->lb[i][1], m->lb[i][2]};
            // R = k x0 x1 x2; dR/dx_s = k (product of the other two); dR . dX; its gradient
            auto prod = [&](const int (&sl)[3], double kk, double& R, double (&dR)[3], double& dRd,
                            double (&ddR)[3]) {
                const double x0 = X[sl[0]], x1 = X[sl[1]], x2 = X[sl[2]];
                const double e0 = dX[sl[0]], e1 = dX[sl[1]], e2 = dX[sl[2]];
                R = kk * (x0 * x1 * x2);
                dR[0] = kk * (x1 * x2);
                dR[1] = kk * (x0 * x2);
                dR[2] = kk * (x0 * x1);
                dRd = dR[0] * e0 + dR[1] * e1 + dR[2] * e2;
                ddR[0] = kk * (e1 * x2 + x1 * e2);
                ddR[1] = kk * (e0 * x2 + x0 * e2);
                ddR[2] = kk * (e0 * x1 + x0 * e1);
            };
            double Rf, dRf[3], dRfd, ddRf[3], Rb = 0.0, dRb[3] = {0.0, 0.0, 0.0}, dRbd = 0.0,
                   ddRb[3] = {0.0, 0.0, 0.0};
            prod(fs, kf, Rf, dRf, dRfd, ddRf);
            if (m->rev[i]) prod(bs, kb, Rb, dRb, dRbd, ddRb);
            const bool tbr = m->has_tb[i] != 0;
            double ctb = 1.0, dctb = 0.0;
            if (tbr) {
                ctb = 0.0;
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    ctb += m->tb[i][j] * X[j];
                    dctb += m->tb[i][j] * dX[j];
                }
            }
            // q = ctb (Rf - Rb); D = dq . dX = dctb (Rf - Rb) + ctb (dRf.dX - dRb.dX)
            const double net = Rf - Rb, dnet = dRfd - dRbd;
            if (tbr) {
#pragma unroll
                for (int j = 0; j < NS; ++j) G[j] += ci * m->tb[i][j] * (net + dnet);
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                G[fs[s]] += ci * ((ctb + dctb) * dRf[s] + ctb * ddRf[s]);
                G[bs[s]] -= ci * ((ctb + dctb) * dRb[s] + ctb * ddRb[s]);
            }
            GT += ci * ((ctb + dctb) * (Rf * dlf - Rb * dlb) + ctb * (dRfd * dlf - dRbd * dlb));
        }
    }
};

// One cell per thread. The forward step is recomputed in registers (rates, the
// Jacobian at frozen T and rho, the pivoted LU of I - dt J, the increment dU); then
// mu = (I - dt J)^-T lambda_{rho Y}, c_i = sum_k mu_k M_k dnu_ik per reaction, and
// with dX the concentration change of dU:
//   d/dX_l  += dt sum_i c_i (dq_i/dX_l + d(dq_i . dX)/dX_l)
//   d/dT    += dt sum_i c_i (dq_i/dT + d(dq_i . dX)/dT)
// then X -> (rho Y, rho) and T -> U* by the implicit-function theorem.
template <int NS, class Reactions>
__device__ __forceinline__ void adj_chem_cell(const AdjChemArgs& A, const Reactions& rx) {
    constexpr int NT = NS - 1, NU = NS + 3;
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    if (c >= A.n) return;
    CMech* m = cmech(A.mech);
    double V[NU], lam[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) {
        V[f] = A.Ustar[(size_t)f * A.n + c];
        lam[f] = A.lamIn[(size_t)f * A.n + c];
    }
    const double T = A.Tstar[c], dt = A.dt;
    const double rho = V[0];
    // concentrations (the padding slot NS of the molecule lists holds 1)
    double X[NS + 1];
    double sr = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        X[j] = V[4 + j] * m->invM[j];
        sr += V[4 + j];
    }
    X[NT] = (rho - sr) * m->invM[NT];
    X[NS] = 1.0;
    const double lnT = log(T), invT = 1.0 / T;
    const double lnC = log(PATM / RU) - lnT;
    double gts[NS + 1], hm1[NS + 1];   // h/(R T) - s/R and h/(R T) - 1 per species
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const bool hi = m->two_range && T >= m->tmid[j];
        double a[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) a[q] = hi ? m->nasa_hi[j][q] : m->nasa[j][q];
        const double hRT = a[0] + T * (0.5 * a[1] + T * (a[2] * (1.0 / 3.0) + T * (0.25 * a[3] + T * (0.2 * a[4])))) +
                           a[5] * invT;
        const double sR = a[0] * lnT + T * (a[1] + T * (0.5 * a[2] + T * (a[3] * (1.0 / 3.0) + T * (0.25 * a[4])))) + a[6];
        gts[j] = hRT - sR;
        hm1[j] = hRT - 1.0;
    }
    gts[NS] = hm1[NS] = 0.0;
    // forward: rates, J, the step
    double S[NT], J[NT][NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        S[k] = 0.0;
#pragma unroll
        for (int q = 0; q < NT; ++q) J[k][q] = 0.0;
    }
    rx.rates(m, X, lnT, invT, lnC, gts, S, J);
    // P (I - dt J) = L U, rows exchanged whole; L below the diagonal (unit diagonal)
    int piv[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
#pragma unroll
        for (int q = 0; q < NT; ++q) J[k][q] = (k == q ? 1.0 : 0.0) - dt * J[k][q];
    }
    unsigned st = 0u;
#pragma unroll
    for (int col = 0; col < NT; ++col) {
        int p = col;
        double amax = fabs(J[col][col]);
#pragma unroll
        for (int r = col + 1; r < NT; ++r) {
            const double ar = fabs(J[r][col]);
            if (ar > amax) { amax = ar; p = r; }
        }
        piv[col] = p;
        if (__any(p != col)) {   // row exchange by selects, where some cell needs one
#pragma unroll
            for (int r = col + 1; r < NT; ++r) {
                const bool sw = (r == p);
#pragma unroll
                for (int q = 0; q < NT; ++q) {
                    const double top = J[col][q], row = J[r][q];
                    J[col][q] = sw ? row : top;
                    J[r][q] = sw ? top : row;
                }
            }
        }
        const double pv = J[col][col];
        if (!(fabs(pv) > 0.0) || !isfinite(pv)) st |= STB_NONFINITE;
        const double ip = 1.0 / pv;
#pragma unroll
        for (int r = col + 1; r < NT; ++r) {
            const double fct = J[r][col] * ip;
            J[r][col] = fct;
#pragma unroll
            for (int q = col + 1; q < NT; ++q) J[r][q] -= fct * J[col][q];
        }
    }
    // dU = (I - dt J)^-1 dt S: permute, forward (L), backward (U)
    double x[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) x[k] = dt * S[k];
#pragma unroll
    for (int col = 0; col < NT; ++col) {
#pragma unroll
        for (int r = col + 1; r < NT; ++r) {
            const bool sw = (r == piv[col]);
            const double a0 = x[col], a1 = x[r];
            x[col] = sw ? a1 : a0;
            x[r] = sw ? a0 : a1;
        }
    }
#pragma unroll
    for (int r = 0; r < NT; ++r) {
#pragma unroll
        for (int q = 0; q < r; ++q) x[r] -= J[r][q] * x[q];
    }
#pragma unroll
    for (int r = NT - 1; r >= 0; --r) {
#pragma unroll
        for (int q = r + 1; q < NT; ++q) x[r] -= J[r][q] * x[q];
        x[r] = x[r] / J[r][r];
    }
    // mu = A^-T lambda: U^T z = lambda, L^T y = z, mu = P^T y
    double mu[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) mu[k] = lam[4 + k];
#pragma unroll
    for (int r = 0; r < NT; ++r) {
#pragma unroll
        for (int q = 0; q < r; ++q) mu[r] -= J[q][r] * mu[q];
        mu[r] = mu[r] / J[r][r];
    }
#pragma unroll
    for (int r = NT - 1; r >= 0; --r) {
#pragma unroll
        for (int q = r + 1; q < NT; ++q) mu[r] -= J[q][r] * mu[q];
    }
#pragma unroll
    for (int col = NT - 1; col >= 0; --col) {
#pragma unroll
        for (int r = col + 1; r < NT; ++r) {
            const bool sw = (r == piv[col]);
            const double a0 = mu[col], a1 = mu[r];
            mu[col] = sw ? a1 : a0;
            mu[r] = sw ? a0 : a1;
        }
    }
    // concentration change of the step (padding slot: none)
    double dX[NS + 1];
    double sd = 0.0;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        dX[j] = x[j] * m->invM[j];
        sd += x[j];
    }
    dX[NT] = -sd * m->invM[NT];
    dX[NS] = 0.0;
    // reverse sweep over the reactions
    double G[NS + 1], GT = 0.0;
#pragma unroll
    for (int j = 0; j <= NS; ++j) G[j] = 0.0;
    rx.sweep(m, X, dX, mu, lnT, invT, lnC, gts, hm1, G, GT);
    // X_j = rho Y_j / M_j (j < NT), X_last = (rho - sum rho Y) / M_last
    double out[NU];
#pragma unroll
    for (int f = 0; f < NU; ++f) out[f] = lam[f];
    const double gl = dt * G[NT] * m->invM[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) out[4 + k] += dt * G[k] * m->invM[k] - gl;
    out[0] += gl;
    // T* = T(U*): implicit-function theorem
    {
        const double ir = 1.0 / rho;
        double Y[NS];
        mass_fractions<NU>(V, ir, Y);
        SpeciesAt<NS> sp;
        species_at<NS>(m, Y, T, sp);
        double dT[NU];
        temperature_grad<NU>(V, Y, sp, dT);
#pragma unroll
        for (int f = 0; f < NU; ++f) out[f] += dt * GT * dT[f];
    }
#pragma unroll
    for (int f = 0; f < NU; ++f) A.lamOut[(size_t)f * A.n + c] = out[f];
    if (st) atomicOr(A.status, st);
}

template <int NS>
__global__ __launch_bounds__(AWG) void adj_chem(AdjChemArgs A) {
    adj_chem_cell<NS>(A, AdjReactions<NS>{});
}

// Loss terms of a run of states: term[n0 + m - 1] = dt sum_q w_q p(U_m at cell_q)
// for the states U_m = base + m * stride, m = 1 .. count - 1, then `last` (if not
// null) as m = count. The terms are summed in step order at the end, so the loss
// does not depend on how the run was cut into segments.
template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_loss(AdjGrid g, const DevMech* mech, const double* base,
                                                long long stride, int count, const double* last,
                                                int n0, long long n, const int* pc, const double* pw,
                                                int np, double dt, double* term) {
    const int ns = (count - 1) + (last ? 1 : 0);
    const int si = blockIdx.x * AWG + threadIdx.x;
    if (si >= ns) return;
    const double* U = (si < count - 1) ? base + (size_t)(si + 1) * stride : last;
    double acc = 0.0;
    DevDomain D{};
    D.gamma = g.gamma;
    D.Q = g.Q;
    for (int q = 0; q < np; ++q) {
        double V[NU];
        for (int f = 0; f < NU; ++f) V[f] = U[(size_t)f * n + pc[q]];
        const double T = (M == DETAILED) ? U[(size_t)NU * n + pc[q]] : 0.0;
        double vx, vy, p;
        halo_prims<M, NU>(V, T, D, cmech(mech), vx, vy, p);
        acc += pw[q] * p;
    }
    term[n0 + si] = dt * acc;
}

// Loss seed of one state: lambda += dt sum_q w_q dp/dU at the probes, theta_Q += dt w_q dp/dQ.
template <int M, int NU>
__global__ void adj_seed(AdjGrid g, const DevMech* mech, const double* U, long long n, const int* pc,
                         const double* pw, int np, double dt, double* lam, double* theta) {
    if (threadIdx.x != 0) return;
    for (int q = 0; q < np; ++q) {
        double V[NU];
        for (int f = 0; f < NU; ++f) V[f] = U[(size_t)f * n + pc[q]];
        const double T = (M == DETAILED) ? U[(size_t)NU * n + pc[q]] : 0.0;
        PState<NU> P;
        pstate<M, NU, false>(g, cmech(mech), V, T, P);
        const double s = dt * pw[q];
        for (int f = 0; f < NU; ++f) lam[(size_t)f * n + pc[q]] += s * P.dp[f];
        theta[0] += s * P.dpQ;
    }
}

// dL/dW0 from dL/dU0 through U0 = cons(W0); the one-step model's Q part to partials.
//   one-step: W = [rho, u, v, p, Y], E = p/(gamma-1) + rho |u|^2/2 + rho Y Q;
//   detailed: W = [p, u, v, T, Y_1..Y_{Ns-1}], rho = p/(R T), E = rho e(T, Y) + rho |u|^2/2.
template <int M, int NU>
__global__ __launch_bounds__(AWG) void adj_chain_ic(AdjGrid g, const DevMech* mech, const double* W,
                                                    const double* lam, long long n, double* gW,
                                                    double* part) {
    __shared__ double sh[8];
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    double pq = 0.0;
    if (c < n) {
        if constexpr (M == ONESTEP) {
            const double rho = W[c], u = W[n + c], v = W[2 * n + c], Y = W[4 * n + c];
            const double l0 = lam[c], l1 = lam[n + c], l2 = lam[2 * n + c], l3 = lam[3 * n + c],
                         l4 = lam[4 * n + c];
            gW[c] = l0 + l1 * u + l2 * v + l3 * (0.5 * (u * u + v * v) + Y * g.Q) + l4 * Y;
            gW[n + c] = l1 * rho + l3 * rho * u;
            gW[2 * n + c] = l2 * rho + l3 * rho * v;
            gW[3 * n + c] = l3 / (g.gamma - 1.0);
            gW[4 * n + c] = l3 * rho * g.Q + l4 * rho;
            pq = l3 * rho * Y;
        } else {
            constexpr int NS = NU - 3, NT = NS - 1;
            CMech* m = cmech(mech);
            const double p = W[c], u = W[n + c], v = W[2 * n + c], T = W[3 * n + c];
            double Y[NS], s = 0.0;
#pragma unroll
            for (int k = 0; k < NT; ++k) {
                Y[k] = W[(size_t)(4 + k) * n + c];
                s += Y[k];
            }
            Y[NT] = 1.0 - s;
            SpeciesAt<NS> sp;
            species_at<NS>(m, Y, T, sp);
            double e = 0.0;
#pragma unroll
            for (int k = 0; k < NS; ++k) e += Y[k] * sp.ek[k];
            const double rho = p / (sp.Rm * T);
            double l[NU];
#pragma unroll
            for (int f = 0; f < NU; ++f) l[f] = lam[(size_t)f * n + c];
            // d/d rho at fixed (u, v, e, Y)
            double lr = l[0] + l[1] * u + l[2] * v + l[3] * (e + 0.5 * (u * u + v * v));
#pragma unroll
            for (int k = 0; k < NT; ++k) lr += l[4 + k] * Y[k];
            const double Rl = m->Rk[NT];
            gW[c] = lr * rho / p;
            gW[n + c] = l[1] * rho + l[3] * rho * u;
            gW[2 * n + c] = l[2] * rho + l[3] * rho * v;
            gW[3 * n + c] = -lr * rho / T + l[3] * rho * sp.cv;
#pragma unroll
            for (int k = 0; k < NT; ++k)
                gW[(size_t)(4 + k) * n + c] = -lr * rho * (m->Rk[k] - Rl) / sp.Rm +
                                              l[3] * rho * (sp.ek[k] - sp.ek[NT]) + l[4 + k] * rho;
        }
    }
    const double sum = block_sum(pq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

}  // namespace janc
