// janc_adjoint.hip -- hand-written discrete adjoint of one SSP-RK3 step of the
// one-step detonation model on a uniform grid (the adjoint method of paper
// Sec. 6.1, Eq. 6.1-6.5, applied to the discrete trajectory: the result is the
// exact gradient of the discrete forward map).
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
//      source, the RK bookkeeping, block partials of d/dalpha, d/dQ, d/dEa;
//   D  one workgroup: the partials summed in a fixed order, the alpha adjoints
//      applied at the argmax cells, theta, and the loss seed of the step start.
// Every thread issues its loads together (clamped indices, masked afterwards):
// the small grids of an adjoint run are bound by memory latency, not bandwidth.
#include "janc_device.h"

namespace janc {

constexpr int NU5 = 5;
constexpr int AWG = 256;


// Source of grid position (i, j) (one coordinate may lie in the 3 ghost layers).
__device__ long long usrc(const AdjGrid& g, int i, int j, unsigned& fl) {
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
__device__ __forceinline__ void load_src(const AdjArgs& A, long long s, unsigned fl, double (&u)[NU5]) {
    const long long sc = s >= 0 ? s : 0;
#pragma unroll
    for (int f = 0; f < NU5; ++f) u[f] = A.V[(size_t)f * A.n + sc];
    if (s < 0) {
        const double* r = A.g.dirU + (size_t)(-s - 1) * (MAXF + 1);
#pragma unroll
        for (int f = 0; f < NU5; ++f) u[f] = r[f];
    }
    if (fl & 1u) u[1] = -u[1];
    if (fl & 2u) u[2] = -u[2];
}

// Pressure and its partial derivatives for the one-step equation of state,
// p = (gamma-1) (E - (m^2 + n^2)/(2 rho) - r Q), in terms of V = [rho, m, n, E, r].
struct PGrad {
    double u, v, p, pr, pm, pn, pE, pY, pQ;
};

__device__ __forceinline__ PGrad pgrad(const AdjGrid& g, const double (&V)[NU5]) {
    PGrad q;
    DevDomain D{};
    D.gamma = g.gamma;
    D.Q = g.Q;
    halo_prims<ONESTEP, NU5>(V, 0.0, D, nullptr, q.u, q.v, q.p);   // the forward's own formula
    const double gm = g.gamma - 1.0;
    q.pr = gm * 0.5 * (q.u * q.u + q.v * q.v);
    q.pm = -gm * q.u;
    q.pn = -gm * q.v;
    q.pE = gm;
    q.pY = -gm * g.Q;
    q.pQ = -gm * V[4];
    return q;
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

// Wave speeds of a cell of state V as the forward reductions compute them.
__device__ __forceinline__ void cell_speeds_of(const AdjGrid& g, const double* V, long long n,
                                               long long c, double& sx, double& sy) {
    double u[NU5];
#pragma unroll
    for (int f = 0; f < NU5; ++f) u[f] = V[(size_t)f * n + c];
    DevDomain D{};
    D.gamma = g.gamma;
    D.R = g.R;
    D.Q = g.Q;
    double T, cs, vx, vy;
    owner_state<ONESTEP, NU5>(u, 0.0, D, nullptr, T, cs, vx, vy);
    sx = fabs(vx) + cs;
    sy = fabs(vy) + cs;
}

// A: alpha_x, alpha_y of every stage input of a run of steps and the lowest
// cell attaining each: block maxima here, one workgroup per slice below.
__global__ __launch_bounds__(AWG) void adj_alpha(AlphaArgs P) {
    __shared__ double sh[8];
    __shared__ int ish[8];
    const int z = blockIdx.y;
    const double* V = P.base[z % 3] + (size_t)(z / 3) * P.step_stride;
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    double sx = -1.0, sy = -1.0;
    if (c < P.n) cell_speeds_of(P.g, V, P.n, c, sx, sy);
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

__global__ __launch_bounds__(AWG) void adj_alpha_reduce(AlphaArgs P) {
    __shared__ double sh[8];
    __shared__ int ish[8];
    const int z = blockIdx.x;
    const double* part = P.part + (size_t)z * P.nbd * 4;
    double bx = -1.0, by = -1.0;
    for (int q = threadIdx.x; q < P.nbd; q += AWG) {
        bx = fmax(bx, part[(size_t)q * 4 + 0]);
        by = fmax(by, part[(size_t)q * 4 + 1]);
    }
    const double gx = block_max(bx, sh), gy = block_max(by, sh);
    int jx = 0x7fffffff, jy = 0x7fffffff;
    for (int q = threadIdx.x; q < P.nbd; q += AWG) {
        if (part[(size_t)q * 4 + 0] == gx) jx = min(jx, (int)part[(size_t)q * 4 + 2]);
        if (part[(size_t)q * 4 + 1] == gy) jy = min(jy, (int)part[(size_t)q * 4 + 3]);
    }
    jx = block_min(jx, ish);
    jy = block_min(jy, ish);
    if (threadIdx.x == 0) {
        P.alpha[2 * z] = gx;
        P.alpha[2 * z + 1] = gy;
        P.argm[2 * z] = jx;
        P.argm[2 * z + 1] = jy;
    }
}

// Split flux of component f at a stencil point (the forward's own formula).
__device__ __forceinline__ void split_flux(const double (&V)[NU5], double vn, double p, int f,
                                           bool xdir, double al, double& Fp, double& Fm) {
    double F = V[f] * vn;
    if (f == (xdir ? 1 : 2)) F += p;
    if (f == 3) F = (V[f] + p) * vn;
    Fp = 0.5 * (F + al * V[f]);
    Fm = 0.5 * (F - al * V[f]);
}

// B: per interface and component, mu_Fhat = b dt (mu_right - mu_left)/dx and
// the reverse of both WENO5 reconstructions; the six stencil states and their
// split fluxes are formed here from the stage input (component = blockIdx.y).
template <int F>
__device__ __forceinline__ void iface_component(const AdjArgs& A, int q) {
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
        double V[NU5], vx, vy, p;
        load_src(A, src, fl, V);
        halo_prims<ONESTEP, NU5>(V, 0.0, D, nullptr, vx, vy, p);
        split_flux(V, xdir ? vx : vy, p, F, xdir, al, Fp[t], Fm[t]);
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

__global__ __launch_bounds__(AWG) void adj_iface(AdjArgs A) {
    const int q = blockIdx.x * AWG + threadIdx.x;
    switch (blockIdx.y) {
        case 0: iface_component<0>(A, q); break;
        case 1: iface_component<1>(A, q); break;
        case 2: iface_component<2>(A, q); break;
        case 3: iface_component<3>(A, q); break;
        default: iface_component<4>(A, q); break;
    }
}

// Gather of the split-flux adjoints of strip position xi (x sweep: row j, xi in
// 0..nx+5) or yj (y sweep: column i, yj in 0..ny+5) from the 5 + 5 interfaces
// whose stencils read it.
__device__ __forceinline__ void gather_strip(const AdjArgs& A, bool xdir, int i, int j, int xi,
                                             double (&mp)[NU5], double (&mm)[NU5]) {
    const AdjGrid& g = A.g;
    const int len = xdir ? g.nx : g.ny;
    const int ni = xdir ? (g.nx + 1) * g.ny : g.nx * (g.ny + 1);
#pragma unroll
    for (int f = 0; f < NU5; ++f) {
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

// Reverse of the split at one strip state V: flux Jacobian and the alpha term.
// out = adjoint of V; pal = d/dalpha part; pQ = d/dQ part.
__device__ __forceinline__ void split_vjp(const AdjGrid& g, const double (&V)[NU5], bool xdir,
                                          double al, const double (&mp)[NU5],
                                          const double (&mm)[NU5], double (&out)[NU5],
                                          double& pal, double& pQ) {
    const PGrad P = pgrad(g, V);
    double a[NU5], bq[NU5];
#pragma unroll
    for (int f = 0; f < NU5; ++f) {
        a[f] = 0.5 * (mp[f] + mm[f]);
        bq[f] = 0.5 * (mp[f] - mm[f]);
    }
    const double rho = V[0], E = V[3], r = V[4];
    const double ir = 1.0 / rho;
    // normal velocity w, tangential t; normal momentum index nm, tangential tm
    const double w = xdir ? P.u : P.v, t = xdir ? P.v : P.u;
    const double pw = xdir ? P.pm : P.pn, pt = xdir ? P.pn : P.pm;
    // flux components: mass, normal momentum, tangential momentum, energy, species
    const double a_mass = a[0], a_nm = a[xdir ? 1 : 2], a_tm = a[xdir ? 2 : 1];
    const double a_E = a[3], a_r = a[4];
    const double d_rho = a_nm * (-w * w + P.pr) + a_tm * (-w * t) +
                         a_E * (-w * (E + P.p) * ir + w * P.pr) + a_r * (-r * w * ir);
    const double d_nm = a_mass + a_nm * (2.0 * w + pw) + a_tm * t + a_E * ((E + P.p) * ir + w * pw) +
                        a_r * (r * ir);
    const double d_tm = a_nm * pt + a_tm * w + a_E * w * pt;
    const double d_E = a_nm * P.pE + a_E * w * (1.0 + P.pE);
    const double d_r = a_nm * P.pY + a_E * w * P.pY + a_r * w;
    out[0] = d_rho;
    out[xdir ? 1 : 2] = d_nm;
    out[xdir ? 2 : 1] = d_tm;
    out[3] = d_E;
    out[4] = d_r;
    pal = 0.0;
#pragma unroll
    for (int f = 0; f < NU5; ++f) {
        out[f] += al * bq[f];
        pal += V[f] * bq[f];
    }
    pQ = a_nm * P.pQ + a_E * w * P.pQ;
}

// Adjoint of one strip position (own or ghost) and its contributions.
__device__ __forceinline__ void strip_adjoint(const AdjArgs& A, bool xdir, int i, int j, int pos,
                                              long long src, unsigned fl, const double (&Vc)[NU5],
                                              double (&out)[NU5], bool add, double& pal,
                                              double& pQ) {
    const AdjGrid& g = A.g;
    double Vs[NU5];
    if (src >= 0) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) Vs[f] = Vc[f];
        if (fl & 1u) Vs[1] = -Vs[1];
        if (fl & 2u) Vs[2] = -Vs[2];
    } else {
        const double* row = g.dirU + (size_t)(-src - 1) * (MAXF + 1);
#pragma unroll
        for (int f = 0; f < NU5; ++f) Vs[f] = row[f];
    }
    double mp[NU5], mm[NU5], o[NU5], pa, pq;
    gather_strip(A, xdir, i, j, pos, mp, mm);
    split_vjp(g, Vs, xdir, A.alpha[xdir ? 0 : 1], mp, mm, o, pa, pq);
    if (src < 0) {
        // Dirichlet ghost: its energy depends on Q through the chemical energy rho Y Q
        const double* row = g.dirU + (size_t)(-src - 1) * (MAXF + 1);
        pq += o[3] * row[4];
    }
    pal += pa;
    pQ += pq;
    if (add) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
            double v = o[f];
            if ((f == 1 && (fl & 1u)) || (f == 2 && (fl & 2u))) v = -v;
            out[f] += v;
        }
    }
}

// C: per interior cell, the adjoint of the stage input: its own x and y strip
// positions, the ghost positions that copy or mirror it (and, on the first or
// last cell of a row or column, the Dirichlet ghosts of that side), the
// explicit Arrhenius source and the RK bookkeeping; per-block partials of the
// alpha, Q and Ea adjoints. Two threads per cell: the first half of the
// workgroup takes the x sweep, the second half the y sweep, and the y part
// reaches the cell's thread through LDS.
constexpr int CPB = AWG / 2;

__global__ __launch_bounds__(AWG) void adj_cell(AdjArgs A) {
    __shared__ double sh[8];
    __shared__ double ysum[NU5][CPB];
    const int lc = threadIdx.x % CPB;
    const bool ydir = threadIdx.x >= CPB;
    const long long c = (long long)blockIdx.x * CPB + lc;
    const AdjGrid& g = A.g;
    double pax = 0.0, pay = 0.0, pQ = 0.0, pEa = 0.0;
    double V[NU5], out[NU5];
#pragma unroll
    for (int f = 0; f < NU5; ++f) out[f] = 0.0;
    const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
    if (c < A.n) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) V[f] = A.V[(size_t)f * A.n + c];
        if (!ydir) {
#pragma unroll
            for (int f = 0; f < NU5; ++f) out[f] = A.b * A.lamW[(size_t)f * A.n + c];
            strip_adjoint(A, true, i, j, i + 3, c, 0u, V, out, true, pax, pQ);
            if (i < 3 || i >= g.nx - 3) {
                for (int gq = 0; gq < 6; ++gq) {
                    const int gi = (gq < 3) ? -1 - gq : g.nx + gq - 3;
                    unsigned fl;
                    const long long s = usrc(g, gi, j, fl);
                    const bool owner = (s == c) || (s < 0 && i == ((gq < 3) ? 0 : g.nx - 1));
                    if (owner) strip_adjoint(A, true, gi, j, gi + 3, s, fl, V, out, s == c, pax, pQ);
                }
            }
        } else if (g.twod) {
            strip_adjoint(A, false, i, j, j + 3, c, 0u, V, out, true, pay, pQ);
            if (j < 3 || j >= g.ny - 3) {
                for (int gq = 0; gq < 6; ++gq) {
                    const int gj = (gq < 3) ? -1 - gq : g.ny + gq - 3;
                    unsigned fl;
                    const long long s = usrc(g, i, gj, fl);
                    const bool owner = (s == c) || (s < 0 && j == ((gq < 3) ? 0 : g.ny - 1));
                    if (owner) strip_adjoint(A, false, i, gj, gj + 3, s, fl, V, out, s == c, pay, pQ);
                }
            }
        }
    }
    if (ydir) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) ysum[f][lc] = out[f];
    }
    __syncthreads();
    if (!ydir && c < A.n) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) out[f] += ysum[f][lc];
        // explicit source S4 = -k r exp(-Ea/T), T = p/(rho R)
        const PGrad P = pgrad(g, V);
        const double mu4 = A.b * A.dt * A.lamW[(size_t)4 * A.n + c];
        const double T = P.p / (V[0] * g.R);
        const double ex = exp(-g.Ea / T);
        const double S = -g.k * V[4] * ex;
        const double dSdT = S * g.Ea / (T * T);
        const double iRr = 1.0 / (V[0] * g.R);
        const double dT[NU5] = {(P.pr - P.p / V[0]) * iRr, P.pm * iRr, P.pn * iRr, P.pE * iRr, P.pY * iRr};
#pragma unroll
        for (int f = 0; f < NU5; ++f) out[f] += mu4 * dSdT * dT[f];
        out[4] += mu4 * (-g.k * ex);
        pQ += mu4 * dSdT * (P.pQ * iRr);
        pEa = mu4 * (-S / T);
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
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

__global__ __launch_bounds__(AWG) void adj_finish(AdjArgs A) {
    __shared__ double sh[8];
    __shared__ double red[4];
    __shared__ double dlam[MAXT][NU5], dacc[MAXT][NU5], dth[MAXT];
    __shared__ long long tc[MAXT];
    __shared__ int uselam[MAXT];
    const AdjGrid& g = A.g;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = threadIdx.x; q < A.nbd; q += AWG) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s4[k] += A.part[(size_t)q * 4 + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = block_sum(s4[k], sh);
        if (threadIdx.x == 0) red[k] = t;
    }
    __syncthreads();
    const int nal = g.twod ? 2 : 1;
    const int nsd = A.seedU ? A.np : 0;
    const int T = nal + nsd;
    const int k = threadIdx.x;
    if (k < T) {
        long long cell = -1;
        double dl[NU5], da[NU5], th = 0.0;
        int ul = 0;
#pragma unroll
        for (int f = 0; f < NU5; ++f) dl[f] = da[f] = 0.0;
        if (k < nal) {
            const int d = k;
            const double mua = red[d];
            const long long ca = A.argm[d];
            if (ca >= 0 && ca < A.n) {   // (no cell attains the maximum only for non-finite data)
                cell = ca;
                double Vc[NU5];
#pragma unroll
                for (int f = 0; f < NU5; ++f) Vc[f] = A.V[(size_t)f * A.n + ca];
                const PGrad P = pgrad(g, Vc);
                const double rho = Vc[0];
                const double cs = sqrt(g.gamma * P.p / rho);
                const double w = d == 0 ? P.u : P.v;
                const double sg = (w > 0.0) ? 1.0 : ((w < 0.0) ? -1.0 : 0.0);
                const double kc = g.gamma / (2.0 * cs * rho);
                double gr[NU5];
                gr[0] = kc * (P.pr - P.p / rho) - sg * w / rho;
                gr[1] = kc * P.pm + (d == 0 ? sg / rho : 0.0);
                gr[2] = kc * P.pn + (d == 1 ? sg / rho : 0.0);
                gr[3] = kc * P.pE;
                gr[4] = kc * P.pY;
#pragma unroll
                for (int f = 0; f < NU5; ++f) {
                    dl[f] = mua * gr[f];
                    da[f] = A.add_out ? mua * gr[f] : 0.0;
                }
                ul = 1;
                th = mua * kc * P.pQ;
            }
        } else {
            // loss seed of the step start state: acc += dt w_q dp/dU at probe q
            const int q = k - nal;
            cell = A.pc[q];
            double Vc[NU5];
#pragma unroll
            for (int f = 0; f < NU5; ++f) Vc[f] = A.seedU[(size_t)f * A.n + cell];
            const PGrad P = pgrad(g, Vc);
            const double s = A.dt * A.pw[q];
            da[0] = s * P.pr;
            da[1] = s * P.pm;
            da[2] = s * P.pn;
            da[3] = s * P.pE;
            da[4] = s * P.pY;
            th = s * P.pQ;
        }
        tc[k] = cell;
        uselam[k] = ul;
        dth[k] = th;
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
            dlam[k][f] = dl[f];
            dacc[k][f] = da[f];
        }
    }
    __syncthreads();
    if (k < T && tc[k] >= 0) {
        bool first = true;
        for (int q = 0; q < k; ++q) first = first && (tc[q] != tc[k]);
        if (first) {
            double sl[NU5], sa[NU5];
            int ul = 0;
#pragma unroll
            for (int f = 0; f < NU5; ++f) sl[f] = sa[f] = 0.0;
            for (int q = k; q < T; ++q) {
                if (tc[q] != tc[k]) continue;
                ul |= uselam[q];
#pragma unroll
                for (int f = 0; f < NU5; ++f) {
                    sl[f] += dlam[q][f];
                    sa[f] += dacc[q][f];
                }
            }
            const long long cc = tc[k];
#pragma unroll
            for (int f = 0; f < NU5; ++f) {
                if (ul) A.lamOut[(size_t)f * A.n + cc] += sl[f];
                A.acc[(size_t)f * A.n + cc] += sa[f];
            }
        }
    }
    if (threadIdx.x == 0) {
        double sQ = red[2];
        for (int q = 0; q < T; ++q) sQ += dth[q];
        A.theta[0] += sQ;
        A.theta[1] += red[3];
    }
}

// Loss terms of a run of states: term[n0 + m - 1] = dt sum_q w_q p(U_m at cell_q)
// for the states U_m = base + m * stride, m = 1 .. count - 1, then `last` (if not
// null) as m = count. The terms are summed in step order at the end, so the loss
// does not depend on how the run was cut into segments.
__global__ __launch_bounds__(AWG) void adj_loss(AdjGrid g, const double* base, long long stride,
                                                int count, const double* last, int n0, long long n,
                                                const int* pc, const double* pw, int np, double dt,
                                                double* term) {
    const int ns = (count - 1) + (last ? 1 : 0);
    const int si = blockIdx.x * AWG + threadIdx.x;
    if (si >= ns) return;
    const double* U = (si < count - 1) ? base + (size_t)(si + 1) * stride : last;
    double acc = 0.0;
    for (int q = 0; q < np; ++q) {
        double V[NU5];
        for (int f = 0; f < NU5; ++f) V[f] = U[(size_t)f * n + pc[q]];
        const PGrad P = pgrad(g, V);
        acc += pw[q] * P.p;
    }
    term[n0 + si] = dt * acc;
}

__global__ void adj_loss_sum(const double* term, int nsteps, double* loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nsteps; ++q) s += term[q];
    loss[0] = s;
}

// Loss seed of one state: lambda += dt sum_q w_q dp/dU at the probes, theta_Q += dt w_q dp/dQ.
__global__ void adj_seed(AdjGrid g, const double* U, long long n, const int* pc, const double* pw,
                         int np, double dt, double* lam, double* theta) {
    if (threadIdx.x != 0) return;
    for (int q = 0; q < np; ++q) {
        double V[NU5];
        for (int f = 0; f < NU5; ++f) V[f] = U[(size_t)f * n + pc[q]];
        const PGrad P = pgrad(g, V);
        const double s = dt * pw[q];
        lam[(size_t)0 * n + pc[q]] += s * P.pr;
        lam[(size_t)1 * n + pc[q]] += s * P.pm;
        lam[(size_t)2 * n + pc[q]] += s * P.pn;
        lam[(size_t)3 * n + pc[q]] += s * P.pE;
        lam[(size_t)4 * n + pc[q]] += s * P.pY;
        theta[0] += s * P.pQ;
    }
}

// dL/dW0 from dL/dU0 through U0 = cons(W0) (one-step model); Q part to partials.
__global__ __launch_bounds__(AWG) void adj_chain_ic(AdjGrid g, const double* W, const double* lam,
                                                    long long n, double* gW, double* part) {
    __shared__ double sh[8];
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    double pq = 0.0;
    if (c < n) {
        const double rho = W[c], u = W[n + c], v = W[2 * n + c], Y = W[4 * n + c];
        const double l0 = lam[c], l1 = lam[n + c], l2 = lam[2 * n + c], l3 = lam[3 * n + c],
                     l4 = lam[4 * n + c];
        gW[c] = l0 + l1 * u + l2 * v + l3 * (0.5 * (u * u + v * v) + Y * g.Q) + l4 * Y;
        gW[n + c] = l1 * rho + l3 * rho * u;
        gW[2 * n + c] = l2 * rho + l3 * rho * v;
        gW[3 * n + c] = l3 / (g.gamma - 1.0);
        gW[4 * n + c] = l3 * rho * g.Q + l4 * rho;
        pq = l3 * rho * Y;
    }
    const double s = block_sum(pq, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void adj_chain_sum(const double* part, int nb, double* theta) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += part[q];
    theta[0] += s;
}

// ------------------------------------------------------------------ launchers
hipError_t adj_alpha_launch(const AlphaArgs& P, hipStream_t s) {
    if (P.nsteps <= 0) return hipSuccess;
    adj_alpha<<<dim3(P.nbd, 3 * P.nsteps), AWG, 0, s>>>(P);
    adj_alpha_reduce<<<3 * P.nsteps, AWG, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t adj_stage(const AdjArgs& A, hipStream_t s) {
    const int ni = (A.g.nx + 1) * A.g.ny + (A.g.twod ? A.g.nx * (A.g.ny + 1) : 0);
    adj_iface<<<dim3((ni + AWG - 1) / AWG, NU5), AWG, 0, s>>>(A);
    adj_cell<<<A.nbd, AWG, 0, s>>>(A);
    adj_finish<<<1, AWG, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_loss_launch(const AdjGrid& g, const double* base, long long stride, int count,
                           const double* last, int n0, long long n, const int* pc, const double* pw,
                           int np, double dt, double* term, hipStream_t s) {
    const int ns = (count - 1) + (last ? 1 : 0);
    if (ns <= 0) return hipSuccess;
    adj_loss<<<(ns + AWG - 1) / AWG, AWG, 0, s>>>(g, base, stride, count, last, n0, n, pc, pw, np,
                                                 dt, term);
    return hipGetLastError();
}

hipError_t adj_loss_sum_launch(const double* term, int nsteps, double* loss, hipStream_t s) {
    adj_loss_sum<<<1, 64, 0, s>>>(term, nsteps, loss);
    return hipGetLastError();
}

hipError_t adj_seed_launch(const AdjGrid& g, const double* U, long long n, const int* pc,
                           const double* pw, int np, double dt, double* lam, double* theta,
                           hipStream_t s) {
    adj_seed<<<1, 64, 0, s>>>(g, U, n, pc, pw, np, dt, lam, theta);
    return hipGetLastError();
}

hipError_t adj_chain_launch(const AdjGrid& g, const double* W, const double* lam, long long n,
                            double* gW, double* part, double* theta, hipStream_t s) {
    const int nb = (int)((n + AWG - 1) / AWG);
    adj_chain_ic<<<nb, AWG, 0, s>>>(g, W, lam, n, gW, part);
    adj_chain_sum<<<1, 64, 0, s>>>(part, nb, theta);
    return hipGetLastError();
}

}  // namespace janc
