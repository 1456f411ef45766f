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
//   A0/A0b  alpha_x = max(|u|+c), alpha_y = max(|v|+c) and their argmax (lowest
//           linear index among equal maxima) from the stage input;
//   A1      per cell of the x and y strips (interior plus 3 ghost layers): the
//           ghost source, the state, and the split fluxes F+/F- (G+/G-);
//   B       per interface: mu_Fhat = (mu_right - mu_left)/dx and the reverse of
//           both WENO5 reconstructions (5 + 5 weights per component);
//   C       per strip cell: gather of the split-flux adjoints from the 5 + 5
//           interfaces that read it, reverse of the split (flux Jacobian and
//           the alpha term), partial sums of d/dalpha and of d/dQ;
//   D       per interior cell: own strip values, ghost cells that copy or mirror
//           it, the explicit Arrhenius source, and the RK bookkeeping;
//   E       one workgroup: the deterministic sums of the partials, the alpha
//           adjoints applied at the argmax cells, theta accumulation.
#include "janc_device.h"

namespace janc {

constexpr int NU5 = 5;
constexpr int AWG = 256;

__host__ __device__ __forceinline__ int xs_n(const AdjGrid& g) { return (g.nx + 6) * g.ny; }
__host__ __device__ __forceinline__ int ys_n(const AdjGrid& g) { return g.twod ? g.nx * (g.ny + 6) : 0; }

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

__device__ __forceinline__ void load_src(const AdjArgs& A, long long s, unsigned fl, double (&u)[NU5]) {
    if (s >= 0) {
#pragma unroll
        for (int f = 0; f < NU5; ++f) u[f] = A.V[(size_t)f * A.n + s];
    } else {
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

// Wave speeds of an interior cell as the forward reductions compute them.
__device__ __forceinline__ void cell_speeds(const AdjArgs& A, long long c, double& sx, double& sy) {
    double V[NU5];
#pragma unroll
    for (int f = 0; f < NU5; ++f) V[f] = A.V[(size_t)f * A.n + c];
    DevDomain D{};
    D.gamma = A.g.gamma;
    D.R = A.g.R;
    D.Q = A.g.Q;
    double T, cs, vx, vy;
    owner_state<ONESTEP, NU5>(V, 0.0, D, nullptr, T, cs, vx, vy);
    sx = fabs(vx) + cs;
    sy = fabs(vy) + cs;
}

__global__ __launch_bounds__(AWG) void adj_alpha(AdjArgs A) {
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    if (c >= A.n) return;
    double sx, sy;
    cell_speeds(A, c, sx, sy);
    atomicMax(&A.amax[0], (unsigned long long)__double_as_longlong(sx));
    atomicMax(&A.amax[1], (unsigned long long)__double_as_longlong(sy));
}

__global__ __launch_bounds__(AWG) void adj_argmax(AdjArgs A) {
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    if (c >= A.n) return;
    double sx, sy;
    cell_speeds(A, c, sx, sy);
    if (__double_as_longlong(sx) == (long long)A.amax[0]) atomicMin(&A.argm[0], (int)c);
    if (__double_as_longlong(sy) == (long long)A.amax[1]) atomicMin(&A.argm[1], (int)c);
}

// A1: strip cells -> state, ghost source, split fluxes.
__global__ __launch_bounds__(AWG) void adj_prep(AdjArgs A) {
    const int q = blockIdx.x * AWG + threadIdx.x;
    const AdjGrid& g = A.g;
    const int nxs = xs_n(g), nys = ys_n(g);
    if (q >= nxs + nys) return;
    const bool xdir = q < nxs;
    int i, j, s;
    if (xdir) {
        j = q / (g.nx + 6);
        i = q - j * (g.nx + 6) - 3;
        s = q;
    } else {
        s = q - nxs;
        const int yj = s / g.nx;
        i = s - yj * g.nx;
        j = yj - 3;
    }
    unsigned fl;
    const long long src = usrc(g, i, j, fl);
    double V[NU5];
    load_src(A, src, fl, V);
    const double al = __longlong_as_double((long long)A.amax[xdir ? 0 : 1]);
    DevDomain D{};
    D.gamma = g.gamma;
    D.Q = g.Q;
    double vx, vy, p;
    halo_prims<ONESTEP, NU5>(V, 0.0, D, nullptr, vx, vy, p);
    const double vn = xdir ? vx : vy;
    const int ns = xdir ? nxs : nys;
    double* Vo = xdir ? A.Vx : A.Vy;
    double* Fp = xdir ? A.Fpx : A.Fpy;
    double* Fm = xdir ? A.Fmx : A.Fmy;
    (xdir ? A.srcx : A.srcy)[s] = (src >= 0) ? (src | ((long long)fl << 40)) : src;
#pragma unroll
    for (int f = 0; f < NU5; ++f) {
        double F = V[f] * vn;
        if (f == (xdir ? 1 : 2)) F += p;
        if (f == 3) F = (V[f] + p) * vn;
        Vo[(size_t)f * ns + s] = V[f];
        Fp[(size_t)f * ns + s] = 0.5 * (F + al * V[f]);
        Fm[(size_t)f * ns + s] = 0.5 * (F - al * V[f]);
    }
}

// B: interfaces -> reverse WENO weights.
__global__ __launch_bounds__(AWG) void adj_iface(AdjArgs A) {
    const int q = blockIdx.x * AWG + threadIdx.x;
    const AdjGrid& g = A.g;
    const int nix = (g.nx + 1) * g.ny, niy = g.twod ? g.nx * (g.ny + 1) : 0;
    if (q >= nix + niy) return;
    const double mscale = A.b * A.dt;
    if (q < nix) {
        const int j = q / (g.nx + 1), k = q - j * (g.nx + 1);
        const int nxs = xs_n(g);
        const int base = j * (g.nx + 6) + k;
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
            const double mr = (k < g.nx) ? A.lamW[(size_t)f * A.n + (size_t)j * g.nx + k] : 0.0;
            const double ml = (k > 0) ? A.lamW[(size_t)f * A.n + (size_t)j * g.nx + k - 1] : 0.0;
            const double fb = mscale * (mr - ml) * g.idx;
            const double* P = A.Fpx + (size_t)f * nxs + base;
            const double* M = A.Fmx + (size_t)f * nxs + base;
            double gp[5], gm[5];
            weno5_adj(P[0], P[1], P[2], P[3], P[4], fb, gp);
            weno5_adj(M[5], M[4], M[3], M[2], M[1], fb, gm);
            double* out = A.cx + (size_t)f * 10 * nix;
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                out[(size_t)m * nix + q] = gp[m];
                out[(size_t)(5 + m) * nix + q] = gm[4 - m];
            }
        }
    } else {
        const int r = q - nix;
        const int k = r / g.nx, i = r - k * g.nx;
        const int nys = ys_n(g);
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
            const double mr = (k < g.ny) ? A.lamW[(size_t)f * A.n + (size_t)k * g.nx + i] : 0.0;
            const double ml = (k > 0) ? A.lamW[(size_t)f * A.n + (size_t)(k - 1) * g.nx + i] : 0.0;
            const double fb = mscale * (mr - ml) * g.idy;
            const double* P = A.Fpy + (size_t)f * nys + (size_t)k * g.nx + i;
            const double* M = A.Fmy + (size_t)f * nys + (size_t)k * g.nx + i;
            const int X = g.nx;
            double gp[5], gm[5];
            weno5_adj(P[0], P[X], P[2 * X], P[3 * X], P[4 * X], fb, gp);
            weno5_adj(M[5 * X], M[4 * X], M[3 * X], M[2 * X], M[X], fb, gm);
            double* out = A.cy + (size_t)f * 10 * niy;
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                out[(size_t)m * niy + r] = gp[m];
                out[(size_t)(5 + m) * niy + r] = gm[4 - m];
            }
        }
    }
}

// C: strip cells -> adjoint of the strip state (flux Jacobian + alpha term).
__global__ __launch_bounds__(AWG) void adj_gather(AdjArgs A) {
    __shared__ double sh[8];
    const int q = blockIdx.x * AWG + threadIdx.x;
    const AdjGrid& g = A.g;
    const int nxs = xs_n(g), nys = ys_n(g);
    const int nix = (g.nx + 1) * g.ny, niy = g.twod ? g.nx * (g.ny + 1) : 0;
    double pax = 0.0, pay = 0.0, pQ = 0.0;
    if (q < nxs + nys) {
        const bool xdir = q < nxs;
        const int ns = xdir ? nxs : nys;
        const int s = xdir ? q : q - nxs;
        double V[NU5], mp[NU5], mm[NU5];
#pragma unroll
        for (int f = 0; f < NU5; ++f) V[f] = (xdir ? A.Vx : A.Vy)[(size_t)f * ns + s];
        if (xdir) {
            const int j = s / (g.nx + 6), xi = s - j * (g.nx + 6);
#pragma unroll
            for (int f = 0; f < NU5; ++f) {
                const double* cf = A.cx + (size_t)f * 10 * nix;
                double ap = 0.0, am = 0.0;
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    const int Ip = xi - m, Im = xi - 1 - m;
                    if (Ip >= 0 && Ip <= g.nx) ap += cf[(size_t)m * nix + j * (g.nx + 1) + Ip];
                    if (Im >= 0 && Im <= g.nx) am += cf[(size_t)(5 + m) * nix + j * (g.nx + 1) + Im];
                }
                mp[f] = ap;
                mm[f] = am;
            }
        } else {
            const int yj = s / g.nx, i = s - yj * g.nx;
#pragma unroll
            for (int f = 0; f < NU5; ++f) {
                const double* cf = A.cy + (size_t)f * 10 * niy;
                double ap = 0.0, am = 0.0;
#pragma unroll
                for (int m = 0; m < 5; ++m) {
                    const int Ip = yj - m, Im = yj - 1 - m;
                    if (Ip >= 0 && Ip <= g.ny) ap += cf[(size_t)m * niy + Ip * g.nx + i];
                    if (Im >= 0 && Im <= g.ny) am += cf[(size_t)(5 + m) * niy + Im * g.nx + i];
                }
                mp[f] = ap;
                mm[f] = am;
            }
        }
        const PGrad P = pgrad(g, V);
        const double al = __longlong_as_double((long long)A.amax[xdir ? 0 : 1]);
        double a[NU5], bq[NU5], out[NU5];
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
        double d_rho = a_nm * (-w * w + P.pr) + a_tm * (-w * t) + a_E * (-w * (E + P.p) * ir + w * P.pr) +
                       a_r * (-r * w * ir);
        double d_nm = a_mass + a_nm * (2.0 * w + pw) + a_tm * t + a_E * ((E + P.p) * ir + w * pw) + a_r * (r * ir);
        double d_tm = a_nm * pt + a_tm * w + a_E * w * pt;
        double d_E = a_nm * P.pE + a_E * w * (1.0 + P.pE);
        double d_r = a_nm * P.pY + a_E * w * P.pY + a_r * w;
        out[0] = d_rho;
        out[xdir ? 1 : 2] = d_nm;
        out[xdir ? 2 : 1] = d_tm;
        out[3] = d_E;
        out[4] = d_r;
        double pal = 0.0;
#pragma unroll
        for (int f = 0; f < NU5; ++f) {
            out[f] += al * bq[f];
            pal += V[f] * bq[f];
        }
        pQ = a_nm * P.pQ + a_E * w * P.pQ;
        const long long src = (xdir ? A.srcx : A.srcy)[s];
        if (src < 0) {
            // Dirichlet ghost: its energy depends on Q through the chemical energy rho Y Q
            const double* row = g.dirU + (size_t)(-src - 1) * (MAXF + 1);
            pQ += out[3] * row[4];
        }
        if (xdir) pax = pal;
        else pay = pal;
        double* go = xdir ? A.gx : A.gy;
#pragma unroll
        for (int f = 0; f < NU5; ++f) go[(size_t)f * ns + s] = out[f];
    }
    const double s0 = block_sum(pax, sh);
    const double s1 = block_sum(pay, sh);
    const double s2 = block_sum(pQ, sh);
    if (threadIdx.x == 0) {
        A.part[(size_t)blockIdx.x * 4 + 0] = s0;
        A.part[(size_t)blockIdx.x * 4 + 1] = s1;
        A.part[(size_t)blockIdx.x * 4 + 2] = s2;
        A.part[(size_t)blockIdx.x * 4 + 3] = 0.0;
    }
}

// D: interior cells -> lambda of the stage input, source term, RK bookkeeping.
__global__ __launch_bounds__(AWG) void adj_combine(AdjArgs A) {
    __shared__ double sh[8];
    const long long c = (long long)blockIdx.x * AWG + threadIdx.x;
    const AdjGrid& g = A.g;
    double pQ = 0.0, pEa = 0.0;
    if (c < A.n) {
        const int j = (int)(c / g.nx), i = (int)(c - (long long)j * g.nx);
        const int nxs = xs_n(g), nys = ys_n(g);
        double out[NU5];
        const int sxs = j * (g.nx + 6) + (i + 3);
#pragma unroll
        for (int f = 0; f < NU5; ++f) out[f] = A.b * A.lamW[(size_t)f * A.n + c] + A.gx[(size_t)f * nxs + sxs];
        if (g.twod) {
            const int sys = (j + 3) * g.nx + i;
#pragma unroll
            for (int f = 0; f < NU5; ++f) out[f] += A.gy[(size_t)f * nys + sys];
        }
        // ghost cells that copy or mirror this cell
        for (int gq = 0; gq < 6; ++gq) {
            const int gi = (gq < 3) ? -1 - gq : g.nx + gq - 3;
            unsigned fl;
            const long long s = usrc(g, gi, j, fl);
            if (s != c) continue;
            const int sx = j * (g.nx + 6) + (gi + 3);
#pragma unroll
            for (int f = 0; f < NU5; ++f) {
                double v = A.gx[(size_t)f * nxs + sx];
                if ((f == 1 && (fl & 1u)) || (f == 2 && (fl & 2u))) v = -v;
                out[f] += v;
            }
        }
        if (g.twod) {
            for (int gq = 0; gq < 6; ++gq) {
                const int gj = (gq < 3) ? -1 - gq : g.ny + gq - 3;
                unsigned fl;
                const long long s = usrc(g, i, gj, fl);
                if (s != c) continue;
                const int sy = (gj + 3) * g.nx + i;
#pragma unroll
                for (int f = 0; f < NU5; ++f) {
                    double v = A.gy[(size_t)f * nys + sy];
                    if ((f == 1 && (fl & 1u)) || (f == 2 && (fl & 2u))) v = -v;
                    out[f] += v;
                }
            }
        }
        // explicit source S4 = -k r exp(-Ea/T), T = p/(rho R)
        double V[NU5];
#pragma unroll
        for (int f = 0; f < NU5; ++f) V[f] = A.V[(size_t)f * A.n + c];
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
        pQ = mu4 * dSdT * (P.pQ * iRr);
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
    const double s0 = block_sum(pQ, sh);
    const double s1 = block_sum(pEa, sh);
    if (threadIdx.x == 0) {
        A.part[(size_t)(A.nbc + blockIdx.x) * 4 + 0] = 0.0;
        A.part[(size_t)(A.nbc + blockIdx.x) * 4 + 1] = 0.0;
        A.part[(size_t)(A.nbc + blockIdx.x) * 4 + 2] = s0;
        A.part[(size_t)(A.nbc + blockIdx.x) * 4 + 3] = s1;
    }
}

// E: one workgroup; deterministic sums, alpha adjoints at the argmax cells.
__global__ void adj_finish(AdjArgs A) {
    if (threadIdx.x != 0) return;
    double sax = 0.0, say = 0.0, sQ = 0.0, sEa = 0.0;
    for (int q = 0; q < A.nbc + A.nbd; ++q) {
        sax += A.part[(size_t)q * 4 + 0];
        say += A.part[(size_t)q * 4 + 1];
        sQ += A.part[(size_t)q * 4 + 2];
        sEa += A.part[(size_t)q * 4 + 3];
    }
    const AdjGrid& g = A.g;
    for (int d = 0; d < (g.twod ? 2 : 1); ++d) {
        const double mua = d == 0 ? sax : say;
        const long long c = A.argm[d];
        if (c < 0 || c >= A.n) continue;   // no cell attained the maximum (cannot happen for finite data)
        double V[NU5];
#pragma unroll
        for (int f = 0; f < NU5; ++f) V[f] = A.V[(size_t)f * A.n + c];
        const PGrad P = pgrad(g, V);
        const double rho = V[0];
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
            A.lamOut[(size_t)f * A.n + c] += mua * gr[f];
            if (A.add_out) A.acc[(size_t)f * A.n + c] += mua * gr[f];
        }
        sQ += mua * kc * P.pQ;
    }
    A.theta[0] += sQ;
    A.theta[1] += sEa;
    A.amax[0] = 0ull;
    A.amax[1] = 0ull;
    A.argm[0] = 0x7fffffff;
    A.argm[1] = 0x7fffffff;
}

// Loss accumulation of the forward pass: loss += dt sum_q w_q p(U[cell_q]).
__global__ void adj_loss(AdjGrid g, const double* U, long long n, const int* pc, const double* pw,
                         int np, double dt, double* loss) {
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int q = 0; q < np; ++q) {
        double V[NU5];
        for (int f = 0; f < NU5; ++f) V[f] = U[(size_t)f * n + pc[q]];
        const PGrad P = pgrad(g, V);
        acc += pw[q] * P.p;
    }
    loss[0] += dt * acc;
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

__global__ void adj_reset(AdjArgs A) {
    if (threadIdx.x == 0) {
        A.amax[0] = 0ull;
        A.amax[1] = 0ull;
        A.argm[0] = 0x7fffffff;
        A.argm[1] = 0x7fffffff;
    }
}

// ------------------------------------------------------------------ launchers
hipError_t adj_stage(const AdjArgs& A, hipStream_t s) {
    const int nc = (int)((A.n + AWG - 1) / AWG);
    const int ns = xs_n(A.g) + ys_n(A.g);
    const int ni = (A.g.nx + 1) * A.g.ny + (A.g.twod ? A.g.nx * (A.g.ny + 1) : 0);
    adj_alpha<<<nc, AWG, 0, s>>>(A);
    adj_argmax<<<nc, AWG, 0, s>>>(A);
    adj_prep<<<(ns + AWG - 1) / AWG, AWG, 0, s>>>(A);
    adj_iface<<<(ni + AWG - 1) / AWG, AWG, 0, s>>>(A);
    adj_gather<<<(ns + AWG - 1) / AWG, AWG, 0, s>>>(A);
    adj_combine<<<nc, AWG, 0, s>>>(A);
    adj_finish<<<1, 64, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_reset_launch(const AdjArgs& A, hipStream_t s) {
    adj_reset<<<1, 64, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_loss_launch(const AdjGrid& g, const double* U, long long n, const int* pc,
                           const double* pw, int np, double dt, double* loss, hipStream_t s) {
    adj_loss<<<1, 64, 0, s>>>(g, U, n, pc, pw, np, dt, loss);
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

int adj_partial_blocks(const AdjGrid& g, long long n, int* nbc, int* nbd) {
    const int ns = (g.nx + 6) * g.ny + (g.twod ? g.nx * (g.ny + 6) : 0);
    *nbc = (ns + AWG - 1) / AWG;
    *nbd = (int)((n + AWG - 1) / AWG);
    return *nbc + *nbd;
}

}  // namespace janc
