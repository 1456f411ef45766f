/*
 * janc_oracle.cpp -- plain FP64 CPU oracle for the per-time-step core update of
 * the compressible reacting-flow solver of arXiv 2504.13750 (JANC).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code, header, table or
 * helper with the HIP library; both sides consume the same seeded primitive
 * inputs and nothing else.
 *
 * Structure: array-of-structs per cell, straightforward loops over cells,
 * ghost-extended copies of each block (the "ghost block" of Sec. 3.1.3), and
 * everything templated on the scalar type so that a forward-mode dual number
 * gives the exact tangent of the discrete map. Build with -O2 -fno-fast-math
 * -ffp-contract=off so every operation is the IEEE operation written here.
 *
 * What is computed (paper Sec. 4):
 *   conserved U = [rho, rho u, rho v, E, rho Y_1 .. rho Y_{Ns-1}]     (Eq. 4.1)
 *   thermally perfect mixture, NASA-7 polynomials (one or two ranges) (Eq. 4.2-4.5)
 *   T from the internal energy by Newton, warm-started               (Sec. 4.2, last paragraph)
 *   Lax-Friedrichs flux vector splitting with a global alpha         (Eq. 4.11)
 *   WENO5 reconstruction of F+ and F-, 3 ghost layers                (Sec. 4.2)
 *   conservative difference                                          (Eq. 4.10)
 *   third-order TVD (SSP) Runge-Kutta                                (Sec. 4.2)
 *   first-order point-implicit chemistry on rho Y_1..rho Y_{Ns-1}    (Eq. 4.12-4.13)
 *   mass-action rates with Arrhenius forward and equilibrium reverse (Eq. 4.6-4.9)
 *   block tables: same-level ghosts, coarse-fine "external boundary" sync,
 *   four-to-one restriction, synchronous and crossover advance       (Sec. 3.1.3-3.1.4, Alg. 2-3,
 *                                                                     Fig. 2)
 *   layer update (masked and buffer cells, subregions, one-to-four
 *   injection of new blocks, unaltered blocks kept)                  (Sec. 3.1.2, 3.1.4, Alg. 2)
 *
 * Readings where the paper is silent:
 *   - WENO5 is the Jiang-Shu form with eps = 1e-6, applied component-wise.
 *   - alpha is recomputed each RK stage over the solved cells of the scope.
 *   - dt = CFL / max((|u|+c)/dx + (|v|+c)/dy) (1-D: the x term only).
 *   - Newton stops when |dT| <= 1e-12 T (at most 50 iterations).
 *   - chemistry follows the flux RK3 step (flux-then-source, as in the
 *     listing of advance_one_step), over the full dt.
 *   - the coarse-fine boundary uses the ring rule: cells within 3 of an
 *     uncovered in-domain cell are not solved; their value is the injection
 *     of the coarser level at the same stage.
 *   - Strang splitting, when selected, takes half the chemistry step before
 *     the RK stages and half after them, with dt from the step-start state.
 *   - regridding masks cells by a normalized central density difference and
 *     refines fixed subregions of each block (see the regridding section).
 *
 * Parity unpinned: the coarse-fine coupling of partially refined hierarchies (ring
 * cells read from the coarser level, and in the crossover advance the coarser level's
 * state held while a finer level steps) has no closed form or independent reference.
 * Its pins cover special cases and properties: full refinement equals the fine
 * uniform grid, restriction is the four-child mean, a constant state survives, one
 * level equals the uniform grid, mirror-image and transposed hierarchies give
 * mirror-image and transposed results, and an advected wave crossing a refined band
 * converges at first order; beyond these the GPU is checked against this code alone.
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double RU = 8.314472;      // J/(mol K), paper Sec. 4.1
const double PATM = 101325.0;    // Pa, Eq. 4.9
const double WENO_EPS = 1e-6;

enum { ST_OK = 0, ST_EINVAL = -1, ST_NONFINITE = -4, ST_NEWTON = -5, ST_NEGATIVE = -6 };
enum { BC_PERIODIC = 0, BC_ZEROGRAD = 1, BC_SLIPWALL = 2, BC_DIRICHLET = 3 };
enum { SIDE_W = 0, SIDE_E = 1, SIDE_S = 2, SIDE_N = 3 };
enum { MODEL_CPG = 0, MODEL_ONESTEP = 1, MODEL_DETAILED = 2 };

// ------------------------------------------------------------------ dual numbers
struct Dual {
    double v, d;
    Dual(double x = 0.0) : v(x), d(0.0) {}
    Dual(double x, double y) : v(x), d(y) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual pow(Dual a, double b) {
    double p = std::pow(a.v, b);
    return Dual(p, b * std::pow(a.v, b - 1.0) * a.d);
}
// derivative of |x| taken as sign(x), zero at x == 0
inline Dual fabs(Dual a) {
    double s = (a.v > 0.0) ? 1.0 : ((a.v < 0.0) ? -1.0 : 0.0);
    return Dual(std::fabs(a.v), s * a.d);
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double der(double) { return 0.0; }
inline double der(const Dual& x) { return x.d; }
using std::exp; using std::log; using std::sqrt; using std::pow; using std::fabs;

template <class S> inline bool finite(const S& x) { return std::isfinite(val(x)); }

// ------------------------------------------------------------------ model data
struct MechData {
    int ns = 0, nr = 0;
    std::vector<double> M, nasa, A, b, Ea, tb;
    std::vector<double> nasa_hi, tmid;   // two-range NASA-7: high set, switch temperature
    std::vector<int> nuf, nub, has_tb, rev;
};

template <class S> struct Phys {
    int model = 0;
    int nU = 0;
    int full_jac = 0;   // point-implicit Jacobian with T following the composition
    S gamma, R, Q, Ea, k;
    const MechData* mech = nullptr;
};

template <class S> struct Prim { S rho, u, v, p, T, c; };

// NASA-7 polynomials, Eq. 4.3-4.5, in units of R_u / M_k.
template <class S> S nasa_cp(const double* a, const S& T) {
    return a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
}
template <class S> S nasa_h(const double* a, const S& T) {
    return a[0] * T + a[1] * T * T / 2.0 + a[2] * T * T * T / 3.0 + a[3] * T * T * T * T / 4.0 +
           a[4] * T * T * T * T * T / 5.0 + a[5];
}
template <class S> S nasa_s(const double* a, const S& T) {
    return a[0] * log(T) + a[1] * T + a[2] * T * T / 2.0 + a[3] * T * T * T / 3.0 +
           a[4] * T * T * T * T / 4.0 + a[6];
}

// NASA-7 coefficients of species k at T. With two temperature ranges (as NASA-7
// tables are published) the high set applies for T >= t_mid of the species, the low
// set below; with one range the single set.
template <class S> const double* coeffs(const MechData& m, int k, const S& T) {
    if (!m.nasa_hi.empty() && val(T) >= m.tmid[k]) return &m.nasa_hi[7 * k];
    return &m.nasa[7 * k];
}

// Mass fractions of all Ns species from the conserved vector (last = complement).
template <class S> void mass_fractions(const MechData& m, const S* U, const S& rho, S* Y) {
    S sum = 0.0;
    for (int k = 0; k < m.ns - 1; ++k) {
        Y[k] = U[4 + k] / rho;
        sum = sum + Y[k];
    }
    Y[m.ns - 1] = 1.0 - sum;
}

// Internal energy e(T) = sum_k Y_k (h_k - R_k T) and cv(T), per unit mass.
template <class S> void mixture_e_cv(const MechData& m, const S* Y, const S& T, S& e, S& cv) {
    e = 0.0;
    cv = 0.0;
    for (int k = 0; k < m.ns; ++k) {
        double Rk = RU / m.M[k];
        const double* a = coeffs(m, k, T);
        e = e + Y[k] * Rk * (nasa_h(a, T) - T);
        cv = cv + Y[k] * Rk * (nasa_cp(a, T) - 1.0);
    }
}

template <class S> S mixture_R(const MechData& m, const S* Y) {
    S r = 0.0;
    for (int k = 0; k < m.ns; ++k) r = r + Y[k] / m.M[k];
    return RU * r;
}

// Newton-Raphson for T from e (Sec. 4.2: warm start from the previous T).
template <class S> int newton_T(const MechData& m, const S* Y, const S& e, S& T) {
    for (int it = 0; it < 50; ++it) {
        S ecur, cv;
        mixture_e_cv(m, Y, T, ecur, cv);
        S dT = (ecur - e) / cv;
        T = T - dT;
        if (!finite(T)) return ST_NONFINITE;
        if (std::fabs(val(dT)) <= 1e-12 * std::fabs(val(T))) return ST_OK;
    }
    return ST_NEWTON;
}

// Primitive state of one cell; T is the Newton warm start for DETAILED.
template <class S> int primitives(const Phys<S>& ph, const S* U, const S& Tguess, Prim<S>& P) {
    P.rho = U[0];
    if (!finite(P.rho)) return ST_NONFINITE;
    if (!(val(P.rho) > 0.0)) return ST_NEGATIVE;
    P.u = U[1] / P.rho;
    P.v = U[2] / P.rho;
    S e = U[3] / P.rho - 0.5 * (P.u * P.u + P.v * P.v);
    S gam;
    if (ph.model == MODEL_CPG) {
        P.p = (ph.gamma - 1.0) * P.rho * e;
        P.T = P.p / (P.rho * ph.R);
        gam = ph.gamma;
    } else if (ph.model == MODEL_ONESTEP) {
        S Y = U[4] / P.rho;
        P.p = (ph.gamma - 1.0) * P.rho * (e - Y * ph.Q);
        P.T = P.p / (P.rho * ph.R);
        gam = ph.gamma;
    } else {
        const MechData& m = *ph.mech;
        S Y[32];
        mass_fractions(m, U, P.rho, Y);
        P.T = Tguess;
        int st = newton_T(m, Y, e, P.T);
        if (st) return st;
        S Rm = mixture_R(m, Y);
        S ecur, cv;
        mixture_e_cv(m, Y, P.T, ecur, cv);
        P.p = P.rho * Rm * P.T;
        gam = (cv + Rm) / cv;
    }
    if (!finite(P.p)) return ST_NONFINITE;
    if (!(val(P.p) > 0.0) || !(val(P.T) > 0.0)) return ST_NEGATIVE;
    P.c = sqrt(gam * P.p / P.rho);
    return ST_OK;
}

// Conserved state and T from the primitive input layout of each model.
template <class S> int conserved_from_primitive(const Phys<S>& ph, const S* W, S* U, S& T) {
    if (ph.model == MODEL_CPG || ph.model == MODEL_ONESTEP) {
        S rho = W[0], u = W[1], v = W[2], p = W[3];
        U[0] = rho;
        U[1] = rho * u;
        U[2] = rho * v;
        U[3] = p / (ph.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
        if (ph.model == MODEL_ONESTEP) {
            U[3] = U[3] + rho * W[4] * ph.Q;
            U[4] = rho * W[4];
        }
        T = p / (rho * ph.R);
    } else {
        const MechData& m = *ph.mech;
        S p = W[0], u = W[1], v = W[2];
        T = W[3];
        S Y[32];
        S sum = 0.0;
        for (int k = 0; k < m.ns - 1; ++k) { Y[k] = W[4 + k]; sum = sum + Y[k]; }
        Y[m.ns - 1] = 1.0 - sum;
        S Rm = mixture_R(m, Y);
        S rho = p / (Rm * T);
        S e, cv;
        mixture_e_cv(m, Y, T, e, cv);
        U[0] = rho;
        U[1] = rho * u;
        U[2] = rho * v;
        U[3] = rho * e + 0.5 * rho * (u * u + v * v);
        for (int k = 0; k < m.ns - 1; ++k) U[4 + k] = rho * Y[k];
    }
    return ST_OK;
}

// Physical flux in direction dir (0 = x: F, 1 = y: G), Eq. 4.1.
template <class S> void physical_flux(int nU, const S* U, const Prim<S>& P, int dir, S* F) {
    S vn = (dir == 0) ? P.u : P.v;
    for (int f = 0; f < nU; ++f) F[f] = U[f] * vn;
    F[1 + dir] = F[1 + dir] + P.p;
    F[3] = (U[3] + P.p) * vn;
}

template <class S> S sq(const S& x) { return x * x; }

// WENO5-JS reconstruction at i+1/2 from f_{i-2..i+2} (left-biased).
template <class S> S weno5(const S& a, const S& b, const S& c, const S& d, const S& e) {
    S q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    S q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    S q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    S b0 = (13.0 / 12.0) * sq(a - 2.0 * b + c) + 0.25 * sq(a - 4.0 * b + 3.0 * c);
    S b1 = (13.0 / 12.0) * sq(b - 2.0 * c + d) + 0.25 * sq(b - d);
    S b2 = (13.0 / 12.0) * sq(c - 2.0 * d + e) + 0.25 * sq(3.0 * c - 4.0 * d + e);
    S a0 = 0.1 / sq(WENO_EPS + b0);
    S a1 = 0.6 / sq(WENO_EPS + b1);
    S a2 = 0.3 / sq(WENO_EPS + b2);
    S s = a0 + a1 + a2;
    S w0 = a0 / s, w1 = a1 / s, w2 = a2 / s;
    return w0 * q0 + w1 * q1 + w2 * q2;
}

// ------------------------------------------------------------------ chemistry
inline int nu_at(const std::vector<int>& nu, int ns, int i, int j) { return nu[i * ns + j]; }

template <class S> S ipow(const S& x, int n) {
    S r = 1.0;
    for (int q = 0; q < n; ++q) r = r * x;
    return r;
}

// Production rates wdot_k (kg/m^3/s), Eq. 4.7-4.9, and optionally the Jacobian
// J[k][m] = d wdot_k / d (rho Y_m) for k, m < Ns-1 at fixed rho and T (Eq. 4.12).
template <class S>
void production(const MechData& m, const S& rho, const S& T, const S* rhoY, S* wdot, S* J) {
    const int ns = m.ns, nt = ns - 1;
    S X[32];
    S sum = 0.0;
    for (int j = 0; j < nt; ++j) { X[j] = rhoY[j] / m.M[j]; sum = sum + rhoY[j]; }
    X[nt] = (rho - sum) / m.M[nt];
    S htil[32], stil[32];
    for (int j = 0; j < ns; ++j) {
        htil[j] = nasa_h(coeffs(m, j, T), T);
        stil[j] = nasa_s(coeffs(m, j, T), T);
    }
    for (int k = 0; k < ns; ++k) wdot[k] = 0.0;
    if (J) for (int q = 0; q < nt * nt; ++q) J[q] = 0.0;
    for (int i = 0; i < m.nr; ++i) {
        S kf = m.A[i] * pow(T, m.b[i]) * exp(-m.Ea[i] / (RU * T));
        S kb = 0.0;
        if (m.rev[i]) {
            S g = 0.0;
            int dn = 0;
            for (int j = 0; j < ns; ++j) {
                int d = nu_at(m.nub, ns, i, j) - nu_at(m.nuf, ns, i, j);
                if (d != 0) {
                    g = g + (double)d * (stil[j] - htil[j] / T);
                    dn += d;
                }
            }
            S Keq = exp(g) * pow(PATM / (RU * T), (double)dn);
            kb = kf / Keq;
        }
        S Rf = kf, Rb = kb;
        for (int j = 0; j < ns; ++j) {
            Rf = Rf * ipow(X[j], nu_at(m.nuf, ns, i, j));
            Rb = Rb * ipow(X[j], nu_at(m.nub, ns, i, j));
        }
        S ctb = 1.0;
        if (m.has_tb[i]) {
            ctb = 0.0;
            for (int j = 0; j < ns; ++j) ctb = ctb + m.tb[i * ns + j] * X[j];
        }
        S q = ctb * (Rf - Rb);
        for (int k = 0; k < ns; ++k) {
            int d = nu_at(m.nub, ns, i, k) - nu_at(m.nuf, ns, i, k);
            if (d != 0) wdot[k] = wdot[k] + m.M[k] * (double)d * q;
        }
        if (!J) continue;
        // dq/dX_j by the product rule on integer powers
        S dq[32];
        for (int j = 0; j < ns; ++j) {
            S dRf = 0.0, dRb = 0.0;
            int nf = nu_at(m.nuf, ns, i, j), nb = nu_at(m.nub, ns, i, j);
            if (nf > 0) {
                dRf = kf * (double)nf * ipow(X[j], nf - 1);
                for (int l = 0; l < ns; ++l)
                    if (l != j) dRf = dRf * ipow(X[l], nu_at(m.nuf, ns, i, l));
            }
            if (nb > 0) {
                dRb = kb * (double)nb * ipow(X[j], nb - 1);
                for (int l = 0; l < ns; ++l)
                    if (l != j) dRb = dRb * ipow(X[l], nu_at(m.nub, ns, i, l));
            }
            dq[j] = ctb * (dRf - dRb);
            if (m.has_tb[i]) dq[j] = dq[j] + m.tb[i * ns + j] * (Rf - Rb);
        }
        // dX_j/d(rho Y_m) = delta_jm / M_m - delta_{j,Ns} / M_Ns (complement species)
        for (int k = 0; k < nt; ++k) {
            int d = nu_at(m.nub, ns, i, k) - nu_at(m.nuf, ns, i, k);
            if (d == 0) continue;
            for (int mm = 0; mm < nt; ++mm) {
                S dqdm = dq[mm] / m.M[mm] - dq[nt] / m.M[nt];
                J[k * nt + mm] = J[k * nt + mm] + m.M[k] * (double)d * dqdm;
            }
        }
    }
}

// Dense solve A x = b by Gaussian elimination with partial pivoting.
template <class S> int gauss_solve(int n, S* A, S* b) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(val(A[r * n + c])) > std::fabs(val(A[piv * n + c]))) piv = r;
        if (!(std::fabs(val(A[piv * n + c])) > 0.0)) return ST_NONFINITE;
        if (piv != c) {
            for (int q = 0; q < n; ++q) std::swap(A[c * n + q], A[piv * n + q]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; ++r) {
            S f = A[r * n + c] / A[c * n + c];
            for (int q = c; q < n; ++q) A[r * n + q] = A[r * n + q] - f * A[c * n + q];
            b[r] = b[r] - f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        S s = b[r];
        for (int q = r + 1; q < n; ++q) s = s - A[r * n + q] * b[q];
        b[r] = s / A[r * n + r];
    }
    return ST_OK;
}

// Point-implicit update of rho Y_1..rho Y_{Ns-1} over dt (Eq. 4.12-4.13); Jext, when
// given, replaces the Jacobian at frozen T.
template <class S> int point_implicit(const MechData& m, const S& rho, const S& T, S* rhoY,
                                      const S& dt, const S* Jext = nullptr) {
    const int nt = m.ns - 1;
    S wdot[32];
    std::vector<S> J(nt * nt), A(nt * nt);
    production(m, rho, T, rhoY, wdot, J.data());
    if (Jext) std::copy(Jext, Jext + nt * nt, J.begin());
    S rhs[32];
    for (int k = 0; k < nt; ++k) {
        for (int q = 0; q < nt; ++q) A[k * nt + q] = (k == q ? 1.0 : 0.0) - dt * J[k * nt + q];
        rhs[k] = wdot[k] * dt;
    }
    int st = gauss_solve(nt, A.data(), rhs);
    if (st) return st;
    for (int k = 0; k < nt; ++k) rhoY[k] = rhoY[k] + rhs[k];
    return ST_OK;
}

// ------------------------------------------------------------------ ghost-extended block
// A block plus 3 ghost layers in x (and in y when 2-D). Only the cross-shaped
// part is filled (corners are never read: the sweeps are dimension by dimension).
template <class S> struct Ext {
    int nU = 0, nx = 0, ny = 0, g = 3, gy = 3, W = 0, H = 0;
    std::vector<S> U, T;
    void init(int nU_, int nx_, int ny_) {
        nU = nU_; nx = nx_; ny = ny_;
        gy = (ny > 1) ? 3 : 0;
        W = nx + 2 * g; H = ny + 2 * gy;
        U.assign((size_t)W * H * nU, S(0.0));
        T.assign((size_t)W * H, S(0.0));
    }
    int idx(int i, int j) const { return (j + gy) * W + (i + g); }
    S* u(int i, int j) { return &U[(size_t)idx(i, j) * nU]; }
    S& t(int i, int j) { return T[idx(i, j)]; }
    bool in_cross(int i, int j) const {
        bool xin = (i >= 0 && i < nx), yin = (j >= 0 && j < ny);
        return (xin && j >= -gy && j < ny + gy) || (yin && i >= -g && i < nx + g);
    }
};

// L(U) on the interior of a ghost-extended block (Eq. 4.10, 4.11; WENO5).
template <class S>
int rhs_ext(const Phys<S>& ph, Ext<S>& E, const S& ax, const S& ay, double dx, double dy,
            std::vector<S>& L) {
    const int nU = ph.nU, nx = E.nx, ny = E.ny;
    const bool twod = E.gy > 0;
    std::vector<Prim<S>> P((size_t)E.W * E.H);
    for (int j = -E.gy; j < ny + E.gy; ++j)
        for (int i = -E.g; i < nx + E.g; ++i) {
            if (!E.in_cross(i, j)) continue;
            int st = primitives(ph, E.u(i, j), E.t(i, j), P[E.idx(i, j)]);
            if (st) return st;
        }
    L.assign((size_t)nx * ny * nU, S(0.0));
    std::vector<S> Fp((size_t)E.W * E.H * nU), Fm((size_t)E.W * E.H * nU);
    std::vector<S> F(nU);
    // x sweep: split fluxes on every cell of the x strip
    for (int j = 0; j < ny; ++j)
        for (int i = -E.g; i < nx + E.g; ++i) {
            int c = E.idx(i, j);
            physical_flux(nU, E.u(i, j), P[c], 0, F.data());
            for (int f = 0; f < nU; ++f) {
                Fp[(size_t)c * nU + f] = 0.5 * (F[f] + ax * E.u(i, j)[f]);
                Fm[(size_t)c * nU + f] = 0.5 * (F[f] - ax * E.u(i, j)[f]);
            }
        }
    std::vector<S> Fh((size_t)(nx + 1) * nU);
    for (int j = 0; j < ny; ++j) {
        for (int i = -1; i < nx; ++i) {       // interface i+1/2
            for (int f = 0; f < nU; ++f) {
                auto p = [&](int ii) { return Fp[(size_t)E.idx(ii, j) * nU + f]; };
                auto m = [&](int ii) { return Fm[(size_t)E.idx(ii, j) * nU + f]; };
                Fh[(size_t)(i + 1) * nU + f] = weno5(p(i - 2), p(i - 1), p(i), p(i + 1), p(i + 2)) +
                                               weno5(m(i + 3), m(i + 2), m(i + 1), m(i), m(i - 1));
            }
        }
        for (int i = 0; i < nx; ++i)
            for (int f = 0; f < nU; ++f)
                L[((size_t)j * nx + i) * nU + f] =
                    -(Fh[(size_t)(i + 1) * nU + f] - Fh[(size_t)i * nU + f]) / dx;
    }
    if (twod) {
        for (int j = -E.gy; j < ny + E.gy; ++j)
            for (int i = 0; i < nx; ++i) {
                int c = E.idx(i, j);
                physical_flux(nU, E.u(i, j), P[c], 1, F.data());
                for (int f = 0; f < nU; ++f) {
                    Fp[(size_t)c * nU + f] = 0.5 * (F[f] + ay * E.u(i, j)[f]);
                    Fm[(size_t)c * nU + f] = 0.5 * (F[f] - ay * E.u(i, j)[f]);
                }
            }
        std::vector<S> Gh((size_t)(ny + 1) * nU);
        for (int i = 0; i < nx; ++i) {
            for (int j = -1; j < ny; ++j) {
                for (int f = 0; f < nU; ++f) {
                    auto p = [&](int jj) { return Fp[(size_t)E.idx(i, jj) * nU + f]; };
                    auto m = [&](int jj) { return Fm[(size_t)E.idx(i, jj) * nU + f]; };
                    Gh[(size_t)(j + 1) * nU + f] =
                        weno5(p(j - 2), p(j - 1), p(j), p(j + 1), p(j + 2)) +
                        weno5(m(j + 3), m(j + 2), m(j + 1), m(j), m(j - 1));
                }
            }
            for (int j = 0; j < ny; ++j)
                for (int f = 0; f < nU; ++f)
                    L[((size_t)j * nx + i) * nU + f] =
                        L[((size_t)j * nx + i) * nU + f] -
                        (Gh[(size_t)(j + 1) * nU + f] - Gh[(size_t)j * nU + f]) / dy;
        }
    }
    // explicit source of the one-step model (user source-term path, Sec. 4.3)
    if (ph.model == MODEL_ONESTEP) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const Prim<S>& q = P[E.idx(i, j)];
                L[((size_t)j * nx + i) * nU + 4] =
                    L[((size_t)j * nx + i) * nU + 4] - ph.k * E.u(i, j)[4] * exp(-ph.Ea / q.T);
            }
    }
    return ST_OK;
}

// SSP-RK3 stage combination (Sec. 4.2; Shu-Osher form).
template <class S> S rk_combine(int stage, const S& U0, const S& Us, const S& L, const S& dt) {
    if (stage == 1) return U0 + dt * L;
    if (stage == 2) return 0.75 * U0 + 0.25 * (Us + dt * L);
    return (1.0 / 3.0) * U0 + (2.0 / 3.0) * (Us + dt * L);
}

// Per-cell T after a stage: Newton warm-started from the previous stage's T.
template <class S> int cell_temperature(const Phys<S>& ph, const S* U, const S& Tprev, S& Tout) {
    Tout = Tprev;
    Prim<S> P;
    int st = primitives(ph, U, Tprev, P);
    if (st) return st;
    Tout = P.T;
    return ST_OK;
}

// Jacobian of the production rates S(rho Y_1..rho Y_{Ns-1}) when T follows the
// composition at fixed rho and internal energy e (the "full" variant: species and T).
// Column m is the tangent of S(rhoY, T(rhoY)) along rho Y_m: T comes from Newton on
// dual numbers started at the converged T, so its tangent is the implicit-function
// derivative -(de/d rhoY_m) / (de/dT).
int full_jacobian(const MechData& m, double rho, double e, double T, const double* rhoY,
                  double* J) {
    const int nt = m.ns - 1;
    for (int mm = 0; mm < nt; ++mm) {
        Dual ry[32], Y[32], w[32];
        Dual sum = 0.0;
        for (int k = 0; k < nt; ++k) {
            ry[k] = Dual(rhoY[k], k == mm ? 1.0 : 0.0);
            Y[k] = ry[k] / Dual(rho);
            sum = sum + Y[k];
        }
        Y[nt] = 1.0 - sum;
        Dual Td(T, 0.0);
        int st = newton_T(m, Y, Dual(e), Td);
        if (st) return st;
        production(m, Dual(rho), Td, ry, w, (Dual*)nullptr);
        for (int k = 0; k < nt; ++k) J[k * nt + mm] = w[k].d;
    }
    return ST_OK;
}

// Chemistry step of one cell (DETAILED), then Newton for the new T.
template <class S> int cell_chemistry(const Phys<S>& ph, S* U, S& T, const S& dt) {
    const MechData& m = *ph.mech;
    int st;
    if constexpr (std::is_same<S, double>::value) {
        if (ph.full_jac) {
            const int nt = m.ns - 1;
            std::vector<double> Jf((size_t)nt * nt);
            const double u = U[1] / U[0], v = U[2] / U[0];
            const double e = U[3] / U[0] - 0.5 * (u * u + v * v);
            st = full_jacobian(m, U[0], e, T, &U[4], Jf.data());
            if (!st) st = point_implicit(m, U[0], T, &U[4], dt, Jf.data());
        } else {
            st = point_implicit(m, U[0], T, &U[4], dt);
        }
    } else {
        if (ph.full_jac) return ST_EINVAL;
        st = point_implicit(m, U[0], T, &U[4], dt);
    }
    if (st) return st;
    S Tn = 0.0;
    st = cell_temperature(ph, U, T, Tn);
    T = Tn;
    return st;
}

// ------------------------------------------------------------------ uniform grid
struct GridCfg {
    int nx, ny;
    double dx, dy;
    int bc[4];
};

template <class S> struct BCStates {
    std::vector<S> U[4];
    S T[4];
};

template <class S>
void fill_uniform(const GridCfg& g, const Phys<S>& ph, const S* U, const S* T,
                  const BCStates<S>& bcs, Ext<S>& E) {
    const int nU = ph.nU, nx = g.nx, ny = g.ny;
    auto put = [&](int i, int j, int si, int sj, int negdir) {
        const S* src = &U[((size_t)sj * nx + si) * nU];
        S* dst = E.u(i, j);
        for (int f = 0; f < nU; ++f) dst[f] = src[f];
        if (negdir >= 0) dst[1 + negdir] = -dst[1 + negdir];
        E.t(i, j) = T[(size_t)sj * nx + si];
    };
    auto put_bc = [&](int i, int j, int side) {
        S* dst = E.u(i, j);
        for (int f = 0; f < nU; ++f) dst[f] = bcs.U[side][f];
        E.t(i, j) = bcs.T[side];
    };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) put(i, j, i, j, -1);
    for (int j = 0; j < ny; ++j)
        for (int gg = 1; gg <= 3; ++gg) {
            // west ghost i = -gg
            switch (g.bc[SIDE_W]) {
                case BC_PERIODIC: put(-gg, j, ((nx - gg) % nx + nx) % nx, j, -1); break;
                case BC_ZEROGRAD: put(-gg, j, 0, j, -1); break;
                case BC_SLIPWALL: put(-gg, j, std::min(gg - 1, nx - 1), j, 0); break;
                default: put_bc(-gg, j, SIDE_W);
            }
            switch (g.bc[SIDE_E]) {
                case BC_PERIODIC: put(nx - 1 + gg, j, (gg - 1) % nx, j, -1); break;
                case BC_ZEROGRAD: put(nx - 1 + gg, j, nx - 1, j, -1); break;
                case BC_SLIPWALL: put(nx - 1 + gg, j, std::max(nx - gg, 0), j, 0); break;
                default: put_bc(nx - 1 + gg, j, SIDE_E);
            }
        }
    if (E.gy == 0) return;
    for (int i = 0; i < nx; ++i)
        for (int gg = 1; gg <= 3; ++gg) {
            switch (g.bc[SIDE_S]) {
                case BC_PERIODIC: put(i, -gg, i, ((ny - gg) % ny + ny) % ny, -1); break;
                case BC_ZEROGRAD: put(i, -gg, i, 0, -1); break;
                case BC_SLIPWALL: put(i, -gg, i, std::min(gg - 1, ny - 1), 1); break;
                default: put_bc(i, -gg, SIDE_S);
            }
            switch (g.bc[SIDE_N]) {
                case BC_PERIODIC: put(i, ny - 1 + gg, i, (gg - 1) % ny, -1); break;
                case BC_ZEROGRAD: put(i, ny - 1 + gg, i, ny - 1, -1); break;
                case BC_SLIPWALL: put(i, ny - 1 + gg, i, std::max(ny - gg, 0), 1); break;
                default: put_bc(i, ny - 1 + gg, SIDE_N);
            }
        }
}

// Global alpha (Eq. 4.11) over interior cells; max keeps the first (lowest-index) maximum.
template <class S>
int alphas_uniform(const GridCfg& g, const Phys<S>& ph, const S* U, const S* T, S& ax, S& ay,
                   S& cflmax) {
    const int n = g.nx * g.ny;
    std::vector<Prim<S>> P(n);
    int status = ST_OK;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < n; ++c) {
        int st = primitives(ph, &U[(size_t)c * ph.nU], T[c], P[c]);
        if (st) {
#pragma omp critical
            status = st;
        }
    }
    if (status) return status;
    ax = fabs(P[0].u) + P[0].c;
    ay = fabs(P[0].v) + P[0].c;
    S s0 = ax / g.dx + ((g.ny > 1) ? ay / g.dy : S(0.0));
    cflmax = s0;
    for (int c = 1; c < n; ++c) {
        S sx = fabs(P[c].u) + P[c].c, sy = fabs(P[c].v) + P[c].c;
        if (val(sx) > val(ax)) ax = sx;
        if (val(sy) > val(ay)) ay = sy;
        S s = sx / g.dx + ((g.ny > 1) ? sy / g.dy : S(0.0));
        if (val(s) > val(cflmax)) cflmax = s;
    }
    return ST_OK;
}

template <class S>
int rhs_uniform(const GridCfg& g, const Phys<S>& ph, const S* U, const S* T, const BCStates<S>& bcs,
                std::vector<S>& L) {
    S ax, ay, cm;
    int st = alphas_uniform(g, ph, U, T, ax, ay, cm);
    if (st) return st;
    const int nU = ph.nU;
    // split the grid into row bands so that the ghost-extended copies stay small
    Ext<S> E;
    E.init(nU, g.nx, g.ny);
    fill_uniform(g, ph, U, T, bcs, E);
    return rhs_ext(ph, E, ax, ay, g.dx, g.dy, L);
}

// split = 0: chemistry over dt after the RK stages (Lie, the order of the paper's
// advance_one_step listing); 1: over dt/2 before and after them (Strang, Sec. 4.2).
struct TimeCfg { double cfl, dt_fixed, t_end; int split; };

template <class S>
int choose_dt(const TimeCfg& tc, const S& cflmax, double t, S& dt) {
    if (tc.dt_fixed > 0.0) dt = S(tc.dt_fixed);
    else dt = tc.cfl / cflmax;
    if (tc.t_end > 0.0) {
        double rem = tc.t_end - t;
        if (rem <= 0.0) { dt = S(0.0); return ST_OK; }
        if (val(dt) > rem) dt = S(rem);
    }
    return ST_OK;
}

// Chemistry over dt on every cell of a uniform grid (AoS state).
template <class S>
int chemistry_cells(const Phys<S>& ph, int n, std::vector<S>& U, std::vector<S>& T, const S& dt) {
    int status = ST_OK;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < n; ++c) {
        int s2 = cell_chemistry(ph, &U[(size_t)c * ph.nU], T[c], dt);
        if (s2) {
#pragma omp critical
            status = s2;
        }
    }
    return status;
}

// One full step on a uniform grid: dt from the state at the step start, RK3 flux
// update, chemistry (DETAILED) after it (Lie) or half before and half after (Strang).
template <class S>
int step_uniform(const GridCfg& g, const Phys<S>& ph, const TimeCfg& tc, const BCStates<S>& bcs,
                 std::vector<S>& U, std::vector<S>& T, double& t, double* dt_used,
                 std::vector<S>* probe_dt = nullptr) {
    const int nU = ph.nU, n = g.nx * g.ny;
    S ax, ay, cm;
    int st = alphas_uniform(g, ph, U.data(), T.data(), ax, ay, cm);
    if (st) return st;
    S dt;
    choose_dt(tc, cm, t, dt);
    if (dt_used) *dt_used = val(dt);
    if (probe_dt) probe_dt->assign(1, dt);
    if (!(val(dt) > 0.0)) return ST_OK;
    // chemistry interval: dt (Lie) or dt/2 on both sides of the stages (Strang)
    const bool strang = tc.split == 1 && ph.model == MODEL_DETAILED;
    const S dtc = strang ? S(0.5) * dt : dt;
    if (strang) {
        st = chemistry_cells(ph, n, U, T, dtc);
        if (st) return st;
    }
    std::vector<S> U0 = U, Us = U, Ts = T, L, Un((size_t)n * nU), Tn(n);
    for (int stage = 1; stage <= 3; ++stage) {
        st = rhs_uniform(g, ph, Us.data(), Ts.data(), bcs, L);
        if (st) return st;
        int status = ST_OK;
#pragma omp parallel for schedule(static)
        for (int c = 0; c < n; ++c) {
            for (int f = 0; f < nU; ++f)
                Un[(size_t)c * nU + f] = rk_combine(stage, U0[(size_t)c * nU + f],
                                                    Us[(size_t)c * nU + f],
                                                    L[(size_t)c * nU + f], dt);
            int s2 = cell_temperature(ph, &Un[(size_t)c * nU], Ts[c], Tn[c]);
            if (s2) {
#pragma omp critical
                status = s2;
            }
        }
        if (status) return status;
        std::swap(Us, Un);
        std::swap(Ts, Tn);
    }
    if (ph.model == MODEL_DETAILED) {
        st = chemistry_cells(ph, n, Us, Ts, dtc);
        if (st) return st;
    }
    U.swap(Us);
    T.swap(Ts);
    t += val(dt);
    return ST_OK;
}

// ------------------------------------------------------------------ block tables
struct BlockRec {
    int domain, level, i0, j0, nx, ny;
    long long offset;
    int valid, pad;
};

struct DomainRec {
    int nx, ny;
    double dx, dy;
    int bc[4];
    int nlevels;
    double gamma, R, Q, Ea, k;
};

struct DomainGeo {
    int nlevels;
    std::vector<std::vector<int>> cover;   // per level, dense block-id map (-1 = uncovered)
    std::vector<int> lw, lh;               // level dimensions
};

struct BlockSet {
    std::vector<DomainRec> dom;
    std::vector<BlockRec> blk;
    std::vector<DomainGeo> geo;
    std::vector<std::vector<char>> ring;   // per block, per cell
    long long pool = 0;
    int nU = 0;
};

// wrap a level coordinate through periodic sides; returns false if outside a non-periodic side
inline bool wrap_inside(const DomainRec& d, int lw, int lh, int& I, int& J) {
    if (I < 0 || I >= lw) {
        if (d.bc[SIDE_W] != BC_PERIODIC) return false;
        I = ((I % lw) + lw) % lw;
    }
    if (J < 0 || J >= lh) {
        if (d.bc[SIDE_S] != BC_PERIODIC) return false;
        J = ((J % lh) + lh) % lh;
    }
    return true;
}

int build_blockset(BlockSet& B) {
    const int nd = (int)B.dom.size();
    B.geo.assign(nd, DomainGeo());
    for (int d = 0; d < nd; ++d) {
        const DomainRec& D = B.dom[d];
        if (D.nlevels < 1 || D.nlevels > 8) return ST_EINVAL;
        if (D.nlevels > 1 && D.ny < 2) return ST_EINVAL;
        DomainGeo& G = B.geo[d];
        G.nlevels = D.nlevels;
        G.cover.resize(D.nlevels);
        for (int l = 0; l < D.nlevels; ++l) {
            G.lw.push_back(D.nx << l);
            G.lh.push_back(D.ny > 1 ? (D.ny << l) : 1);
            G.cover[l].assign((size_t)G.lw[l] * G.lh[l], -1);
        }
    }
    for (int b = 0; b < (int)B.blk.size(); ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid) continue;
        if (r.domain < 0 || r.domain >= nd) return ST_EINVAL;
        DomainGeo& G = B.geo[r.domain];
        if (r.level < 0 || r.level >= G.nlevels) return ST_EINVAL;
        int lw = G.lw[r.level], lh = G.lh[r.level];
        if (r.nx < 1 || r.ny < 1 || r.i0 < 0 || r.j0 < 0 || r.i0 + r.nx > lw || r.j0 + r.ny > lh)
            return ST_EINVAL;
        if (r.offset < 0 || r.offset + (long long)r.nx * r.ny > B.pool) return ST_EINVAL;
        for (int j = 0; j < r.ny; ++j)
            for (int i = 0; i < r.nx; ++i) {
                int& c = G.cover[r.level][(size_t)(r.j0 + j) * lw + (r.i0 + i)];
                if (c >= 0) return ST_EINVAL;    // overlapping blocks
                c = b;
            }
    }
    for (int d = 0; d < nd; ++d)
        for (int c : B.geo[d].cover[0])
            if (c < 0) return ST_EINVAL;         // level 0 must tile the domain
    // ring cells (coarse-fine "external boundary" layers, Sec. 3.1.4)
    B.ring.assign(B.blk.size(), std::vector<char>());
    for (int b = 0; b < (int)B.blk.size(); ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid) continue;
        B.ring[b].assign((size_t)r.nx * r.ny, 0);
        if (r.level == 0) continue;
        const DomainRec& D = B.dom[r.domain];
        const DomainGeo& G = B.geo[r.domain];
        int lw = G.lw[r.level], lh = G.lh[r.level];
        for (int j = 0; j < r.ny; ++j)
            for (int i = 0; i < r.nx; ++i) {
                bool ring = false;
                for (int dd = 1; dd <= 3 && !ring; ++dd) {
                    const int off[4][2] = {{-dd, 0}, {dd, 0}, {0, -dd}, {0, dd}};
                    for (int q = 0; q < 4 && !ring; ++q) {
                        int I = r.i0 + i + off[q][0], J = r.j0 + j + off[q][1];
                        if (!wrap_inside(D, lw, lh, I, J)) continue;
                        if (G.cover[r.level][(size_t)J * lw + I] < 0) ring = true;
                    }
                }
                B.ring[b][(size_t)j * r.nx + i] = ring ? 1 : 0;
            }
    }
    // proper nesting: every coarse parent of a fine block is covered one level down
    for (int b = 0; b < (int)B.blk.size(); ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid || r.level == 0) continue;
        if ((r.i0 | r.j0 | r.nx | r.ny) & 1) return ST_EINVAL;
        const DomainGeo& G = B.geo[r.domain];
        int cw = G.lw[r.level - 1];
        for (int j = 0; j < r.ny; j += 2)
            for (int i = 0; i < r.nx; i += 2)
                if (G.cover[r.level - 1][(size_t)((r.j0 + j) >> 1) * cw + ((r.i0 + i) >> 1)] < 0)
                    return ST_EINVAL;
    }
    return ST_OK;
}

struct Src {
    long long cell = -1;   // pool cell, or -1 for a Dirichlet state
    int side = -1;         // Dirichlet side
    int negx = 0, negy = 0;
    int level = -1;        // level of the source cell
};

// Effective value of level-l cell (I, J): boundary rule, then the same-level
// block that covers it, or the injection of the coarser level when it is
// uncovered or a ring cell.
int resolve(const BlockSet& B, int d, int l, int I, int J, Src& s) {
    const DomainRec& D = B.dom[d];
    const DomainGeo& G = B.geo[d];
    int lw = G.lw[l], lh = G.lh[l];
    s = Src();
    if (I < 0 || I >= lw) {
        int side = (I < 0) ? SIDE_W : SIDE_E;
        switch (D.bc[side]) {
            case BC_PERIODIC: I = ((I % lw) + lw) % lw; break;
            case BC_ZEROGRAD: I = (I < 0) ? 0 : lw - 1; break;
            case BC_SLIPWALL: I = (I < 0) ? -I - 1 : 2 * lw - 1 - I; s.negx ^= 1; break;
            default: s.side = side; return ST_OK;
        }
    }
    if (J < 0 || J >= lh) {
        int side = (J < 0) ? SIDE_S : SIDE_N;
        switch (D.bc[side]) {
            case BC_PERIODIC: J = ((J % lh) + lh) % lh; break;
            case BC_ZEROGRAD: J = (J < 0) ? 0 : lh - 1; break;
            case BC_SLIPWALL: J = (J < 0) ? -J - 1 : 2 * lh - 1 - J; s.negy ^= 1; break;
            default: s.side = side; return ST_OK;
        }
    }
    for (;;) {
        lw = G.lw[l];
        int b = G.cover[l][(size_t)J * lw + I];
        if (b >= 0) {
            const BlockRec& r = B.blk[b];
            int li = I - r.i0, lj = J - r.j0;
            if (!B.ring[b][(size_t)lj * r.nx + li]) {
                s.cell = r.offset + (long long)lj * r.nx + li;
                s.level = l;
                return ST_OK;
            }
        }
        if (l == 0) return ST_EINVAL;
        --l;
        I >>= 1;
        J >>= 1;
    }
}

template <class S>
void load_src(const BlockSet& B, int d, const Src& s, const std::vector<std::vector<S>>& bcU,
              const std::vector<S>& bcT, const S* U, const S* T, long long pool, S* out, S& Tout) {
    const int nU = B.nU;
    if (s.cell < 0) {
        for (int f = 0; f < nU; ++f) out[f] = bcU[d * 4 + s.side][f];
        Tout = bcT[d * 4 + s.side];
        return;
    }
    for (int f = 0; f < nU; ++f) out[f] = U[(size_t)f * pool + s.cell];
    if (s.negx) out[1] = -out[1];
    if (s.negy) out[2] = -out[2];
    Tout = T[s.cell];
}

// Four-to-one restriction finest level first (Alg. 2 interpolate_fine_to_coarse), then
// the ring cells of every refined level take the injection of the restricted coarser
// level. Domains whose dt is 0 are left alone.
template <class S>
int restrict_and_refill(const BlockSet& B, const std::vector<Phys<S>>& phys,
                        const std::vector<std::vector<S>>& bcU, const std::vector<S>& bcT,
                        std::vector<S>& Uout, std::vector<S>& Tout, const std::vector<S>& dt) {
    const int nU = B.nU;
    const long long pool = B.pool;
    const int nd = (int)B.dom.size(), nb = (int)B.blk.size();
    auto solved = [&](int b, int i, int j) { return !B.ring[b][(size_t)j * B.blk[b].nx + i]; };
    // restriction, finest level first: a covered coarse cell becomes the mean of its 4 children
    int maxlev = 0;
    for (int d = 0; d < nd; ++d) maxlev = std::max(maxlev, B.dom[d].nlevels - 1);
    for (int lev = maxlev; lev >= 1; --lev) {
        struct Upd { long long cell; int dom; std::vector<S> u; };
        std::vector<Upd> upd;
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid || r.level != lev) continue;
            const int d = r.domain;
            if (!(val(dt[d]) > 0.0)) continue;
            const DomainGeo& G = B.geo[d];
            int cw = G.lw[lev - 1];
            for (int cj = r.j0 / 2; cj < (r.j0 + r.ny) / 2; ++cj)
                for (int ci = r.i0 / 2; ci < (r.i0 + r.nx) / 2; ++ci) {
                    S ch[4][64];
                    S Tch;
                    for (int q = 0; q < 4; ++q) {
                        Src s;
                        if (resolve(B, d, lev, 2 * ci + (q & 1), 2 * cj + (q >> 1), s)) return ST_EINVAL;
                        load_src(B, d, s, bcU, bcT, Uout.data(), Tout.data(), pool, ch[q], Tch);
                    }
                    Upd u;
                    int cb = G.cover[lev - 1][(size_t)cj * cw + ci];
                    const BlockRec& cr = B.blk[cb];
                    u.cell = cr.offset + (long long)(cj - cr.j0) * cr.nx + (ci - cr.i0);
                    u.dom = d;
                    u.u.resize(nU);
                    for (int f = 0; f < nU; ++f)
                        u.u[f] = ((ch[0][f] + ch[1][f]) + (ch[2][f] + ch[3][f])) * 0.25;
                    upd.push_back(u);
                }
        }
        // all means are formed from pre-restriction values before any coarse cell changes
        for (size_t q = 0; q < upd.size(); ++q) {
            long long c = upd[q].cell;
            for (int f = 0; f < nU; ++f) Uout[(size_t)f * pool + c] = upd[q].u[f];
        }
        // T of restricted cells is re-solved, warm-started from the coarse cell's T
        for (size_t q = 0; q < upd.size(); ++q) {
            long long c = upd[q].cell;
            S Tn = 0.0;
            int st = cell_temperature(phys[upd[q].dom], upd[q].u.data(), Tout[c], Tn);
            if (st) return st;
            Tout[c] = Tn;
        }
    }
    // ring cells take the injection of the (restricted) coarser level
    for (int lev = 1; lev <= maxlev; ++lev) {
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid || r.level != lev || !(val(dt[r.domain]) > 0.0)) continue;
            for (int j = 0; j < r.ny; ++j)
                for (int i = 0; i < r.nx; ++i) {
                    if (solved(b, i, j)) continue;
                    Src s;
                    if (resolve(B, r.domain, lev - 1, (r.i0 + i) >> 1, (r.j0 + j) >> 1, s)) return ST_EINVAL;
                    S u[64], Tv;
                    load_src(B, r.domain, s, bcU, bcT, Uout.data(), Tout.data(), pool, u, Tv);
                    long long c = r.offset + (long long)j * r.nx + i;
                    for (int f = 0; f < nU; ++f) Uout[(size_t)f * pool + c] = u[f];
                    Tout[c] = Tv;
                }
        }
    }
    return ST_OK;
}

template <class S>
int step_blocks(BlockSet& B, const std::vector<Phys<S>>& phys, const TimeCfg& tc,
                const std::vector<std::vector<S>>& bcU, const std::vector<S>& bcT,
                std::vector<S>& Upool, std::vector<S>& Tpool, std::vector<double>& t,
                double* dt_out) {
    const int nU = B.nU;
    const long long pool = B.pool;
    const int nd = (int)B.dom.size(), nb = (int)B.blk.size();
    std::vector<S> dt(nd);
    std::vector<Prim<S>> Pc((size_t)pool);   // primitives of solved cells
    // the three stage inputs U^(0), U^(1), U^(2) live in separate pool arrays (SoA: field-major)
    std::vector<S> U1((size_t)pool * nU), U2((size_t)pool * nU), T1(pool), T2(pool);
    std::vector<S> Uout = Upool, Tout = Tpool;
    int status = ST_OK;

    auto solved = [&](int b, int i, int j) { return !B.ring[b][(size_t)j * B.blk[b].nx + i]; };

    // prims of all solved cells of a stage state; per (domain, level) alpha and per-domain cfl
    auto reductions = [&](const std::vector<S>& Us, const std::vector<S>& Ts,
                          std::vector<S>& ax, std::vector<S>& ay, std::vector<S>& cm,
                          std::vector<char>& have) -> int {
        int st = ST_OK;
#pragma omp parallel for schedule(dynamic)
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid) continue;
            const Phys<S>& ph = phys[r.domain];
            for (int j = 0; j < r.ny; ++j)
                for (int i = 0; i < r.nx; ++i) {
                    if (!solved(b, i, j)) continue;
                    long long c = r.offset + (long long)j * r.nx + i;
                    S u[64];
                    for (int f = 0; f < nU; ++f) u[f] = Us[(size_t)f * pool + c];
                    int s2 = primitives(ph, u, Ts[c], Pc[c]);
                    if (s2) {
#pragma omp critical
                        st = s2;
                    }
                }
        }
        if (st) return st;
        const int L = 8;
        ax.assign((size_t)nd * L, S(0.0));
        ay.assign((size_t)nd * L, S(0.0));
        cm.assign(nd, S(0.0));
        have.assign((size_t)nd * L, 0);
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid) continue;
            const DomainRec& D = B.dom[r.domain];
            double dxl = D.dx / (1 << r.level), dyl = D.dy / (1 << r.level);
            int slot = r.domain * L + r.level;
            for (int j = 0; j < r.ny; ++j)
                for (int i = 0; i < r.nx; ++i) {
                    if (!solved(b, i, j)) continue;
                    const Prim<S>& P = Pc[r.offset + (long long)j * r.nx + i];
                    S sx = fabs(P.u) + P.c, sy = fabs(P.v) + P.c;
                    S s = sx / dxl + ((D.ny > 1) ? sy / dyl : S(0.0));
                    if (!have[slot]) { ax[slot] = sx; ay[slot] = sy; have[slot] = 1; }
                    else {
                        if (val(sx) > val(ax[slot])) ax[slot] = sx;
                        if (val(sy) > val(ay[slot])) ay[slot] = sy;
                    }
                    if (val(s) > val(cm[r.domain])) cm[r.domain] = s;
                }
        }
        return ST_OK;
    };

    std::vector<S> ax, ay, cm;
    std::vector<char> have;
    status = reductions(Upool, Tpool, ax, ay, cm, have);
    if (status) return status;
    for (int d = 0; d < nd; ++d) {
        choose_dt(tc, cm[d], t[d], dt[d]);
        if (dt_out) dt_out[d] = val(dt[d]);
    }
    // chemistry on the solved cells of every valid block over f * dt (DETAILED)
    auto chemistry = [&](std::vector<S>& Uc, std::vector<S>& Tc, double f) -> int {
        int status2 = ST_OK;
#pragma omp parallel for schedule(dynamic)
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid || !(val(dt[r.domain]) > 0.0)) continue;
            const S dtc = f * dt[r.domain];
            for (int j = 0; j < r.ny; ++j)
                for (int i = 0; i < r.nx; ++i) {
                    if (!solved(b, i, j)) continue;
                    long long c = r.offset + (long long)j * r.nx + i;
                    S u[64];
                    for (int f2 = 0; f2 < nU; ++f2) u[f2] = Uc[(size_t)f2 * pool + c];
                    int st = cell_chemistry(phys[r.domain], u, Tc[c], dtc);
                    for (int f2 = 0; f2 < nU; ++f2) Uc[(size_t)f2 * pool + c] = u[f2];
                    if (st) {
#pragma omp critical
                        status2 = st;
                    }
                }
        }
        return status2;
    };
    const bool detailed = B.nU > 0 && phys[0].model == MODEL_DETAILED;
    const bool strang = detailed && tc.split == 1;
    if (strang) {
        // first half; stage 1's alpha from the state it leaves
        status = chemistry(Upool, Tpool, 0.5);
        if (!status) status = reductions(Upool, Tpool, ax, ay, cm, have);
        if (status) return status;
    }

    const std::vector<S>* Uin = &Upool;
    const std::vector<S>* Tin = &Tpool;
    for (int stage = 1; stage <= 3; ++stage) {
        if (stage > 1) {
            status = reductions(*Uin, *Tin, ax, ay, cm, have);
            if (status) return status;
        }
        std::vector<S>& Udst = (stage == 1) ? U1 : (stage == 2) ? U2 : Uout;
        std::vector<S>& Tdst = (stage == 1) ? T1 : (stage == 2) ? T2 : Tout;
#pragma omp parallel for schedule(dynamic)
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid) continue;
            const int d = r.domain;
            if (!(val(dt[d]) > 0.0)) {
                // a finished domain keeps its state
                for (int j = 0; j < r.ny; ++j)
                    for (int i = 0; i < r.nx; ++i) {
                        long long c = r.offset + (long long)j * r.nx + i;
                        for (int f = 0; f < nU; ++f) Udst[(size_t)f * pool + c] = (*Uin)[(size_t)f * pool + c];
                        Tdst[c] = (*Tin)[c];
                    }
                continue;
            }
            const Phys<S>& ph = phys[d];
            const DomainRec& D = B.dom[d];
            Ext<S> E;
            E.init(nU, r.nx, (D.ny > 1) ? r.ny : 1);
            int st = ST_OK;
            for (int j = -E.gy; j < r.ny + E.gy && !st; ++j)
                for (int i = -E.g; i < r.nx + E.g && !st; ++i) {
                    if (!E.in_cross(i, j)) continue;
                    Src s;
                    st = resolve(B, d, r.level, r.i0 + i, r.j0 + j, s);
                    if (!st) load_src(B, d, s, bcU, bcT, Uin->data(), Tin->data(), pool, E.u(i, j), E.t(i, j));
                }
            std::vector<S> L;
            int slot = d * 8 + r.level;
            if (!st) st = rhs_ext(ph, E, ax[slot], ay[slot], D.dx / (1 << r.level),
                                  D.dy / (1 << r.level), L);
            if (!st) {
                for (int j = 0; j < r.ny && !st; ++j)
                    for (int i = 0; i < r.nx && !st; ++i) {
                        if (!solved(b, i, j)) continue;
                        long long c = r.offset + (long long)j * r.nx + i;
                        S un[64];
                        for (int f = 0; f < nU; ++f) {
                            S u0 = Upool[(size_t)f * pool + c];
                            S us = (*Uin)[(size_t)f * pool + c];
                            un[f] = rk_combine(stage, u0, us, L[((size_t)j * r.nx + i) * nU + f], dt[d]);
                            Udst[(size_t)f * pool + c] = un[f];
                        }
                        S Tn = 0.0;
                        st = cell_temperature(ph, un, (*Tin)[c], Tn);
                        Tdst[c] = Tn;
                    }
            }
            if (st) {
#pragma omp critical
                status = st;
            }
        }
        if (status) return status;
        Uin = &Udst;
        Tin = &Tdst;
    }
    if (detailed) {
        status = chemistry(Uout, Tout, strang ? 0.5 : 1.0);
        if (status) return status;
    }
    status = restrict_and_refill(B, phys, bcU, bcT, Uout, Tout, dt);
    if (status) return status;
    Upool.swap(Uout);
    Tpool.swap(Tout);
    for (int d = 0; d < nd; ++d) t[d] += val(dt[d]);
    return ST_OK;
}

// Wave-speed maxima over the solved cells of the valid blocks of one level (all levels
// when lev < 0) of a state: alpha_x, alpha_y per (domain, level) (Eq. 4.11) and the
// per-domain CFL bound max((|u|+c)/dx + (|v|+c)/dy), with the spacing of level 0 when
// spacing0 is set, else each block's own level spacing.
template <class S>
int level_maxima(const BlockSet& B, const std::vector<Phys<S>>& phys, const S* Us, const S* Ts,
                 int lev, bool spacing0, std::vector<S>& ax, std::vector<S>& ay,
                 std::vector<S>& cm) {
    const int nU = B.nU, nd = (int)B.dom.size(), nb = (int)B.blk.size();
    const long long pool = B.pool;
    const int L = 8;
    ax.assign((size_t)nd * L, S(0.0));
    ay.assign((size_t)nd * L, S(0.0));
    cm.assign(nd, S(0.0));
    for (int b = 0; b < nb; ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid || (lev >= 0 && r.level != lev)) continue;
        const DomainRec& D = B.dom[r.domain];
        const int sl = spacing0 ? 0 : r.level;
        const double dxl = D.dx / (1 << sl), dyl = D.dy / (1 << sl);
        const int slot = r.domain * L + r.level;
        for (int j = 0; j < r.ny; ++j)
            for (int i = 0; i < r.nx; ++i) {
                if (B.ring[b][(size_t)j * r.nx + i]) continue;
                const long long c = r.offset + (long long)j * r.nx + i;
                S u[64];
                for (int f = 0; f < nU; ++f) u[f] = Us[(size_t)f * pool + c];
                Prim<S> P;
                const int st = primitives(phys[r.domain], u, Ts[c], P);
                if (st) return st;
                const S sx = fabs(P.u) + P.c, sy = fabs(P.v) + P.c;
                const S sc = sx / dxl + ((D.ny > 1) ? sy / dyl : S(0.0));
                if (val(sx) > val(ax[slot])) ax[slot] = sx;
                if (val(sy) > val(ay[slot])) ay[slot] = sy;
                if (val(sc) > val(cm[r.domain])) cm[r.domain] = sc;
            }
    }
    return ST_OK;
}

// One step of the crossover advance (Fig. 2a, Alg. 2): the deepest level first; every
// two steps of a level are followed by one step of the next coarser level, and each
// level's time step is half that of the coarser one, dt_l = dt_0 / 2^l. dt_0 keeps every
// level within the CFL bound: dt_0 = CFL / max over all levels' solved cells of
// (|u|+c)/dx_0 + (|v|+c)/dy_0. While a level advances, the coarser levels hold their
// current states: halo cells of the level that are uncovered there, and its ring cells,
// take the injection of that current coarser state at every RK stage. After the level-0
// step every level is at t + dt_0; then the four-to-one restriction and the ring refill
// of the synchronous advance.
template <class S>
int step_blocks_crossover(BlockSet& B, const std::vector<Phys<S>>& phys, const TimeCfg& tc,
                          const std::vector<std::vector<S>>& bcU, const std::vector<S>& bcT,
                          std::vector<S>& Upool, std::vector<S>& Tpool, std::vector<double>& t,
                          double* dt_out) {
    const int nU = B.nU;
    const long long pool = B.pool;
    const int nd = (int)B.dom.size(), nb = (int)B.blk.size();
    std::vector<S> ax, ay, cm;
    int status = level_maxima(B, phys, Upool.data(), Tpool.data(), -1, true, ax, ay, cm);
    if (status) return status;
    std::vector<S> dt0(nd);
    for (int d = 0; d < nd; ++d) {
        choose_dt(tc, cm[d], t[d], dt0[d]);
        if (dt_out) dt_out[d] = val(dt0[d]);
    }
    int maxlev = 0;
    for (int d = 0; d < nd; ++d) maxlev = std::max(maxlev, B.dom[d].nlevels - 1);
    std::vector<S> U1((size_t)pool * nU), U2((size_t)pool * nU), T1(pool), T2(pool);

    // one RK3 step (and chemistry) of the blocks of level lev, time step dt_0 / 2^lev
    auto advance_level = [&](int lev) -> int {
        std::vector<S> dtl(nd);
        for (int d = 0; d < nd; ++d) dtl[d] = dt0[d] * std::ldexp(1.0, -lev);
        // Strang: the level's first half chemistry step, in place
        const bool strang = tc.split == 1 && nU > 0 && phys[0].model == MODEL_DETAILED;
        if (strang) {
            int status1 = ST_OK;
#pragma omp parallel for schedule(dynamic)
            for (int b = 0; b < nb; ++b) {
                const BlockRec& r = B.blk[b];
                if (!r.valid || r.level != lev || !(val(dtl[r.domain]) > 0.0)) continue;
                const S dtc = 0.5 * dtl[r.domain];
                for (int j = 0; j < r.ny; ++j)
                    for (int i = 0; i < r.nx; ++i) {
                        if (B.ring[b][(size_t)j * r.nx + i]) continue;
                        const long long c = r.offset + (long long)j * r.nx + i;
                        S u[64];
                        for (int f = 0; f < nU; ++f) u[f] = Upool[(size_t)f * pool + c];
                        const int st = cell_chemistry(phys[r.domain], u, Tpool[c], dtc);
                        for (int f = 0; f < nU; ++f) Upool[(size_t)f * pool + c] = u[f];
                        if (st) {
#pragma omp critical
                            status1 = st;
                        }
                    }
            }
            if (status1) return status1;
        }
        std::vector<S> Unew = Upool, Tnew = Tpool;
        const std::vector<S>* Uin = &Upool;
        const std::vector<S>* Tin = &Tpool;
        for (int stage = 1; stage <= 3; ++stage) {
            int st = level_maxima(B, phys, Uin->data(), Tin->data(), lev, false, ax, ay, cm);
            if (st) return st;
            std::vector<S>& Udst = (stage == 1) ? U1 : (stage == 2) ? U2 : Unew;
            std::vector<S>& Tdst = (stage == 1) ? T1 : (stage == 2) ? T2 : Tnew;
            int status2 = ST_OK;
#pragma omp parallel for schedule(dynamic)
            for (int b = 0; b < nb; ++b) {
                const BlockRec& r = B.blk[b];
                if (!r.valid || r.level != lev) continue;
                const int d = r.domain;
                if (!(val(dtl[d]) > 0.0)) {
                    for (long long c = r.offset; c < r.offset + (long long)r.nx * r.ny; ++c) {
                        for (int f = 0; f < nU; ++f) Udst[(size_t)f * pool + c] = (*Uin)[(size_t)f * pool + c];
                        Tdst[c] = (*Tin)[c];
                    }
                    continue;
                }
                const Phys<S>& ph = phys[d];
                const DomainRec& D = B.dom[d];
                Ext<S> E;
                E.init(nU, r.nx, (D.ny > 1) ? r.ny : 1);
                int st2 = ST_OK;
                for (int j = -E.gy; j < r.ny + E.gy && !st2; ++j)
                    for (int i = -E.g; i < r.nx + E.g && !st2; ++i) {
                        if (!E.in_cross(i, j)) continue;
                        Src sr;
                        st2 = resolve(B, d, lev, r.i0 + i, r.j0 + j, sr);
                        if (st2) break;
                        // this level's cells at the stage; coarser levels at their current state
                        const bool same = sr.cell >= 0 && sr.level == lev;
                        load_src(B, d, sr, bcU, bcT, same ? Uin->data() : Upool.data(),
                                 same ? Tin->data() : Tpool.data(), pool, E.u(i, j), E.t(i, j));
                    }
                std::vector<S> L;
                const int slot = d * 8 + lev;
                if (!st2) st2 = rhs_ext(ph, E, ax[slot], ay[slot], D.dx / (1 << lev),
                                        D.dy / (1 << lev), L);
                if (!st2) {
                    for (int j = 0; j < r.ny && !st2; ++j)
                        for (int i = 0; i < r.nx && !st2; ++i) {
                            if (B.ring[b][(size_t)j * r.nx + i]) continue;
                            const long long c = r.offset + (long long)j * r.nx + i;
                            S un[64];
                            for (int f = 0; f < nU; ++f) {
                                const S u0 = Upool[(size_t)f * pool + c];
                                const S us = (*Uin)[(size_t)f * pool + c];
                                un[f] = rk_combine(stage, u0, us, L[((size_t)j * r.nx + i) * nU + f], dtl[d]);
                                Udst[(size_t)f * pool + c] = un[f];
                            }
                            S Tn = 0.0;
                            st2 = cell_temperature(ph, un, (*Tin)[c], Tn);
                            Tdst[c] = Tn;
                        }
                }
                if (st2) {
#pragma omp critical
                    status2 = st2;
                }
            }
            if (status2) return status2;
            Uin = &Udst;
            Tin = &Tdst;
        }
        int status3 = ST_OK;
#pragma omp parallel for schedule(dynamic)
        for (int b = 0; b < nb; ++b) {
            const BlockRec& r = B.blk[b];
            if (!r.valid || r.level != lev || !(val(dtl[r.domain]) > 0.0)) continue;
            for (int j = 0; j < r.ny; ++j)
                for (int i = 0; i < r.nx; ++i) {
                    if (B.ring[b][(size_t)j * r.nx + i]) continue;
                    const long long c = r.offset + (long long)j * r.nx + i;
                    S u[64];
                    for (int f = 0; f < nU; ++f) u[f] = Unew[(size_t)f * pool + c];
                    if (phys[r.domain].model == MODEL_DETAILED) {
                        const S dtc = strang ? 0.5 * dtl[r.domain] : dtl[r.domain];
                        const int st = cell_chemistry(phys[r.domain], u, Tnew[c], dtc);
                        if (st) {
#pragma omp critical
                            status3 = st;
                        }
                    }
                    for (int f = 0; f < nU; ++f) Upool[(size_t)f * pool + c] = u[f];
                    Tpool[c] = Tnew[c];
                }
        }
        return status3;
    };
    // the recursion of Alg. 2: two steps of level l + 1, then one of level l
    struct Rec {
        decltype(advance_level)& adv;
        int maxlev;
        int run(int l) {
            if (l < maxlev) {
                int st = run(l + 1);
                if (!st) st = run(l + 1);
                if (st) return st;
            }
            return adv(l);
        }
    } rec{advance_level, maxlev};
    status = rec.run(0);
    if (status) return status;
    status = restrict_and_refill(B, phys, bcU, bcT, Upool, Tpool, dt0);
    if (status) return status;
    for (int d = 0; d < nd; ++d) t[d] += val(dt0[d]);
    return ST_OK;
}

// ------------------------------------------------------------------ regridding
// Updating the refinement layers (Sec. 3.1.2 and the layer-update and refinement
// operations of Sec. 3.1.4; Alg. 2): level by level, each block of the new layer l
// is divided into fixed subregions of `sub` x `sub` layer-l cells (the last row and
// column may be narrower); a subregion becomes a layer-(l+1) block when a masked
// cell of layer l lies in it or within `buffer` cells of it (the buffer cells).
// A cell is masked by the density-gradient criterion
//     max(|rho(I+1,J) - rho(I-1,J)|, |rho(I,J+1) - rho(I,J-1)|) > 2 threshold rho(I,J)
// on the effective layer-l field of the hierarchy before the update (values of the
// covering layer-l block, else of the coarser layer: the ghost rules of the solver).
// Subregions that contain coarse-fine ring cells of layer l stay unrefined, so
// that refined blocks sit on solved cells. Blocks identical to a block of the old
// table keep their data; new blocks take the one-to-four injection of the new
// coarser layer.
struct RegridCfg { double threshold; int buffer, sub; };

// density of layer-l cell (I, J) on the effective field (boundary rules included)
double effective_density(const BlockSet& B, int d, int l, int I, int J, const double* bc_rho,
                         const double* U) {
    Src s;
    resolve(B, d, l, I, J, s);
    if (s.cell < 0) return bc_rho[d * 4 + s.side];
    return U[s.cell];   // field 0 of the pool is rho
}

bool density_masked(const BlockSet& B, int d, int l, int I, int J, double thr,
                    const double* bc_rho, const double* U) {
    const double r = effective_density(B, d, l, I, J, bc_rho, U);
    const double gx = std::fabs(effective_density(B, d, l, I + 1, J, bc_rho, U) -
                                effective_density(B, d, l, I - 1, J, bc_rho, U));
    const double gy = std::fabs(effective_density(B, d, l, I, J + 1, bc_rho, U) -
                                effective_density(B, d, l, I, J - 1, bc_rho, U));
    return std::max(gx, gy) > 2.0 * thr * r;
}

int regrid_table(const BlockSet& B, const double* bc_rho, const double* U, const RegridCfg& cfg,
                 std::vector<BlockRec>& out) {
    out.clear();
    long long off = 0;
    for (const BlockRec& r : B.blk)
        if (r.valid && r.level == 0) {
            BlockRec n = r;
            n.offset = off;
            off += (long long)r.nx * r.ny;
            out.push_back(n);
        }
    int maxlev = 0;
    for (const DomainRec& D : B.dom) maxlev = std::max(maxlev, D.nlevels - 1);
    for (int l = 0; l < maxlev; ++l) {
        // the new hierarchy up to layer l, for its ring cells
        BlockSet N;
        N.dom = B.dom;
        N.blk = out;
        N.pool = off;
        N.nU = B.nU;
        int st = build_blockset(N);
        if (st) return st;
        const size_t nprev = out.size();
        for (size_t b = 0; b < nprev; ++b) {
            const BlockRec r = out[b];
            if (r.level != l || l + 1 >= B.dom[r.domain].nlevels) continue;
            const int lw = B.geo[r.domain].lw[l], lh = B.geo[r.domain].lh[l];
            for (int y0 = 0; y0 < r.ny; y0 += cfg.sub)
                for (int x0 = 0; x0 < r.nx; x0 += cfg.sub) {
                    const int w = std::min(cfg.sub, r.nx - x0), h = std::min(cfg.sub, r.ny - y0);
                    bool ring = false;
                    for (int j = y0; j < y0 + h && !ring; ++j)
                        for (int i = x0; i < x0 + w && !ring; ++i) ring = N.ring[b][(size_t)j * r.nx + i] != 0;
                    if (ring) continue;
                    bool mask = false;
                    const int I0 = r.i0 + x0, J0 = r.j0 + y0;
                    for (int J = J0 - cfg.buffer; J < J0 + h + cfg.buffer && !mask; ++J)
                        for (int I = I0 - cfg.buffer; I < I0 + w + cfg.buffer && !mask; ++I) {
                            if (I < 0 || I >= lw || J < 0 || J >= lh) continue;
                            mask = density_masked(B, r.domain, l, I, J, cfg.threshold, bc_rho, U);
                        }
                    if (!mask) continue;
                    BlockRec n{};
                    n.domain = r.domain;
                    n.level = l + 1;
                    n.i0 = 2 * I0;
                    n.j0 = 2 * J0;
                    n.nx = 2 * w;
                    n.ny = 2 * h;
                    n.offset = off;
                    n.valid = 1;
                    off += (long long)n.nx * n.ny;
                    out.push_back(n);
                }
        }
    }
    return ST_OK;
}

// Data of the new table: copies of unaltered blocks, injection for new ones.
void regrid_fill(const BlockSet& Bo, const double* Uo, const double* To, const BlockSet& Bn,
                 double* Un, double* Tn) {
    const int nU = Bn.nU;
    for (const BlockRec& r : Bn.blk) {
        const BlockRec* same = nullptr;
        for (const BlockRec& q : Bo.blk)
            if (q.valid && q.domain == r.domain && q.level == r.level && q.i0 == r.i0 &&
                q.j0 == r.j0 && q.nx == r.nx && q.ny == r.ny)
                same = &q;
        for (int j = 0; j < r.ny; ++j)
            for (int i = 0; i < r.nx; ++i) {
                const long long c = r.offset + (long long)j * r.nx + i;
                long long src;
                const double *Us, *Ts;
                long long ps;
                if (same) {
                    src = same->offset + (long long)j * r.nx + i;
                    Us = Uo; Ts = To; ps = Bo.pool;
                } else {
                    // the parent cell on the new coarser layer (already filled)
                    const DomainGeo& G = Bn.geo[r.domain];
                    const int I = (r.i0 + i) >> 1, J = (r.j0 + j) >> 1;
                    const int pb = G.cover[r.level - 1][(size_t)J * G.lw[r.level - 1] + I];
                    const BlockRec& P = Bn.blk[pb];
                    src = P.offset + (long long)(J - P.j0) * P.nx + (I - P.i0);
                    Us = Un; Ts = Tn; ps = Bn.pool;
                }
                for (int f = 0; f < nU; ++f) Un[(size_t)f * Bn.pool + c] = Us[(size_t)f * ps + src];
                Tn[c] = Ts[src];
            }
    }
}

// ------------------------------------------------------------------ C views
struct OMech {
    int ns, nr;
    const double *M, *nasa, *A, *b, *Ea;
    const int *nuf, *nub;
    const double* tb;
    const int *has_tb, *rev;
    const double *nasa_high, *t_mid;   // two-range NASA-7 (both null: one range)
};
struct OPhys { int model; double gamma, R, Q, Ea, k; };
struct OGrid { int nx, ny; double dx, dy; int bc[4]; };
struct OTime { double cfl, dt_fixed, t_end; int split, jac; };

MechData mech_from(const OMech* m) {
    MechData d;
    if (!m) return d;
    d.ns = m->ns; d.nr = m->nr;
    d.M.assign(m->M, m->M + m->ns);
    d.nasa.assign(m->nasa, m->nasa + 7 * m->ns);
    if (m->nasa_high && m->t_mid) {
        d.nasa_hi.assign(m->nasa_high, m->nasa_high + 7 * m->ns);
        d.tmid.assign(m->t_mid, m->t_mid + m->ns);
    }
    d.A.assign(m->A, m->A + m->nr);
    d.b.assign(m->b, m->b + m->nr);
    d.Ea.assign(m->Ea, m->Ea + m->nr);
    d.nuf.assign(m->nuf, m->nuf + m->nr * m->ns);
    d.nub.assign(m->nub, m->nub + m->nr * m->ns);
    d.tb.assign(m->tb, m->tb + m->nr * m->ns);
    d.has_tb.assign(m->has_tb, m->has_tb + m->nr);
    d.rev.assign(m->rev, m->rev + m->nr);
    return d;
}

int n_fields(int model, int ns) {
    return model == MODEL_CPG ? 4 : model == MODEL_ONESTEP ? 5 : 3 + ns;
}

template <class S> Phys<S> phys_from(const OPhys* p, const MechData* m) {
    Phys<S> ph;
    ph.model = p->model;
    ph.gamma = p->gamma; ph.R = p->R; ph.Q = p->Q; ph.Ea = p->Ea; ph.k = p->k;
    ph.mech = m;
    ph.nU = n_fields(p->model, m ? m->ns : 0);
    return ph;
}

GridCfg grid_from(const OGrid* g) {
    GridCfg c;
    c.nx = g->nx; c.ny = g->ny; c.dx = g->dx; c.dy = g->dy;
    for (int q = 0; q < 4; ++q) c.bc[q] = g->bc[q];
    return c;
}

// SoA [nU][n] (x fastest) <-> AoS
template <class S> void soa_to_aos(int nU, long long n, const double* in, std::vector<S>& out) {
    out.resize((size_t)n * nU);
    for (long long c = 0; c < n; ++c)
        for (int f = 0; f < nU; ++f) out[(size_t)c * nU + f] = S(in[(size_t)f * n + c]);
}
template <class S> void aos_to_soa(int nU, long long n, const std::vector<S>& in, double* out) {
    for (long long c = 0; c < n; ++c)
        for (int f = 0; f < nU; ++f) out[(size_t)f * n + c] = val(in[(size_t)c * nU + f]);
}

template <class S>
int bc_states_from(const Phys<S>& ph, const OGrid* g, const double* bc_prim, BCStates<S>& bcs) {
    for (int s = 0; s < 4; ++s) {
        bcs.U[s].assign(ph.nU, S(0.0));
        bcs.T[s] = S(0.0);
        if (g->bc[s] == BC_DIRICHLET) {
            if (!bc_prim) return ST_EINVAL;
            std::vector<S> W(ph.nU);
            for (int f = 0; f < ph.nU; ++f) W[f] = S(bc_prim[s * ph.nU + f]);
            conserved_from_primitive(ph, W.data(), bcs.U[s].data(), bcs.T[s]);
        }
    }
    return ST_OK;
}

// Re-solve T from U with the given T as the warm start (call entry).
template <class S> int resolve_T_all(const Phys<S>& ph, long long n, const std::vector<S>& U,
                                     std::vector<S>& T) {
    int status = ST_OK;
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < n; ++c) {
        S Tn = 0.0;
        int st = cell_temperature(ph, &U[(size_t)c * ph.nU], T[c], Tn);
        T[c] = Tn;
        if (st) {
#pragma omp critical
            status = st;
        }
    }
    return status;
}

}  // namespace

// ================================================================== exported API
extern "C" {

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads() {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_n_fields(int model, int ns) { return n_fields(model, ns); }

// Primitive [nU][n] -> conserved [nU][n] and T[n].
int oracle_init_state(const OPhys* p, const OMech* m, long long n, const double* W, double* U,
                      double* T) {
    MechData md = mech_from(m);
    Phys<double> ph = phys_from<double>(p, m ? &md : nullptr);
    const int nU = ph.nU;
    std::vector<double> w(nU), u(nU);
    for (long long c = 0; c < n; ++c) {
        for (int f = 0; f < nU; ++f) w[f] = W[(size_t)f * n + c];
        double t;
        conserved_from_primitive(ph, w.data(), u.data(), t);
        for (int f = 0; f < nU; ++f) U[(size_t)f * n + c] = u[f];
        T[c] = t;
    }
    return ST_OK;
}

// Primitive (rho, u, v, p, T, c) per cell from conserved U (SoA), T as Newton warm start.
int oracle_primitives(const OPhys* p, const OMech* m, long long n, const double* U,
                      const double* Tguess, double* out /* [6][n] */) {
    MechData md = mech_from(m);
    Phys<double> ph = phys_from<double>(p, m ? &md : nullptr);
    std::vector<double> u(ph.nU);
    for (long long c = 0; c < n; ++c) {
        for (int f = 0; f < ph.nU; ++f) u[f] = U[(size_t)f * n + c];
        Prim<double> P;
        int st = primitives(ph, u.data(), Tguess[c], P);
        if (st) return st;
        double v[6] = {P.rho, P.u, P.v, P.p, P.T, P.c};
        for (int q = 0; q < 6; ++q) out[(size_t)q * n + c] = v[q];
    }
    return ST_OK;
}

double oracle_weno5(const double* f) { return weno5(f[0], f[1], f[2], f[3], f[4]); }

void oracle_species_thermo(const OMech* m, int k, double T, double* h, double* cp, double* s) {
    const double* a = (m->nasa_high && m->t_mid && T >= m->t_mid[k]) ? &m->nasa_high[7 * k]
                                                                      : &m->nasa[7 * k];
    double Rk = RU / m->M[k];
    *h = Rk * nasa_h(a, T);
    *cp = Rk * nasa_cp(a, T);
    *s = Rk * nasa_s(a, T);
}

int oracle_temperature(const OMech* m, const double* Y, double e, double Tguess, double* T) {
    MechData md = mech_from(m);
    double t = Tguess;
    int st = newton_T(md, Y, e, t);
    *T = t;
    return st;
}

void oracle_mixture_e_cv(const OMech* m, const double* Y, double T, double* e, double* cv) {
    MechData md = mech_from(m);
    mixture_e_cv(md, Y, T, *e, *cv);
}

void oracle_production(const OMech* m, double rho, double T, const double* rhoY, double* wdot,
                       double* J) {
    MechData md = mech_from(m);
    production(md, rho, T, rhoY, wdot, J);
}

int oracle_point_implicit(const OMech* m, double rho, double T, double* rhoY, double dt) {
    MechData md = mech_from(m);
    return point_implicit(md, rho, T, rhoY, dt);
}

// The species + T Jacobian (see full_jacobian) at (rho, e, T, rhoY); J [Ns-1][Ns-1].
int oracle_full_jacobian(const OMech* m, double rho, double e, double T, const double* rhoY,
                         double* J) {
    MechData md = mech_from(m);
    return full_jacobian(md, rho, e, T, rhoY, J);
}

// L(U) on a uniform grid (one evaluation of the semi-discrete right-hand side).
int oracle_rhs(const OGrid* g, const OPhys* p, const OMech* m, const double* bc_prim,
               const double* U, const double* T, double* L) {
    MechData md = mech_from(m);
    Phys<double> ph = phys_from<double>(p, m ? &md : nullptr);
    GridCfg gc = grid_from(g);
    BCStates<double> bcs;
    if (bc_states_from(ph, g, bc_prim, bcs)) return ST_EINVAL;
    long long n = (long long)gc.nx * gc.ny;
    std::vector<double> Ua, Ta(T, T + n), La;
    soa_to_aos(ph.nU, n, U, Ua);
    int st = rhs_uniform(gc, ph, Ua.data(), Ta.data(), bcs, La);
    if (st) return st;
    aos_to_soa(ph.nU, n, La, L);
    return ST_OK;
}

// nsteps steps on a uniform grid; U [nU][ny][nx], T [ny][nx] updated in place, *t advanced.
int oracle_step(const OGrid* g, const OPhys* p, const OMech* m, const double* bc_prim,
                const OTime* tm, double* U, double* T, int nsteps, double* t, double* dt_log) {
    MechData md = mech_from(m);
    Phys<double> ph = phys_from<double>(p, m ? &md : nullptr);
    GridCfg gc = grid_from(g);
    if (gc.nx < 1 || gc.ny < 1) return ST_EINVAL;
    BCStates<double> bcs;
    if (bc_states_from(ph, g, bc_prim, bcs)) return ST_EINVAL;
    if (tm->split != 0 && (tm->split != 1 || ph.model != MODEL_DETAILED)) return ST_EINVAL;
    if (tm->jac != 0 && (tm->jac != 1 || ph.model != MODEL_DETAILED)) return ST_EINVAL;
    ph.full_jac = tm->jac;
    TimeCfg tc{tm->cfl, tm->dt_fixed, tm->t_end, tm->split};
    long long n = (long long)gc.nx * gc.ny;
    std::vector<double> Ua, Ta(T, T + n);
    soa_to_aos(ph.nU, n, U, Ua);
    int st = resolve_T_all(ph, n, Ua, Ta);
    for (int s = 0; s < nsteps && !st; ++s) {
        double dt = 0.0;
        st = step_uniform(gc, ph, tc, bcs, Ua, Ta, *t, &dt);
        if (dt_log) dt_log[s] = dt;
    }
    aos_to_soa(ph.nU, n, Ua, U);
    std::copy(Ta.begin(), Ta.end(), T);
    return st;
}

struct ODomain { int nx, ny; double dx, dy; int bc[4]; int nlevels; double gamma, R, Q, Ea, k; };

// nsteps steps over a block table (pool SoA [nU][pool]); t_dom[ndom] advanced per domain;
// dt_log [nsteps][ndom] (optional); crossover = 0: synchronous advance (Fig. 2b), 1: the
// crossover advance (Fig. 2a), where one step is one level-0 step.
int oracle_step_blocks(int model, const OMech* m, int ndom, const ODomain* doms,
                       const double* bc_prim /* [ndom][4][nU] */, int nblocks,
                       const BlockRec* blocks, long long pool, const OTime* tm, double* U,
                       double* T, int nsteps, double* t_dom, double* dt_log, int crossover) {
    if (tm->split != 0 && (tm->split != 1 || model != MODEL_DETAILED)) return ST_EINVAL;
    if (tm->jac != 0 && (tm->jac != 1 || model != MODEL_DETAILED)) return ST_EINVAL;
    MechData md = mech_from(m);
    BlockSet B;
    B.pool = pool;
    B.nU = n_fields(model, m ? m->ns : 0);
    std::vector<Phys<double>> phys(ndom);
    std::vector<std::vector<double>> bcU(4 * ndom);
    std::vector<double> bcT(4 * ndom, 0.0);
    for (int d = 0; d < ndom; ++d) {
        DomainRec r;
        r.nx = doms[d].nx; r.ny = doms[d].ny; r.dx = doms[d].dx; r.dy = doms[d].dy;
        for (int q = 0; q < 4; ++q) r.bc[q] = doms[d].bc[q];
        r.nlevels = doms[d].nlevels;
        r.gamma = doms[d].gamma; r.R = doms[d].R; r.Q = doms[d].Q; r.Ea = doms[d].Ea; r.k = doms[d].k;
        B.dom.push_back(r);
        OPhys op{model, r.gamma, r.R, r.Q, r.Ea, r.k};
        phys[d] = phys_from<double>(&op, m ? &md : nullptr);
        phys[d].full_jac = tm->jac;
        for (int s = 0; s < 4; ++s) {
            bcU[d * 4 + s].assign(B.nU, 0.0);
            if (r.bc[s] == BC_DIRICHLET) {
                if (!bc_prim) return ST_EINVAL;
                conserved_from_primitive(phys[d], &bc_prim[((size_t)d * 4 + s) * B.nU],
                                         bcU[d * 4 + s].data(), bcT[d * 4 + s]);
            }
        }
    }
    B.blk.assign(blocks, blocks + nblocks);
    int st = build_blockset(B);
    if (st) return st;
    std::vector<double> Up(U, U + (size_t)pool * B.nU), Tp(T, T + pool);
    // call entry: T re-solved on every cell of a valid block
    for (int b = 0; b < nblocks && !st; ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid) continue;
        for (long long c = r.offset; c < r.offset + (long long)r.nx * r.ny && !st; ++c) {
            double u[64], Tn = 0.0;
            for (int f = 0; f < B.nU; ++f) u[f] = Up[(size_t)f * pool + c];
            st = cell_temperature(phys[r.domain], u, Tp[c], Tn);
            Tp[c] = Tn;
        }
    }
    std::vector<double> t(t_dom, t_dom + ndom);
    std::vector<double> dts(ndom);
    for (int s = 0; s < nsteps && !st; ++s) {
        const TimeCfg tc{tm->cfl, tm->dt_fixed, tm->t_end, tm->split};
        st = crossover ? step_blocks_crossover(B, phys, tc, bcU, bcT, Up, Tp, t, dts.data())
                       : step_blocks(B, phys, tc, bcU, bcT, Up, Tp, t, dts.data());
        if (dt_log)
            for (int d = 0; d < ndom; ++d) dt_log[(size_t)s * ndom + d] = dts[d];
    }
    std::copy(Up.begin(), Up.end(), U);
    std::copy(Tp.begin(), Tp.end(), T);
    std::copy(t.begin(), t.end(), t_dom);
    return st;
}

// Ring flags of a block table (1 = coarse-fine ring cell), pool-indexed; invalid blocks = 2.
int oracle_ring_flags(int model, int ns, int ndom, const ODomain* doms, int nblocks,
                      const BlockRec* blocks, long long pool, unsigned char* flags) {
    BlockSet B;
    B.pool = pool;
    B.nU = n_fields(model, ns);
    for (int d = 0; d < ndom; ++d) {
        DomainRec r;
        r.nx = doms[d].nx; r.ny = doms[d].ny; r.dx = doms[d].dx; r.dy = doms[d].dy;
        for (int q = 0; q < 4; ++q) r.bc[q] = doms[d].bc[q];
        r.nlevels = doms[d].nlevels;
        r.gamma = doms[d].gamma; r.R = doms[d].R; r.Q = doms[d].Q; r.Ea = doms[d].Ea; r.k = doms[d].k;
        B.dom.push_back(r);
    }
    B.blk.assign(blocks, blocks + nblocks);
    int st = build_blockset(B);
    if (st) return st;
    std::fill(flags, flags + pool, (unsigned char)2);
    for (int b = 0; b < nblocks; ++b) {
        const BlockRec& r = B.blk[b];
        if (!r.valid) continue;
        for (long long q = 0; q < (long long)r.nx * r.ny; ++q) flags[r.offset + q] = B.ring[b][q];
    }
    return ST_OK;
}

static void domains_into(BlockSet& B, int ndom, const ODomain* doms) {
    for (int d = 0; d < ndom; ++d) {
        DomainRec r;
        r.nx = doms[d].nx; r.ny = doms[d].ny; r.dx = doms[d].dx; r.dy = doms[d].dy;
        for (int q = 0; q < 4; ++q) r.bc[q] = doms[d].bc[q];
        r.nlevels = doms[d].nlevels;
        r.gamma = doms[d].gamma; r.R = doms[d].R; r.Q = doms[d].Q; r.Ea = doms[d].Ea; r.k = doms[d].k;
        B.dom.push_back(r);
    }
}

struct ORegrid { double threshold; int buffer, sub; };

// New block table of a hierarchy (pool SoA, field 0 = rho) by the density-gradient
// criterion: out[cap] receives it with packed offsets, *nout its length (when it
// exceeds cap the call returns ST_EINVAL), *pool_out the new pool size. bc_rho
// [ndom][4]: density of each Dirichlet side.
int oracle_regrid(int model, int ns, int ndom, const ODomain* doms, const double* bc_rho,
                  int nblocks, const BlockRec* blocks, long long pool, const double* U,
                  const ORegrid* cfg, BlockRec* out, int cap, int* nout, long long* pool_out) {
    if (!(cfg->threshold >= 0.0) || cfg->buffer < 0 || cfg->sub < 4 || cfg->sub > 128 || cfg->sub % 4)
        return ST_EINVAL;
    BlockSet B;
    B.pool = pool;
    B.nU = n_fields(model, ns);
    domains_into(B, ndom, doms);
    B.blk.assign(blocks, blocks + nblocks);
    int st = build_blockset(B);
    if (st) return st;
    for (const BlockRec& r : B.blk)
        if (r.valid && r.level == 0 && B.dom[r.domain].nlevels > 1 && ((r.nx | r.ny) & 3))
            return ST_EINVAL;
    std::vector<BlockRec> nb;
    st = regrid_table(B, bc_rho, U, RegridCfg{cfg->threshold, cfg->buffer, cfg->sub}, nb);
    if (st) return st;
    *nout = (int)nb.size();
    *pool_out = 0;
    for (const BlockRec& r : nb) *pool_out += (long long)r.nx * r.ny;
    if ((int)nb.size() > cap) return ST_EINVAL;
    std::copy(nb.begin(), nb.end(), out);
    return ST_OK;
}

// Pools of a new table from the old hierarchy (see regrid_fill).
int oracle_regrid_fill(int model, int ns, int ndom, const ODomain* doms, int nold,
                       const BlockRec* old, long long pool_old, const double* Uold,
                       const double* Told, int nnew, const BlockRec* nw, long long pool_new,
                       double* Unew, double* Tnew) {
    BlockSet Bo, Bn;
    Bo.pool = pool_old;
    Bn.pool = pool_new;
    Bo.nU = Bn.nU = n_fields(model, ns);
    domains_into(Bo, ndom, doms);
    domains_into(Bn, ndom, doms);
    Bo.blk.assign(old, old + nold);
    Bn.blk.assign(nw, nw + nnew);
    int st = build_blockset(Bo);
    if (!st) st = build_blockset(Bn);
    if (st) return st;
    for (int b = 1; b < nnew; ++b)
        if (nw[b].level < nw[b - 1].level) return ST_EINVAL;   // coarser layers first
    regrid_fill(Bo, Uold, Told, Bn, Unew, Tnew);
    return ST_OK;
}

// Tangent of the probe loss L = sum_{n=1..N} dt sum_q w_q p(U^n[cell_q]) on a uniform grid
// with fixed dt, seeded by (dW0, dQ, dEa). The initial state is built from the primitives W0,
// so its dependence on Q enters through E0. Returns loss and its directional derivative.
int oracle_loss_tangent(const OGrid* g, const OPhys* p, const OMech* m, const double* bc_prim,
                        double dt_fixed, const double* W0, const double* dW0, double dQ,
                        double dEa, int nsteps, int nprobes, const int* probe,
                        const double* pw, double* loss, double* dloss) {
    MechData md = mech_from(m);
    Phys<Dual> ph = phys_from<Dual>(p, m ? &md : nullptr);
    ph.Q = Dual(p->Q, dQ);
    ph.Ea = Dual(p->Ea, dEa);
    GridCfg gc = grid_from(g);
    BCStates<Dual> bcs;
    if (bc_states_from(ph, g, bc_prim, bcs)) return ST_EINVAL;
    const long long n = (long long)gc.nx * gc.ny;
    const int nU = ph.nU;
    std::vector<Dual> U((size_t)n * nU), T(n);
    std::vector<Dual> w(nU);
    for (long long c = 0; c < n; ++c) {
        for (int f = 0; f < nU; ++f) w[f] = Dual(W0[(size_t)f * n + c], dW0 ? dW0[(size_t)f * n + c] : 0.0);
        conserved_from_primitive(ph, w.data(), &U[(size_t)c * nU], T[c]);
    }
    int st = resolve_T_all(ph, n, U, T);
    TimeCfg tc{0.0, dt_fixed, 0.0};
    double t = 0.0;
    Dual acc = 0.0;
    for (int s = 0; s < nsteps && !st; ++s) {
        st = step_uniform(gc, ph, tc, bcs, U, T, t, nullptr);
        if (st) break;
        for (int q = 0; q < nprobes; ++q) {
            Prim<Dual> P;
            st = primitives(ph, &U[(size_t)probe[q] * nU], T[probe[q]], P);
            if (st) break;
            acc = acc + Dual(dt_fixed) * (pw[q] * P.p);
        }
    }
    *loss = acc.v;
    *dloss = acc.d;
    return st;
}

}  // extern "C"
