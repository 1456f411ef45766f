// janc_adjoint.hip -- launchers of the discrete adjoint kernels (janc_adjoint.h): the
// one-step model here, the detailed model through the per-species-count launch tables of
// janc_species.hip.
#include "janc_adjoint.h"

namespace janc {

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

__global__ void adj_loss_sum(const double* term, int nsteps, double* loss) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nsteps; ++q) s += term[q];
    loss[0] = s;
}

__global__ void adj_chain_sum(const double* part, int nb, double* theta) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int q = 0; q < nb; ++q) s += part[q];
    theta[0] += s;
}

// ------------------------------------------------------------------ launchers
// The one-step model's kernels are launched here, the detailed model's through the
// per-species-count tables.
hipError_t adj_alpha_launch(int model, int ns, const AlphaArgs& P, hipStream_t s) {
    if (P.nsteps <= 0) return hipSuccess;
    if (model == ONESTEP) {
        adj_alpha<ONESTEP, 5><<<dim3(P.nbd, 3 * P.nsteps), AWG, 0, s>>>(P);
    } else {
        const SpeciesOps* o = species_ops(ns);
        if (!o) return hipErrorInvalidValue;
        hipError_t e = o->adj_alpha(P, s);
        if (e != hipSuccess) return e;
    }
    adj_alpha_reduce<<<3 * P.nsteps, AWG, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t adj_stage(int model, int ns, const AdjArgs& A, hipStream_t s) {
    if (model != ONESTEP) {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->adj_stage(A, s) : hipErrorInvalidValue;
    }
    const int ni = (A.g.nx + 1) * A.g.ny + (A.g.twod ? A.g.nx * (A.g.ny + 1) : 0);
    adj_iface<ONESTEP, 5><<<dim3((ni + AWG - 1) / AWG, 5), AWG, 0, s>>>(A);
    adj_cell<ONESTEP, 5><<<A.nbd, AWG, 0, s>>>(A);
    adj_finish<ONESTEP, 5><<<1, AWG, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_chem_launch(int ns, const AdjChemArgs& A, hipStream_t s) {
    const SpeciesOps* o = species_ops(ns);
    return o ? o->adj_chem(A, s) : hipErrorInvalidValue;
}

hipError_t adj_loss_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                           const double* base, long long stride, int count, const double* last,
                           int n0, long long n, const int* pc, const double* pw, int np, double dt,
                           double* term, hipStream_t s) {
    const int nst = (count - 1) + (last ? 1 : 0);
    if (nst <= 0) return hipSuccess;
    if (model != ONESTEP) {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->adj_loss(g, mech, base, stride, count, last, n0, n, pc, pw, np, dt, term, s)
                 : hipErrorInvalidValue;
    }
    adj_loss<ONESTEP, 5><<<(nst + AWG - 1) / AWG, AWG, 0, s>>>(g, mech, base, stride, count, last, n0,
                                                              n, pc, pw, np, dt, term);
    return hipGetLastError();
}

hipError_t adj_loss_sum_launch(const double* term, int nsteps, double* loss, hipStream_t s) {
    adj_loss_sum<<<1, 64, 0, s>>>(term, nsteps, loss);
    return hipGetLastError();
}

hipError_t adj_seed_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                           const double* U, long long n, const int* pc, const double* pw, int np,
                           double dt, double* lam, double* theta, hipStream_t s) {
    if (model != ONESTEP) {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->adj_seed(g, mech, U, n, pc, pw, np, dt, lam, theta, s) : hipErrorInvalidValue;
    }
    adj_seed<ONESTEP, 5><<<1, 64, 0, s>>>(g, mech, U, n, pc, pw, np, dt, lam, theta);
    return hipGetLastError();
}

hipError_t adj_chain_launch(int model, int ns, const AdjGrid& g, const DevMech* mech,
                            const double* W, const double* lam, long long n, double* gW,
                            double* part, double* theta, hipStream_t s) {
    const int nb = (int)((n + AWG - 1) / AWG);
    if (model == ONESTEP) {
        adj_chain_ic<ONESTEP, 5><<<nb, AWG, 0, s>>>(g, mech, W, lam, n, gW, part);
    } else {
        const SpeciesOps* o = species_ops(ns);
        if (!o) return hipErrorInvalidValue;
        hipError_t e = o->adj_chain(g, mech, W, lam, n, gW, part, s);
        if (e != hipSuccess) return e;
    }
    adj_chain_sum<<<1, 64, 0, s>>>(part, nb, theta);
    return hipGetLastError();
}

}  // namespace janc
