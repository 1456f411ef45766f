// janc_species.hip -- the detailed model's kernels for one species count, compiled once
// per count with -DJANC_NS=<count> (2 .. MAXS): the step (stage, entry, chemistry,
// restriction, ring refill, primitive-to-conserved conversion) and the discrete adjoint
// (alpha, interface and cell reverses, chemistry reverse, loss terms, seeds, chain to the
// primitives). janc_kernels.hip and janc_adjoint.hip reach them through species_ops().
#include "janc_launch.h"
#include "janc_adjoint.h"

#ifndef JANC_NS
#error "compile with -DJANC_NS=<species count>"
#endif

namespace janc {
namespace {

constexpr int NS = JANC_NS, NU = NS + 3;
static_assert(NS >= 2 && NS <= MAXS && NU <= MAXF, "species count out of range");

hipError_t stage(int kind_mask, int tile_w, const StageArgs& a, int first, int n, int owner,
                 hipStream_t s) {
    return launch_stage_m<DETAILED, NU>(kind_mask, tile_w, a, first, n, owner, s);
}

hipError_t init(const StageArgs& a, hipStream_t s) {
    init_kernel<DETAILED, NU><<<a.ntiles, WG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t chem(const StageArgs& a, hipStream_t s) {
    if (a.full_jac) chem_kernel<NS, true><<<a.ntiles, WG, 0, s>>>(a);
    else chem_kernel<NS, false><<<a.ntiles, WG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t restrict_fine(const StageArgs& a, const int* fine_blocks, int nfine, hipStream_t s) {
    restrict_kernel<DETAILED, NU><<<dim3(nfine, RESTRICT_SPLIT), WG, 0, s>>>(a, fine_blocks);
    return hipGetLastError();
}

hipError_t ring_fill(const StageArgs& a, const int* ring_blocks, int nring, hipStream_t s) {
    ring_fill_kernel<NU><<<dim3(nring, RESTRICT_SPLIT), WG, 0, s>>>(a, ring_blocks);
    return hipGetLastError();
}

hipError_t prim_to_cons(const DevMech* mech, long long n, const double* W, double* U, double* T,
                        long long sin, long long sout, hipStream_t s) {
    const int nb = (int)((n + WG - 1) / WG);
    prim_to_cons_kernel<DETAILED, NU><<<nb, WG, 0, s>>>(mech, 0.0, 0.0, 0.0, n, W, U, T, sin, sout);
    return hipGetLastError();
}

hipError_t adj_alpha_l(const AlphaArgs& P, hipStream_t s) {
    adj_alpha<DETAILED, NU><<<dim3(P.nbd, 3 * P.nsteps), AWG, 0, s>>>(P);
    return hipGetLastError();
}

hipError_t adj_stage_l(const AdjArgs& A, hipStream_t s) {
    const int ni = (A.g.nx + 1) * A.g.ny + (A.g.twod ? A.g.nx * (A.g.ny + 1) : 0);
    adj_iface<DETAILED, NU><<<dim3((ni + AWG - 1) / AWG, NU), AWG, 0, s>>>(A);
    adj_cell<DETAILED, NU><<<A.nbd, AWG, 0, s>>>(A);
    adj_finish<DETAILED, NU><<<1, AWG, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_chem_l(const AdjChemArgs& A, hipStream_t s) {
    adj_chem<NS><<<(int)((A.n + AWG - 1) / AWG), AWG, 0, s>>>(A);
    return hipGetLastError();
}

hipError_t adj_loss_l(const AdjGrid& g, const DevMech* mech, const double* base, long long stride,
                      int count, const double* last, int n0, long long n, const int* pc,
                      const double* pw, int np, double dt, double* term, hipStream_t s) {
    const int nst = (count - 1) + (last ? 1 : 0);
    adj_loss<DETAILED, NU><<<(nst + AWG - 1) / AWG, AWG, 0, s>>>(g, mech, base, stride, count, last,
                                                                n0, n, pc, pw, np, dt, term);
    return hipGetLastError();
}

hipError_t adj_seed_l(const AdjGrid& g, const DevMech* mech, const double* U, long long n,
                      const int* pc, const double* pw, int np, double dt, double* lam, double* theta,
                      hipStream_t s) {
    adj_seed<DETAILED, NU><<<1, 64, 0, s>>>(g, mech, U, n, pc, pw, np, dt, lam, theta);
    return hipGetLastError();
}

hipError_t adj_chain_l(const AdjGrid& g, const DevMech* mech, const double* W, const double* lam,
                       long long n, double* gW, double* part, hipStream_t s) {
    adj_chain_ic<DETAILED, NU><<<(int)((n + AWG - 1) / AWG), AWG, 0, s>>>(g, mech, W, lam, n, gW, part);
    return hipGetLastError();
}

const SpeciesOps ops = {NS, stage, init, chem, restrict_fine, ring_fill, prim_to_cons,
                        adj_alpha_l, adj_stage_l, adj_chem_l, adj_loss_l, adj_seed_l, adj_chain_l};

}  // namespace

#define JANC_CAT2(a, b) a##b
#define JANC_CAT(a, b) JANC_CAT2(a, b)
const SpeciesOps* JANC_CAT(species_ops_, JANC_NS)() { return &ops; }

}  // namespace janc
