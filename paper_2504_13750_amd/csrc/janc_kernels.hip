// janc_kernels.hip -- launchers of the JANC step kernels (janc_kernels.h): the
// calorically perfect and one-step models here, the detailed model through the
// per-species-count launch tables of janc_species.hip.
#include "janc_launch.h"

namespace janc {

__global__ void clear_kernel(unsigned long long* buf, int n) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) buf[q] = 0ull;
}

__global__ void zero_int_kernel(int* p) {
    if (threadIdx.x == 0) *p = 0;
}

// ------------------------------------------------------------------ launchers
// The per-species-count tables (janc_species.hip, one translation unit per count).
const SpeciesOps* species_ops_2();
const SpeciesOps* species_ops_3();
const SpeciesOps* species_ops_4();
const SpeciesOps* species_ops_5();
const SpeciesOps* species_ops_6();
const SpeciesOps* species_ops_7();
const SpeciesOps* species_ops_8();
const SpeciesOps* species_ops_9();
const SpeciesOps* species_ops_10();
const SpeciesOps* species_ops_11();
const SpeciesOps* species_ops_12();
static_assert(JANC_NS_FIRST == 2 && JANC_NS_LAST == 12, "species tables 2 .. 12");

const SpeciesOps* species_ops(int ns) {
    switch (ns) {
        case 2: return species_ops_2();
        case 3: return species_ops_3();
        case 4: return species_ops_4();
        case 5: return species_ops_5();
        case 6: return species_ops_6();
        case 7: return species_ops_7();
        case 8: return species_ops_8();
        case 9: return species_ops_9();
        case 10: return species_ops_10();
        case 11: return species_ops_11();
        case 12: return species_ops_12();
        default: return nullptr;
    }
}

bool model_supported(int model, int ns) {
    if (model == CPG || model == ONESTEP) return true;
    return model == DETAILED && species_ops(ns) != nullptr;
}

hipError_t launch_zero_int(int* p, hipStream_t s) {
    zero_int_kernel<<<1, 64, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t launch_clear_reduce(const Reduce& r, int which, hipStream_t s) {
    const int n = ((which < 0) ? RED_BUFS * r.stride : r.stride) * SLOT_WORDS;
    unsigned long long* p = (which < 0) ? r.buf : r.buf + (size_t)which * r.stride * SLOT_WORDS;
    clear_kernel<<<1, WG, 0, s>>>(p, n);
    return hipGetLastError();
}


hipError_t launch_stage(int model, int ns, int kind_mask, int tile_w, const StageArgs& a,
                        int first_tile, int ntiles, hipStream_t s) {
    const int owner = (first_tile == 0) ? 1 : 0;
    if (ntiles <= 0) return hipSuccess;
    if (model == CPG) return launch_stage_m<CPG, 4>(kind_mask, tile_w, a, first_tile, ntiles, owner, s);
    if (model == ONESTEP) return launch_stage_m<ONESTEP, 5>(kind_mask, tile_w, a, first_tile, ntiles, owner, s);
    const SpeciesOps* o = species_ops(ns);
    return o ? o->stage(kind_mask, tile_w, a, first_tile, ntiles, owner, s) : hipErrorInvalidValue;
}

int halo_table_stride(int tile_w, int kind_mask) {
    int np2 = Geom<16, 16>::NP;
    if (tile_w == 32) np2 = Geom<32, 8>::NP;
    else if (tile_w == 64) np2 = Geom<64, 4>::NP;
    const int np1 = Geom<WG, 1>::NP;
    int n = (kind_mask & 1) ? np2 : 0;
    if (kind_mask & 2) n = max(n, np1);
    return n > 0 ? n : np2;
}

hipError_t launch_halo_table(int tile_w, const StageArgs& a, int* out, int stride, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (tile_w == 32) halo_table_kernel<32, 8><<<a.ntiles, WG, 0, s>>>(a, out, stride);
    else if (tile_w == 64) halo_table_kernel<64, 4><<<a.ntiles, WG, 0, s>>>(a, out, stride);
    else halo_table_kernel<16, 16><<<a.ntiles, WG, 0, s>>>(a, out, stride);
    return hipGetLastError();
}

hipError_t launch_init(int model, int ns, int tile_w, const StageArgs& a, hipStream_t s) {
    (void)tile_w;
    const int n = a.ntiles;
    if (n <= 0) return hipSuccess;
    if (model == CPG) init_kernel<CPG, 4><<<n, WG, 0, s>>>(a);
    else if (model == ONESTEP) init_kernel<ONESTEP, 5><<<n, WG, 0, s>>>(a);
    else {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->init(a, s) : hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_chem(int model, int ns, int tile_w, const StageArgs& a, hipStream_t s) {
    (void)tile_w;
    if (model != DETAILED || a.ntiles <= 0) return hipSuccess;
    const SpeciesOps* o = species_ops(ns);
    return o ? o->chem(a, s) : hipErrorInvalidValue;
}


hipError_t launch_restrict(int model, int ns, const StageArgs& a, const int* fine_blocks, int nfine,
                           hipStream_t s) {
    if (nfine <= 0) return hipSuccess;
    const dim3 grid(nfine, RESTRICT_SPLIT);
    if (model == CPG) restrict_kernel<CPG, 4><<<grid, WG, 0, s>>>(a, fine_blocks);
    else if (model == ONESTEP) restrict_kernel<ONESTEP, 5><<<grid, WG, 0, s>>>(a, fine_blocks);
    else {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->restrict_fine(a, fine_blocks, nfine, s) : hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ring_fill(int model, int ns, const StageArgs& a, const int* ring_blocks, int nring,
                            hipStream_t s) {
    if (nring <= 0) return hipSuccess;
    const dim3 grid(nring, RESTRICT_SPLIT);
    if (model == CPG) ring_fill_kernel<4><<<grid, WG, 0, s>>>(a, ring_blocks);
    else if (model == ONESTEP) ring_fill_kernel<5><<<grid, WG, 0, s>>>(a, ring_blocks);
    else {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->ring_fill(a, ring_blocks, nring, s) : hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_prim_to_cons(int model, int ns, const DevMech* mech, double gamma, double R,
                               double Q, long long n, const double* W, double* U, double* T,
                               long long sin, long long sout, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)((n + WG - 1) / WG);
    if (model == CPG) prim_to_cons_kernel<CPG, 4><<<nb, WG, 0, s>>>(mech, gamma, R, Q, n, W, U, T, sin, sout);
    else if (model == ONESTEP) prim_to_cons_kernel<ONESTEP, 5><<<nb, WG, 0, s>>>(mech, gamma, R, Q, n, W, U, T, sin, sout);
    else {
        const SpeciesOps* o = species_ops(ns);
        return o ? o->prim_to_cons(mech, n, W, U, T, sin, sout, s) : hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace janc
