// Layer update (regridding) of a block hierarchy: the density-gradient mask with
// buffer cells evaluated per candidate subregion (Sec. 3.1.2), and the data of a
// new table: copies of unaltered blocks and one-to-four injection for new ones
// (Sec. 3.1.4, refinement and updating-refinement-layer operations).
#include "janc_device.h"

namespace janc {

// Effective layer-`lev` density of cell (I, J): the covering block's cell, else the
// coarser layer's (resolve), or the Dirichlet row outside the domain.
__device__ __forceinline__ double rho_at(const StageArgs& a, CDom& D, int lev, int I, int J) {
    unsigned fl = 0u;
    const long long src = resolve(a, D, lev, I, J, fl);
    return (src >= 0) ? a.Uin[src] : a.dirU[(size_t)(-src - 1) * (MAXF + 1)];
}

// One workgroup per candidate: flag it when a masked layer-`lev` cell lies in the
// candidate rectangle widened by `buffer` cells (clipped to the layer).
__global__ __launch_bounds__(WG) void regrid_flag_kernel(StageArgs a, const RegridCand* cand,
                                                         int lev, int buffer, double thr,
                                                         int* flags) {
    __shared__ int hit;
    const RegridCand C = cand[blockIdx.x];
    CDom& D = cdom(a.dom, C.domain);
    const int W = D.nx0 << lev, H = D.twod ? (D.ny0 << lev) : 1;
    if (threadIdx.x == 0) hit = 0;
    __syncthreads();
    const int ww = C.w + 2 * buffer, n = ww * (C.h + 2 * buffer);
    for (int q = threadIdx.x; q < n; q += WG) {
        const int I = C.i0 - buffer + q % ww, J = C.j0 - buffer + q / ww;
        if (I < 0 || I >= W || J < 0 || J >= H) continue;
        const double r = rho_at(a, D, lev, I, J);
        const double gx = fabs(rho_at(a, D, lev, I + 1, J) - rho_at(a, D, lev, I - 1, J));
        const double gy = fabs(rho_at(a, D, lev, I, J + 1) - rho_at(a, D, lev, I, J - 1));
        if (fmax(gx, gy) > 2.0 * thr * r) hit = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) flags[blockIdx.x] = hit;
}

// One workgroup per block of the new plan (a = new plan, Uin/Tin = old pools,
// Uout/Tout = new pools): copy from the old pool at src, or inject from the new
// plan's coarser layer (already filled by an earlier launch).
__global__ __launch_bounds__(WG) void regrid_fill_kernel(StageArgs a, const RegridFill* job,
                                                         long long old_pool, int nu) {
    const RegridFill F = job[blockIdx.x];
    const DevBlock B = a.blk[F.block];
    CDom& D = cdom(a.dom, B.domain);
    const int n = B.nx * B.ny;
    for (int q = threadIdx.x; q < n; q += WG) {
        const int li = q % B.nx, lj = q / B.nx;
        const long long dst = B.offset + q;
        if (F.src >= 0) {
            const long long s = F.src + q;
            for (int f = 0; f < nu; ++f) a.Uout[(size_t)f * a.pool + dst] = a.Uin[(size_t)f * old_pool + s];
            a.Tout[dst] = a.Tin[s];
        } else {
            const int l = B.level - 1, I = (B.i0 + li) >> 1, J = (B.j0 + lj) >> 1;
            const int pb = a.maps[D.map_off[l] + (J >> 3) * D.map_w[l] + (I >> 3)];
            const DevBlock& P = a.blk[pb];
            const long long s = P.offset + (long long)(J - P.j0) * P.nx + (I - P.i0);
            for (int f = 0; f < nu; ++f) a.Uout[(size_t)f * a.pool + dst] = a.Uout[(size_t)f * a.pool + s];
            a.Tout[dst] = a.Tout[s];
        }
    }
}

hipError_t launch_regrid_flag(const StageArgs& a, const RegridCand* cand, int n, int lev,
                              int buffer, double thr, int* flags, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    regrid_flag_kernel<<<n, WG, 0, s>>>(a, cand, lev, buffer, thr, flags);
    return hipGetLastError();
}

hipError_t launch_regrid_fill(const StageArgs& a, const RegridFill* job, int n, long long old_pool,
                              int nu, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    regrid_fill_kernel<<<n, WG, 0, s>>>(a, job, old_pool, nu);
    return hipGetLastError();
}

}  // namespace janc
