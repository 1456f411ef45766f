// janc_launch.h -- host launcher of the stage kernel templates of janc_kernels.h (kept out
// of that header, which holds device code only and is also compiled at run time).
#pragma once

#include "janc_kernels.h"

namespace janc {

template <int M, int NU>
hipError_t launch_stage_m(int kind_mask, int tile_w, const StageArgs& a, int first,
                                 int n, int owner, hipStream_t s) {
    const bool h1 = kind_mask & 2, h2 = kind_mask & 1;
#define JANC_STAGE(TXv, TYv)                                                                      \
    do {                                                                                          \
        if (h1 && h2) stage_kernel<M, NU, TXv, TYv, true, true><<<n, WG, 0, s>>>(a, first, owner);   \
        else if (h1) stage_kernel<M, NU, TXv, TYv, true, false><<<n, WG, 0, s>>>(a, first, owner);  \
        else stage_kernel<M, NU, TXv, TYv, false, true><<<n, WG, 0, s>>>(a, first, owner);          \
    } while (0)
    if (tile_w == 32) JANC_STAGE(32, 8);
    else if (tile_w == 64) JANC_STAGE(64, 4);
    else JANC_STAGE(16, 16);
#undef JANC_STAGE
    return hipGetLastError();
}

}  // namespace janc
