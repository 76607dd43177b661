// sweep_kernel.h -- per-image sweep kernel template: one wave per tile,
// four waves per workgroup, workgroups remapped so each XCD takes a
// contiguous run of tiles.
#pragma once

#include "sweep_impl.h"

namespace hx {

template <int KS, int C, int MODE>
__global__ __launch_bounds__(256) void k_sweep(ImgArgs a, Taps tp, float theta, int ty,
                                               int nstrips, int ntiles) {
    using S = SweepShape<KS, C, MODE>;
    const int wave = threadIdx.x >> 6;
    const int t = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
    if (t >= ntiles) return;
    const int by = t / nstrips, bx = t - by * nstrips;
    float thr2 = 0.0f;
    if constexpr (MODE == SM_MASK) thr2 = thr2_from(*a.slot, theta);
    float gmax = 0.0f;
    // Odd bands sweep upwards (shared halo rows are read at the same time).
    sweep_tile<KS, C, MODE>(a, tp, bx * S::OW, by * ty, ty, thr2, gmax, nullptr, (by & 1) != 0);
    if constexpr (S::DO_MAX) {
        gmax = wave_max(gmax);
        if (lane_id() == 0) atomic_max_g2(a.slot, gmax);
    }
}

template <int KS, int C, int MODE>
hipError_t launch_sweep_t(int ty, const ImgArgs& a, const Taps& t, float theta,
                          hipStream_t s) {
    using S = SweepShape<KS, C, MODE>;
    const int nstrips = (a.W + S::OW - 1) / S::OW;
    const int nbands = (a.H + ty - 1) / ty;
    const int ntiles = nstrips * nbands;
    const int grid = (ntiles + 3) / 4;
    hipLaunchKernelGGL((k_sweep<KS, C, MODE>), dim3(grid), dim3(256), 0, s, a, t, theta,
                       ty, nstrips, ntiles);
    return hipGetLastError();
}

}  // namespace hx
