// sweep_inst.hip -- instantiates the per-image sweep kernels for one blur
// size HX_KS and one mode HX_MODE (the build compiles this file once per
// pair, in parallel) for C in {1,2,4} columns per lane; the tile height is
// a run-time argument.
#include "sweep_kernel.h"

#ifndef HX_KS
#error "HX_KS must be defined"
#endif
#ifndef HX_MODE
#error "HX_MODE must be defined"
#endif

#define HX_CAT2(a, b, c, d) a##b##c##d
#define HX_CAT(a, b, c, d) HX_CAT2(a, b, c, d)
#define HX_FN HX_CAT(launch_sweep_k, HX_KS, _m, HX_MODE)

namespace hx {

hipError_t HX_FN(int c, int ty, const ImgArgs& a, const Taps& t, float theta,
                 hipStream_t s) {
    if (!sweep_supported(HX_KS, c, ty)) return hipErrorInvalidValue;
    if (c == 1) return launch_sweep_t<HX_KS, 1, HX_MODE>(ty, a, t, theta, s);
    if (c == 2) return launch_sweep_t<HX_KS, 2, HX_MODE>(ty, a, t, theta, s);
    if (c == 4) return launch_sweep_t<HX_KS, 4, HX_MODE>(ty, a, t, theta, s);
    return hipErrorInvalidValue;
}

}  // namespace hx
