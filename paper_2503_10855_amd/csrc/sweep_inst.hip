// sweep_inst.hip -- instantiates the per-image sweep kernels for one blur
// size HX_KS and one mode HX_MODE (the build compiles this file once per
// pair, in parallel) over every tile shape: C in {1,2,4} columns per lane,
// TY in {16,32,64,128} rows.
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
#define HX_CASE(C, TY) \
    if (c == C && ty == TY) return launch_sweep_t<HX_KS, C, TY, HX_MODE>(a, t, theta, s);
    HX_CASE(1, 16) HX_CASE(1, 32) HX_CASE(1, 64) HX_CASE(1, 128)
    HX_CASE(2, 16) HX_CASE(2, 32) HX_CASE(2, 64) HX_CASE(2, 128)
    HX_CASE(4, 16) HX_CASE(4, 32) HX_CASE(4, 64) HX_CASE(4, 128)
#undef HX_CASE
    return hipErrorInvalidValue;
}

}  // namespace hx
