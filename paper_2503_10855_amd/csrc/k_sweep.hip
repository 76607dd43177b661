// k_sweep.hip -- dispatch of the per-image sweep kernels by (mode, ksize).
#include "hx_kernels.h"

namespace hx {

#define HX_DECL(K, M)                                                        \
    hipError_t launch_sweep_k##K##_m##M(int c, int ty, const ImgArgs& a,   \
                                        const Taps& t, float theta,          \
                                        hipStream_t s);
#define HX_DECL_K(K) HX_DECL(K, 0) HX_DECL(K, 1) HX_DECL(K, 2) HX_DECL(K, 3) HX_DECL(K, 4)
HX_DECL_K(3)
HX_DECL_K(5)
HX_DECL_K(7)
#undef HX_DECL_K
#undef HX_DECL

bool sweep_supported(int ks, int c, int ty) {
    return (ks == 3 || ks == 5 || ks == 7) && (c == 1 || c == 2 || c == 4) &&
           ty >= 8 && ty <= 256 && ty % 8 == 0;
}

hipError_t launch_sweep(int mode, int ks, int c, int ty, const ImgArgs& a,
                        const Taps& t, float theta, hipStream_t s) {
#define HX_M(K)                                                             \
    switch (mode) {                                                         \
        case 0: return launch_sweep_k##K##_m0(c, ty, a, t, theta, s);       \
        case 1: return launch_sweep_k##K##_m1(c, ty, a, t, theta, s);       \
        case 2: return launch_sweep_k##K##_m2(c, ty, a, t, theta, s);       \
        case 3: return launch_sweep_k##K##_m3(c, ty, a, t, theta, s);       \
        case 4: return launch_sweep_k##K##_m4(c, ty, a, t, theta, s);       \
        default: return hipErrorInvalidValue;                               \
    }
    if (ks == 3) { HX_M(3) }
    if (ks == 5) { HX_M(5) }
    if (ks == 7) { HX_M(7) }
#undef HX_M
    return hipErrorInvalidValue;
}

}  // namespace hx
