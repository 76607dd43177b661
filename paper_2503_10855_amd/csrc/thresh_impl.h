// thresh_impl.h -- pass 2 of the STORE schedule for four pixels: the
// pass-1 code (G^2 where Z = 1, else -1) against tau^2.
#pragma once

#include "hx_kernels.h"

namespace hx {

struct alignas(16) F4 {
    float v[4];
};

// Pixels (y, x..x+3) of image a; code rows have pitch a.op (a multiple of
// 4 floats, 16-byte aligned), so the float4 read stays inside the row.
__device__ __forceinline__ void threshold4(const ImgArgs& a, int y, int x,
                                           float thr2, bool mvec) {
    const gptr<const F4> c = (gptr<const F4>)(as_global(a.fout) + (int64_t)y * a.op + x);
    const uint32_t m0 = c->v[0] > thr2, m1 = c->v[1] > thr2, m2 = c->v[2] > thr2,
                   m3 = c->v[3] > thr2;
    const gptr<uint8_t> rp = as_global(a.mask) + (int64_t)y * a.mp + x;
    if (mvec & (x + 3 < a.W)) {
        *(gptr<uint32_t>)rp = m0 | (m1 << 8) | (m2 << 16) | (m3 << 24);
    } else {
        const uint32_t mm[4] = {m0, m1, m2, m3};
        for (int e = 0; e < 4 && x + e < a.W; ++e) rp[e] = (uint8_t)mm[e];
    }
}

}  // namespace hx
