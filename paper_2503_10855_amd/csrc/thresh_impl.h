// thresh_impl.h -- pass 2 of the STORE schedule: 16-bit pass-1 codes ->
// mask, eight pixels per call, with an exact recompute of G^2 for the
// pixels whose code cannot decide.
#pragma once

#include "hx_kernels.h"

namespace hx {

struct alignas(16) U4 {
    uint32_t v[4];
};

// B at (y, x) (already clamped), by the same fma chains as every sweep:
// horizontal passes over the clamped row, then the vertical pass.
__device__ __forceinline__ float blur_at(const ImgArgs& a, const Taps& tp, int ks,
                                         int y, int x) {
    const int r = ks / 2;
    float col[kMaxK];
    for (int i = 0; i < ks; ++i) {
        const gptr<const float> rp =
            as_global(a.src) + (int64_t)clampi(y - r + i, 0, a.H - 1) * a.sp;
        float row[kMaxK];
        for (int j = 0; j < ks; ++j) row[j] = rp[clampi(x - r + j, 0, a.W - 1)];
        col[i] = blur_chain_rt(row, tp, ks);
    }
    return blur_chain_rt(col, tp, ks);
}

// The exact G^2 of pixel (y, x), identical to the sweeps' value: B at the
// clamped 3x3 neighbourhood, then the Sobel pieces in the shared order.
__device__ __noinline__ float g2_exact(const ImgArgs& a, const Taps& tp, int ks, int y,
                                       int x) {
    float dxr[3], syr[3];
    for (int d = 0; d < 3; ++d) {
        const int yy = clampi(y - 1 + d, 0, a.H - 1);
        const float l = blur_at(a, tp, ks, yy, clampi(x - 1, 0, a.W - 1));
        const float c = blur_at(a, tp, ks, yy, x);
        const float r = blur_at(a, tp, ks, yy, clampi(x + 1, 0, a.W - 1));
        dxr[d] = sobel_dx(l, r);
        syr[d] = sobel_sy(l + r, c);
    }
    return sobel_g2(dxr[0], dxr[1], dxr[2], syr[0], syr[2]);
}

// Pixels (y, x..x+7) of image a; x is a multiple of 8 and code rows are
// padded to a multiple of 8, so the 16-byte read stays inside the row.
__device__ __forceinline__ void threshold8(const ImgArgs& a, const Taps& tp, int ks,
                                           int y, int x, float thr2, bool mvec,
                                           bool exact_all) {
    const gptr<const U4> cq = (gptr<const U4>)(as_global(a.code) + (int64_t)y * a.cp + x);
    uint32_t w[4] = {cq->v[0], cq->v[1], cq->v[2], cq->v[3]};
    uint32_t m[8];
    bool any_amb = false;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t c = (w[e >> 1] >> (16 * (e & 1))) & 0xffffu;
        m[e] = code16_decide(c, thr2);
        if (exact_all && !(c & 0x8000u)) m[e] = 2u;
        any_amb |= (m[e] == 2u) & (x + e < a.W);
    }
    if (any_amb) {
        for (int e = 0; e < 8; ++e)
            if (m[e] == 2u && x + e < a.W) m[e] = g2_exact(a, tp, ks, y, x + e) > thr2 ? 1u : 0u;
    }
    const gptr<uint8_t> rp = as_global(a.mask) + (int64_t)y * a.mp + x;
    if (mvec & (x + 7 < a.W)) {
        ((gptr<uint32_t>)rp)[0] = m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24);
        ((gptr<uint32_t>)rp)[1] = m[4] | (m[5] << 8) | (m[6] << 16) | (m[7] << 24);
    } else {
        for (int e = 0; e < 8 && x + e < a.W; ++e) rp[e] = (uint8_t)m[e];
    }
}

}  // namespace hx
