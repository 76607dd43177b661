// sweep_impl.h -- the fused register sweep over one tile of one image.
//
// One wave64 owns a strip of SW = 64*C input columns (C per lane) and
// walks it downwards one input row per step.  Every stencil stage is a
// fork over pixels (the paper's fork-join form); here they are fused into
// one pass: each step
//   A  loads input row v (prefetched PF rows ahead) and forms the
//      horizontal blur Bh(v) of the lane's C columns (neighbour columns
//      come from the adjacent lanes via DPP),
//   B  finishes the vertical blur B(v-R) from the ring of the last k Bh
//      rows, and its row pieces (e+w sums, Sobel dx and sy),
//   C  forms L and G^2 of row v-R-1 from the last three B rows, and the
//      horizontal 3-max / 3-min of L,
//   D  forms Z of row v-R-2 from three max/min rows and emits its output.
// Rings are indexed by step mod P, and the step loop is unrolled by P, so
// every ring slot is a fixed register.  Every value is computed by the
// helpers in hx_device.h, in the same order as the depth-1 stage kernels.
//
// Borders: each stage reads its input at clamped coordinates.  Rows: the
// input row index is clamped; a B or L row below the image is a copy of
// the last real row; the row above the image is overwritten with row 0 as
// soon as row 0 exists (before any valid output reads it).  Columns: the
// input column is clamped, and the B and L values of columns outside the
// image are replaced by the first / last real column's value.
#pragma once

#include "hx_kernels.h"

namespace hx {

template <int KS, int C, int TY, int MODE>
struct SweepShape {
    static constexpr int R = KS / 2;
    static constexpr int HX = R + 2;                       // chain halo
    static constexpr int HL = ((HX + C - 1) / C) * C;      // left halo
    static constexpr int SW = 64 * C;                      // strip width
    static constexpr int OW = ((SW - HL - HX) / C) * C;    // output width
    static constexpr int P = KS >= 5 ? KS : 6;             // ring period
    static constexpr int NS = TY + 2 * HX;                 // steps
    static constexpr int PF = P - 1 < 4 ? P - 1 : 4;       // prefetch rows
    static constexpr bool NEED_L =
        MODE == SM_STORE || MODE == SM_MASK || MODE == SM_BGL;
    static constexpr bool NEED_Z = MODE == SM_STORE || MODE == SM_MASK;
    static constexpr bool DO_MAX = MODE != SM_MASK;
};

template <int C>
struct alignas(4 * C) VecF {
    float v[C];
};

// Value of the lane (self + q), q a constant after unrolling.
__device__ __forceinline__ float lane_fetch_q(float v, int q) {
    if (q == 0) return v;
    if (q == 1) return from_right(v);
    if (q == -1) return from_left(v);
    if (q == 2) return from_right(from_right(v));
    if (q == -2) return from_left(from_left(v));
    if (q == 3) return from_right(from_right(from_right(v)));
    return from_left(from_left(from_left(v)));
}

__device__ __forceinline__ float max3f(float a, float b, float c) {
    return __builtin_fmaxf(__builtin_fmaxf(a, b), c);
}
__device__ __forceinline__ float min3f(float a, float b, float c) {
    return __builtin_fminf(__builtin_fminf(a, b), c);
}

// Replace the values of columns outside [0, W) with column 0's / W-1's.
template <int C, int HL, int SW>
__device__ __forceinline__ void fix_cols(float (&x)[C], int x0, int xs,
                                         int cbase, int W) {
    if (x0 == 0) {
        // Column 0 sits in lane HL/C, element 0.
        const float v0 = __int_as_float(
            __builtin_amdgcn_readlane(__float_as_int(x[0]), HL / C));
#pragma unroll
        for (int e = 0; e < C; ++e)
            if (cbase + e < 0) x[e] = v0;
    }
    if (xs + SW > W) {
        const int cw = W - 1 - xs;
        const int ln = cw / C, el = cw - ln * C;
        // Column W-1 is element `el` of lane `ln` (both wave-uniform): read
        // every element of that lane and pick one with a scalar select.
        int pick = 0;
#pragma unroll
        for (int k = 0; k < C; ++k) {
            const int vk = __builtin_amdgcn_readlane(__float_as_int(x[k]), ln);
            pick = (el == k) ? vk : pick;
        }
        const float vw = __int_as_float(pick);
#pragma unroll
        for (int e = 0; e < C; ++e)
            if (cbase + e > W - 1) x[e] = vw;
    }
}

// Run one tile: output columns [x0, x0+OW) x rows [y0, y0+TY), clipped to
// the image.  thr2 is used by SM_MASK only.  gmax accumulates G^2 over the
// tile's output pixels (per lane; the caller reduces it).
template <int KS, int C, int TY, int MODE>
__device__ __forceinline__ void sweep_tile(const ImgArgs& a, const Taps& tp,
                                           int x0, int y0, float thr2,
                                           float& gmax) {
    using S = SweepShape<KS, C, TY, MODE>;
    constexpr int R = S::R, HX = S::HX, HL = S::HL, SW = S::SW, OW = S::OW;
    constexpr int P = S::P, NS = S::NS, PF = S::PF;

    const int lane = lane_id();
    const int H = a.H, W = a.W;
    const int xs = x0 - HL;
    const int cbase = xs + C * lane;
    const bool bx = (xs < 0) | (xs + SW > W);
    const bool by = (y0 - HX < 0) | (y0 + TY + HX > H);
    const int ylim = min(y0 + TY, H);
    const bool lane_out = (cbase >= x0) & (cbase < x0 + OW);
    bool ecol[C];
#pragma unroll
    for (int e = 0; e < C; ++e) ecol[e] = lane_out & (cbase + e < W);
    const bool vec_ok =
        ((reinterpret_cast<uintptr_t>(a.src) % (4 * C)) == 0) & ((a.sp % C) == 0);
    const bool mask_vec =
        ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) & ((a.mp % 4) == 0);

    auto load_row = [&](int v, float (&dst)[C]) {
        const int row = by ? clampi(v, 0, H - 1) : v;
        const float* rp = a.src + (int64_t)row * a.sp;
        if (!bx & vec_ok) {
            const VecF<C> q = *reinterpret_cast<const VecF<C>*>(rp + cbase);
#pragma unroll
            for (int e = 0; e < C; ++e) dst[e] = q.v[e];
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                dst[e] = rp[bx ? clampi(cbase + e, 0, W - 1) : cbase + e];
        }
    };
    auto store_f = [&](float* base, int row, const float (&val)[C]) {
        float* rp = base + (int64_t)row * a.op + cbase;
        if (!bx) {
            if (lane_out) {
                VecF<C> q;
#pragma unroll
                for (int e = 0; e < C; ++e) q.v[e] = val[e];
                *reinterpret_cast<VecF<C>*>(rp) = q;
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ecol[e]) rp[e] = val[e];
        }
    };

    float pf[P][C];   // prefetched input rows
    float bh[P][C];   // horizontal blur rows
    float bb[P][C];   // B rows
    float ew[P][C];   // B(x-1) + B(x+1)
    float dx[P][C];   // Sobel dx
    float sy[P][C];   // Sobel sy
    float hmx[P][C];  // 3-wide max of L
    float hmn[P][C];  // 3-wide min of L
    float g2d[C];     // G^2 of the row waiting for its Z

#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(y0 - HX + j, pf[j]);

    for (int s0 = 0; s0 < NS; s0 += P) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int s = s0 + j;
            if (s < NS) {
                const int v = y0 - HX + s;
                if (s + PF < NS) load_row(v + PF, pf[(j + PF) % P]);

                // ---- A: horizontal blur of input row v
                {
                    float ext[C + 2 * R];
#pragma unroll
                    for (int k = 0; k < C + 2 * R; ++k) {
                        const int kk = k - R;
                        const int q = kk >= 0 ? kk / C : -((-kk + C - 1) / C);
                        ext[k] = lane_fetch_q(pf[j][kk - q * C], q);
                    }
#pragma unroll
                    for (int e = 0; e < C; ++e)
                        bh[j][e] = blur_chain<KS>(&ext[e], tp);
                }

                // ---- B: vertical blur, row vb = v - R
                if (s >= 2 * R) {
                    const int vb = v - R;
                    float b[C];
#pragma unroll
                    for (int e = 0; e < C; ++e) {
                        float col[KS];
#pragma unroll
                        for (int i = 0; i < KS; ++i)
                            col[i] = bh[(j - 2 * R + i + 4 * P) % P][e];
                        b[e] = blur_chain<KS>(col, tp);
                    }
                    if (by && vb >= H) {
#pragma unroll
                        for (int e = 0; e < C; ++e) b[e] = bb[(j + P - 1) % P][e];
                    }
                    if (bx) fix_cols<C, HL, SW>(b, x0, xs, cbase, W);
                    const float bl0 = from_left(b[C - 1]);
                    const float br0 = from_right(b[0]);
#pragma unroll
                    for (int e = 0; e < C; ++e) {
                        const float l = e > 0 ? b[e - 1] : bl0;
                        const float r = e < C - 1 ? b[e + 1] : br0;
                        bb[j][e] = b[e];
                        ew[j][e] = l + r;
                        dx[j][e] = sobel_dx(l, r);
                        sy[j][e] = sobel_sy(ew[j][e], b[e]);
                    }
                    if (by && vb == 0) {
#pragma unroll
                        for (int e = 0; e < C; ++e) {
                            bb[(j + P - 1) % P][e] = bb[j][e];
                            dx[(j + P - 1) % P][e] = dx[j][e];
                            sy[(j + P - 1) % P][e] = sy[j][e];
                        }
                    }
                }

                // ---- C: L and G^2 of row vl = v - R - 1
                if (s >= 2 * R + 2) {
                    const int vl = v - R - 1;
                    const int ju = (j + 2 * P - 2) % P;
                    const int jc = (j + P - 1) % P;
                    float g2[C];
#pragma unroll
                    for (int e = 0; e < C; ++e)
                        g2[e] = sobel_g2(dx[ju][e], dx[jc][e], dx[j][e], sy[ju][e],
                                         sy[j][e]);
                    const bool row_out = (vl >= y0) & (vl < ylim);
                    if constexpr (S::DO_MAX) {
                        if (row_out) {
#pragma unroll
                            for (int e = 0; e < C; ++e)
                                gmax = __builtin_fmaxf(gmax, ecol[e] ? g2[e] : 0.0f);
                        }
                    }
                    if constexpr (MODE == SM_BG) {
                        if (row_out) {
                            store_f(a.fout, vl, bb[jc]);
                            store_f(a.g2, vl, g2);
                        }
                    }
                    if constexpr (S::NEED_L) {
                        float l[C];
#pragma unroll
                        for (int e = 0; e < C; ++e)
                            l[e] = lap_from(bb[ju][e] + bb[j][e], ew[jc][e], bb[jc][e]);
                        if constexpr (MODE == SM_BGL) {
                            if (row_out) {
                                store_f(a.fout, vl, l);
                                store_f(a.g2, vl, g2);
                            }
                        }
                        if constexpr (S::NEED_Z) {
                            if (bx) fix_cols<C, HL, SW>(l, x0, xs, cbase, W);
                            const float ll0 = from_left(l[C - 1]);
                            const float lr0 = from_right(l[0]);
#pragma unroll
                            for (int e = 0; e < C; ++e) {
                                const float lf = e > 0 ? l[e - 1] : ll0;
                                const float rt = e < C - 1 ? l[e + 1] : lr0;
                                hmx[j][e] = max3f(lf, l[e], rt);
                                hmn[j][e] = min3f(lf, l[e], rt);
                            }
                            if (by && vl >= H) {
#pragma unroll
                                for (int e = 0; e < C; ++e) {
                                    hmx[j][e] = hmx[jc][e];
                                    hmn[j][e] = hmn[jc][e];
                                }
                            }
                            if (by && vl == 0) {
#pragma unroll
                                for (int e = 0; e < C; ++e) {
                                    hmx[jc][e] = hmx[j][e];
                                    hmn[jc][e] = hmn[j][e];
                                }
                            }
                            // ---- D: Z of row vz = vl - 1, and the output
                            if (s >= 2 * R + 4) {
                                const int vz = vl - 1;
                                if ((vz >= y0) & (vz < ylim)) {
                                    bool z[C];
#pragma unroll
                                    for (int e = 0; e < C; ++e)
                                        z[e] = zero_cross(
                                            max3f(hmx[ju][e], hmx[jc][e], hmx[j][e]),
                                            min3f(hmn[ju][e], hmn[jc][e], hmn[j][e]));
                                    if constexpr (MODE == SM_STORE) {
                                        float code[C];
#pragma unroll
                                        for (int e = 0; e < C; ++e)
                                            code[e] = pass1_code(z[e], g2d[e]);
                                        store_f(a.fout, vz, code);
                                    } else {
                                        uint8_t* rp = a.mask + (int64_t)vz * a.mp + cbase;
                                        uint32_t m[C];
#pragma unroll
                                        for (int e = 0; e < C; ++e)
                                            m[e] = (z[e] & (g2d[e] > thr2)) ? 1u : 0u;
                                        if (!bx & (C == 4) & mask_vec) {
                                            if (lane_out) {
                                                uint32_t w = 0;
#pragma unroll
                                                for (int e = 0; e < C; ++e) w |= m[e] << (8 * e);
                                                *reinterpret_cast<uint32_t*>(rp) = w;
                                            }
                                        } else {
#pragma unroll
                                            for (int e = 0; e < C; ++e)
                                                if (ecol[e]) rp[e] = (uint8_t)m[e];
                                        }
                                    }
                                }
                            }
#pragma unroll
                            for (int e = 0; e < C; ++e) g2d[e] = g2[e];
                        }
                    }
                }
            }
        }
    }
}

}  // namespace hx
