// sweep_impl.h -- the fused register sweep over one tile of one image.
//
// One wave64 owns a strip of SW = 64*C input columns (C per lane) and
// walks it downwards one input row per step.  Every stencil stage is a
// fork over pixels (the paper's fork-join form); here they are fused into
// one pass: each step
//   A  takes input row v (loaded PF rows ahead) and forms the horizontal
//      blur Bh(v) of the lane's C columns (neighbour columns come from the
//      adjacent lanes via DPP moves),
//   B  finishes the vertical blur B(v-R) from the last k Bh rows, and its
//      row pieces (e+w sums, Sobel dx and sy),
//   C  forms L and G^2 of row v-R-1 from the last three B rows, and the
//      horizontal 3-max / 3-min of L,
//   D  forms Z of row v-R-2 from three max/min rows and emits its output.
// The first 2R+4 steps fill this pipeline and are unrolled with
// compile-time stage flags; the remaining TY steps run as a loop unrolled
// by the ring period P = 8 (which divides TY), so every ring slot is a
// fixed register and the steady state has no stage conditions.  Every
// value is computed by the helpers in hx_device.h, in the same order as
// the depth-1 stage kernels, so all schedules agree bit for bit.
//
// Tiles whose whole input window lies inside the image (the common case)
// run an instantiation with no border logic at all.  The others run one
// that applies the clamped-coordinate rule per stage: rows -- the input
// row index is clamped; a B or L row below the image is a copy of the last
// real row; the row above the image is overwritten with row 0 as soon as
// row 0 exists (before any valid output reads it); columns -- the input
// column is clamped, and the B and L values of columns outside the image
// are replaced by the first / last real column's value.
#pragma once

#include <utility>

#include "hx_kernels.h"

namespace hx {

template <int KS, int C, int TY, int MODE>
struct SweepShape {
    static constexpr int R = KS / 2;
    static constexpr int HX = R + 2;                       // chain halo
    static constexpr int HL = ((HX + C - 1) / C) * C;      // left halo
    static constexpr int SW = 64 * C;                      // strip width
    static constexpr int OW = ((SW - HL - HX) / C) * C;    // output width
    static constexpr int NS = TY + 2 * HX;                 // steps
    static constexpr int NP = 2 * R + 4;                   // pipeline fill
    static constexpr int P = 8;                            // ring period
#ifndef HX_SWEEP_PF
#define HX_SWEEP_PF 6
#endif
    static constexpr int PF = HX_SWEEP_PF;                 // prefetch rows
    static constexpr bool NEED_L =
        MODE == SM_STORE || MODE == SM_MASK || MODE == SM_SPEC || MODE == SM_BGL;
    static constexpr bool NEED_Z =
        MODE == SM_STORE || MODE == SM_MASK || MODE == SM_SPEC;
    static constexpr bool DO_MAX = MODE != SM_MASK;
    static constexpr bool EAGER = MODE == SM_MAXONLY;  // see the steady state
    static_assert(TY % P == 0, "tile height must be a multiple of the ring period");
    static_assert(KS <= P, "the horizontal-blur ring must hold k rows");
};

template <int C>
struct alignas(4 * C) VecF {
    float v[C];
};

template <int V>
using IC = std::integral_constant<int, V>;

template <class F, int... Is>
__device__ __forceinline__ void static_for(F&& f, std::integer_sequence<int, Is...>) {
    (f(IC<Is>{}), ...);
}

// Value held by lane (self + Q); lanes whose source is outside the wave
// read 0 (those values only ever feed halo columns that are discarded).
__device__ __forceinline__ float dpp_from_left(float v) {
    return __int_as_float(
        __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {
    return __int_as_float(
        __builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}
template <int Q>
__device__ __forceinline__ float lane_fetch(float v) {
    if constexpr (Q == 0) return v;
    else if constexpr (Q > 0) return lane_fetch<Q - 1>(dpp_from_right(v));
    else return lane_fetch<Q + 1>(dpp_from_left(v));
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
// the image.  BX / BY: the tile's input window crosses a column / row
// border of the image.  thr2 is used by SM_MASK and SM_SPEC only.  gmax
// accumulates G^2 over real image pixels of the tile (per lane; the caller
// reduces).  sp: SM_SPEC's list of the pixels it set.
template <int KS, int C, int TY, int MODE, bool BX, bool BY>
__device__ __forceinline__ void sweep_body(const ImgArgs& a, const Taps& tp,
                                           int x0, int y0, float thr2,
                                           float& gmax, SpecTile* sp) {
    using S = SweepShape<KS, C, TY, MODE>;
    constexpr int R = S::R, HX = S::HX, HL = S::HL, SW = S::SW, OW = S::OW;
    constexpr int NS = S::NS, NP = S::NP, P = S::P, PF = S::PF;

    const int lane = lane_id();
    const int H = a.H, W = a.W;
    const int xs = x0 - HL;
    const int cbase = xs + C * lane;
    const int ylim = min(y0 + TY, H);
    const bool lane_out = (cbase >= x0) & (cbase < x0 + OW);
    // Lanes whose every column has a valid G^2 (its neighbourhood lies in
    // the strip); outside the border variants those are all real pixels.
    const bool gvalid = (cbase >= xs + R + 1) & (cbase + C <= xs + SW - R - 1);
    bool ecol[C];
#pragma unroll
    for (int e = 0; e < C; ++e) ecol[e] = lane_out & (cbase + e < W);
    const bool vec_ok =
        ((reinterpret_cast<uintptr_t>(a.src) % (4 * C)) == 0) & ((a.sp % C) == 0);
    const bool mask_vec =
        ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) & ((a.mp % 4) == 0);

    auto load_row = [&](int v, float (&dst)[C]) {
        const int row = BY ? clampi(v, 0, H - 1) : v;
        const gptr<const float> rp = as_global(a.src) + (int64_t)row * a.sp;
        if (!BX && vec_ok) {
            const gptr<const VecF<C>> q = (gptr<const VecF<C>>)(rp + cbase);
#pragma unroll
            for (int e = 0; e < C; ++e) dst[e] = q->v[e];
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                dst[e] = rp[BX ? clampi(cbase + e, 0, W - 1) : cbase + e];
        }
    };
    auto store_f = [&](float* base, int row, const float (&val)[C]) {
        const gptr<float> rp = as_global(base) + (int64_t)row * a.op + cbase;
        if constexpr (!BX) {
            if (lane_out) {
                const gptr<VecF<C>> q = (gptr<VecF<C>>)rp;
#pragma unroll
                for (int e = 0; e < C; ++e) q->v[e] = val[e];
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
    uint32_t hz[P];   // per row: bit e = the 3-wide window at column e holds
                      // an L > 0 (bits 0..C-1) / holds only L > 0 (bits 8..)
    float g2d[C];     // G^2 of the row waiting for its Z
    float gacc = 0.0f;

    // One step; J = s mod P, DB/DC/DD: stages B, C, D are active; LD: the
    // step prefetches input row v + PF (every step but the last PF): 1
    // always, 0 never, 2 decided at run time.
    auto step = [&](auto jt, auto dbt, auto dct, auto ddt, auto ldt, int s) {
        constexpr int J = decltype(jt)::value;
        constexpr bool DB = decltype(dbt)::value != 0;
        constexpr bool DC = decltype(dct)::value != 0;
        constexpr bool DD = decltype(ddt)::value != 0;
        constexpr int LD = decltype(ldt)::value;
        constexpr int J1 = (J + P - 1) % P, J2 = (J + P - 2) % P;
        const int v = y0 - HX + s;
        if constexpr (LD == 1) load_row(v + PF, pf[(J + PF) % P]);
        if constexpr (LD == 2)
            if (s + PF < NS) load_row(v + PF, pf[(J + PF) % P]);

        // ---- A: horizontal blur of input row v
        {
            float ext[C + 2 * R];
            static_for([&](auto kt) {
                constexpr int kk = decltype(kt)::value - R;
                constexpr int q = kk >= 0 ? kk / C : -((-kk + C - 1) / C);
                ext[kk + R] = lane_fetch<q>(pf[J][kk - q * C]);
            }, std::make_integer_sequence<int, C + 2 * R>{});
#pragma unroll
            for (int e = 0; e < C; ++e) bh[J][e] = blur_chain<KS>(&ext[e], tp);
        }

        // ---- B: vertical blur, row vb = v - R
        if constexpr (DB) {
            const int vb = v - R;
            float b[C];
#pragma unroll
            for (int e = 0; e < C; ++e) {
                float col[KS];
#pragma unroll
                for (int i = 0; i < KS; ++i) col[i] = bh[(J - 2 * R + i + 4 * P) % P][e];
                b[e] = blur_chain<KS>(col, tp);
            }
            if constexpr (BY) {
                if (vb >= H) {
#pragma unroll
                    for (int e = 0; e < C; ++e) b[e] = bb[J1][e];
                }
            }
            if constexpr (BX) fix_cols<C, HL, SW>(b, x0, xs, cbase, W);
            const float bl0 = lane_fetch<-1>(b[C - 1]);
            const float br0 = lane_fetch<1>(b[0]);
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const float l = e > 0 ? b[e - 1] : bl0;
                const float r = e < C - 1 ? b[e + 1] : br0;
                bb[J][e] = b[e];
                ew[J][e] = l + r;
                dx[J][e] = sobel_dx(l, r);
                sy[J][e] = sobel_sy(ew[J][e], b[e]);
            }
            if constexpr (BY) {
                if (vb == 0) {  // the row above the image is row 0
#pragma unroll
                    for (int e = 0; e < C; ++e) {
                        bb[J1][e] = bb[J][e];
                        dx[J1][e] = dx[J][e];
                        sy[J1][e] = sy[J][e];
                    }
                }
            }
        }

        // ---- C: L and G^2 of row vl = v - R - 1
        if constexpr (DC) {
            const int vl = v - R - 1;
            float g2[C];
#pragma unroll
            for (int e = 0; e < C; ++e)
                g2[e] = sobel_g2(dx[J2][e], dx[J1][e], dx[J][e], sy[J2][e], sy[J][e]);
            if constexpr (S::DO_MAX) {
                if constexpr (!BX && !BY) {
                    // Every row of an interior tile is a real pixel row and
                    // max is idempotent: no per-row masking needed.
#pragma unroll
                    for (int e = 0; e + 1 < C; e += 2) gacc = max3f(gacc, g2[e], g2[e + 1]);
                    if constexpr (C % 2) gacc = __builtin_fmaxf(gacc, g2[C - 1]);
                } else {
                    if ((vl >= y0) & (vl < ylim)) {
#pragma unroll
                        for (int e = 0; e < C; ++e)
                            gacc = __builtin_fmaxf(gacc, ecol[e] ? g2[e] : 0.0f);
                    }
                }
            }
            const bool row_out = (vl >= y0) & (vl < ylim);
            if constexpr (MODE == SM_BG) {
                if (row_out) {
                    store_f(a.fout, vl, bb[J1]);
                    store_f(a.g2, vl, g2);
                }
            }
            if constexpr (S::NEED_L) {
                float l[C];
#pragma unroll
                for (int e = 0; e < C; ++e)
                    l[e] = lap_from(bb[J2][e] + bb[J][e], ew[J1][e], bb[J1][e]);
                if constexpr (MODE == SM_BGL) {
                    if (row_out) {
                        store_f(a.fout, vl, l);
                        store_f(a.g2, vl, g2);
                    }
                }
                if constexpr (S::NEED_Z) {
                    if constexpr (BX) fix_cols<C, HL, SW>(l, x0, xs, cbase, W);
                    // Z needs only the sign of L: whether the 3x3 window
                    // holds an L > 0 (its max is > 0) and whether it holds
                    // only L > 0 (its min is > 0).  Kept as bits, C per row.
                    // l > 0 exactly when its bits, read as a signed
                    // integer, are >= 1 (-0 reads as INT_MIN): clamping
                    // them to [0, 1] gives the bit without a compare.
                    uint32_t sg = 0;
#pragma unroll
                    for (int e = 0; e < C; ++e)
                        sg |= (uint32_t)min(max(__float_as_int(l[e]), 0), 1) << e;
                    const uint32_t sl = (uint32_t)__builtin_amdgcn_mov_dpp(
                        (int)sg, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
                    const uint32_t sr = (uint32_t)__builtin_amdgcn_mov_dpp(
                        (int)sg, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
                    // Bit e + 1 of ext is column e; bits 0 and C + 1 the
                    // neighbouring lanes' edge columns.
                    const uint32_t ext =
                        ((sl >> (C - 1)) & 1u) | (sg << 1) | ((sr & 1u) << (C + 1));
                    constexpr uint32_t CM = (1u << C) - 1u;
                    hz[J] = ((ext | (ext >> 1) | (ext >> 2)) & CM) |
                            (((ext & (ext >> 1) & (ext >> 2)) & CM) << 8);
                    if constexpr (BY) {
                        if (vl >= H) hz[J] = hz[J1];
                        if (vl == 0) hz[J1] = hz[J];
                    }
                    // ---- D: Z of row vz = vl - 1, and the output
                    if constexpr (DD) {
                        const int vz = vl - 1;
                        if (!BY || ((vz >= y0) & (vz < ylim))) {
                            const uint32_t any = hz[J2] | hz[J1] | hz[J];
                            const uint32_t all = hz[J2] & hz[J1] & hz[J];
                            const uint32_t zb = any & ~(all >> 8) & CM;
                            if constexpr (MODE == SM_STORE) {
                                float code[C];
#pragma unroll
                                for (int e = 0; e < C; ++e)
                                    code[e] = pass1_code((zb >> e) & 1u, g2d[e]);
                                store_f(a.fout, vz, code);
                            } else {
                                static_assert(C <= 4, "one mask byte per column in a word");
                                const gptr<uint8_t> rp =
                                    as_global(a.mask) + (int64_t)vz * a.mp + cbase;
                                // Mask byte e (bit 8e of mw) = Z and G^2 > thr2.
                                // G^2 > thr2 is the sign of thr2 - G^2 (exact
                                // for finite values: the difference of two
                                // different floats is never rounded to 0);
                                // Z's C bits are spread one per byte by a
                                // multiply.
                                uint32_t gw = 0;
#pragma unroll
                                for (int e = 0; e < C; ++e)
                                    gw |= (__float_as_uint(thr2 - g2d[e]) >> 31) << (8 * e);
                                const uint32_t mw = gw & ((zb * 0x00204081u) & 0x01010101u);
                                if (!BX && (C == 4) && mask_vec) {
                                    if (lane_out) *(gptr<uint32_t>)rp = mw;
                                } else {
#pragma unroll
                                    for (int e = 0; e < C; ++e)
                                        if (ecol[e]) rp[e] = (uint8_t)((mw >> (8 * e)) & 1u);
                                }
                                if constexpr (MODE == SM_SPEC) {
                                    // List the lanes that set a bit in this
                                    // row, packed in lane order after the
                                    // tile's earlier entries: their C values
                                    // of G^2, and row | lane | set columns.
                                    // The multiply gathers byte e's bit into
                                    // bit 24 + e.
                                    uint32_t bits = (mw * 0x01020408u) >> 24;
                                    if constexpr (BX) {
                                        uint32_t em = 0;
#pragma unroll
                                        for (int e = 0; e < C; ++e) em |= ecol[e] ? (1u << e) : 0u;
                                        bits &= em;
                                    } else {
                                        bits = lane_out ? bits : 0u;
                                    }
                                    const uint64_t bal = __ballot(bits != 0u);
                                    if (bal) {
                                        if (bits) {
                                            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(bal >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                                            const int64_t idx = (int64_t)(sp->n + below);
                                            const gptr<VecF<C>> q =
                                                (gptr<VecF<C>>)(as_global(sp->code) + idx * C);
#pragma unroll
                                            for (int e = 0; e < C; ++e) q->v[e] = g2d[e];
                                            as_global(sp->row)[idx] =
                                                (int32_t)(((uint32_t)(vz - y0) << 10) |
                                                          ((uint32_t)lane << 4) | bits);
                                        }
                                        sp->n += (uint32_t)__builtin_popcountll(bal);
                                    }
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int e = 0; e < C; ++e) g2d[e] = g2[e];
                }
            }
        }
    };

    // Prefetch, then the pipeline fill with compile-time stage flags.
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(y0 - HX + j, pf[j]);
    static_for([&](auto st) {
        constexpr int s = decltype(st)::value;
        step(IC<s % P>{}, IC<(s >= 2 * R)>{}, IC<(s >= 2 * R + 2)>{},
             IC<(s >= 2 * R + 4)>{}, IC<(s + PF < NS)>{}, s);
    }, std::make_integer_sequence<int, NP>{});
    // Steady state: every stage active, TY steps in groups of P.  With
    // S::EAGER every group but the last prefetches unconditionally, so no
    // load is conditional at run time and the wait before each use allows
    // the full prefetch depth in flight; the heavier modes keep the run-time
    // check, which holds their registers within three waves per SIMD.
    static_assert(PF <= P, "the last group holds every step without a prefetch");
    if constexpr (S::EAGER) {
        for (int s0 = NP; s0 < NS - P; s0 += P) {
            static_for([&](auto jt) {
                constexpr int jj = decltype(jt)::value;
                step(IC<(NP + jj) % P>{}, IC<1>{}, IC<1>{}, IC<1>{}, IC<1>{}, s0 + jj);
            }, std::make_integer_sequence<int, P>{});
        }
        static_for([&](auto jt) {
            constexpr int jj = decltype(jt)::value;
            step(IC<(NP + jj) % P>{}, IC<1>{}, IC<1>{}, IC<1>{}, IC<(jj + PF < P)>{},
                 NS - P + jj);
        }, std::make_integer_sequence<int, P>{});
    } else {
        for (int s0 = NP; s0 < NS; s0 += P) {
            static_for([&](auto jt) {
                constexpr int jj = decltype(jt)::value;
                step(IC<(NP + jj) % P>{}, IC<1>{}, IC<1>{}, IC<1>{}, IC<2>{}, s0 + jj);
            }, std::make_integer_sequence<int, P>{});
        }
    }
    if constexpr (!BX && !BY) gacc = gvalid ? gacc : 0.0f;
    gmax = __builtin_fmaxf(gmax, gacc);
}

template <int KS, int C, int TY, int MODE>
__device__ __forceinline__ void sweep_tile(const ImgArgs& a, const Taps& tp,
                                           int x0, int y0, float thr2,
                                           float& gmax, SpecTile* sp = nullptr) {
    using S = SweepShape<KS, C, TY, MODE>;
    const int xs = x0 - S::HL;
    const bool bx = (xs < 0) | (xs + S::SW > a.W);
    const bool by = (y0 - S::HX < 0) | (y0 + TY + S::HX > a.H);
    if (!bx & !by)
        sweep_body<KS, C, TY, MODE, false, false>(a, tp, x0, y0, thr2, gmax, sp);
    else if (!bx)
        sweep_body<KS, C, TY, MODE, false, true>(a, tp, x0, y0, thr2, gmax, sp);
    else if (!by)
        sweep_body<KS, C, TY, MODE, true, false>(a, tp, x0, y0, thr2, gmax, sp);
    else
        sweep_body<KS, C, TY, MODE, true, true>(a, tp, x0, y0, thr2, gmax, sp);
}

}  // namespace hx
