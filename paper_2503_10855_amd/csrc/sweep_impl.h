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
//      row pieces (e+w sums, Sobel sy),
//   C  forms L and G^2 of row v-R-1 from the last three B rows (n+s sums
//      and Sobel vs down each column), and the row's words of the signs of
//      L and of its 3-wide windows,
//   D  forms Z of row v-R-2 from three rows of window words and emits its
//      output.
// The first 2R+4 steps fill this pipeline and are unrolled with
// compile-time stage flags; the remaining `ty` steps (the tile height, a
// run-time multiple of the ring period P = 8) run as a loop unrolled by P,
// so every ring slot is a fixed register and the steady state has no stage
// conditions.  Every value is computed by the helpers in hx_device.h, in
// the same order as the depth-1 stage kernels, so all schedules agree bit
// for bit.
//
// Stages C and D keep a row's per-column decisions in one 32-bit word per
// lane, one byte per column (the layout of the lane's mask bytes): the
// signs of L (0/1), the 3-wide windows' "holds an L > 0" / "holds only
// L > 0" (OR / AND of the word and its copies shifted by one column, the
// neighbouring lanes' edge bytes shifted in by one DPP move and one
// alignbit each), and the threshold G^2 > thr2 as 0x00/0xff bytes (the
// sign bytes of thr2 - G^2 gathered by v_perm_b32).  Z over three rows is
// one OR3 and one AND3, and the mask word is Z AND the threshold bytes.
//
// Tiles whose whole input window lies inside the image (the common case)
// run an instantiation with no border logic at all.  The others run one
// that applies the clamped-coordinate rule per stage: rows -- the input
// row index is clamped; a B or L row below the image is a copy of the last
// real row; the row above the image is overwritten with row 0 as soon as
// row 0 exists (before any valid output reads it); columns -- the input
// column is clamped, and the B and L values of columns outside the image
// are replaced by the first / last real column's value.
//
// Addresses: a row's base address is wave-uniform (scalar registers) and
// each lane adds a 32-bit unsigned byte offset, so loads and stores use the
// scalar-base form and no per-lane 64-bit address arithmetic.
#pragma once

#include <utility>

#include "hx_kernels.h"

namespace hx {

template <int KS, int C, int MODE>
struct SweepShape {
    static constexpr int R = KS / 2;
    static constexpr int HX = R + 2;                       // chain halo
    static constexpr int HL = ((HX + C - 1) / C) * C;      // left halo
    static constexpr int SW = 64 * C;                      // strip width
    static constexpr int OW = ((SW - HL - HX) / C) * C;    // output width
    // Rows of halo above and below a tile: blur, Laplacian and zero
    // crossing need R + 2; blur and Sobel alone (the max-only sweep) R + 1.
    static constexpr int HY = MODE == SM_MAXONLY ? R + 1 : R + 2;
    static constexpr int NP = 2 * HY;                      // pipeline fill
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
    static_assert(KS <= P, "the horizontal-blur ring must hold k rows");
    static_assert(HY <= HX && NP <= 2 * R + 4, "stage D starts after the fill");
};

// Tile heights are multiples of the ring period.
constexpr int kSweepRowStep = 8;

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

// One bit per lane (bit i = lane i), held in scalar registers.
using lmask = uint64_t;

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

// 1 if l > 0, else 0 (for finite l): the bits of l as a signed integer,
// clamped to [0, 1] in one instruction.
__device__ __forceinline__ uint32_t pos_bit(float l) {
    uint32_t r;
    asm("v_med3_i32 %0, %1, 0, 1" : "=v"(r) : "v"(l));
    return r;
}

// Row words of stage D hold one byte per column of the lane (byte e =
// column e, bytes C..3 zero).  The low bytes of b[0..C-1] packed so.
template <int C>
__device__ __forceinline__ uint32_t col_bytes(const uint32_t (&b)[C]) {
    if constexpr (C == 4) {
        // Two byte gathers (v_perm_b32: selector 0x0c gives a zero byte).
        return __builtin_amdgcn_perm(b[1], b[0], 0x0c0c0400u) |
               __builtin_amdgcn_perm(b[3], b[2], 0x04000c0cu);
    } else {
        uint32_t w = b[0];
#pragma unroll
        for (int e = 1; e < C; ++e) w |= b[e] << (8 * e);
        return w;
    }
}

// Byte e = 0xff if t[e] has its sign bit set, else 0 (v_perm_b32 selectors
// 9 and 11 replicate the sign bit of byte 3 of its low / high source).
template <int C>
__device__ __forceinline__ uint32_t col_sign_bytes(const float (&t)[C]) {
    const uint32_t t0 = __float_as_uint(t[0]);
    if constexpr (C == 1) {
        return __builtin_amdgcn_perm(t0, t0, 0x0c0c0c09u);
    } else {
        const uint32_t lo = __builtin_amdgcn_perm(__float_as_uint(t[1]), t0, 0x0c0c0b09u);
        if constexpr (C == 2) return lo;
        else return lo | __builtin_amdgcn_perm(__float_as_uint(t[3]), __float_as_uint(t[2]),
                                               0x0b090c0cu);
    }
}

// A row word shifted by one column, the neighbouring lane's edge column
// shifted in: byte e of the result is column e-1 (from_left) or e+1
// (from_right) of the lane's row, counted across lanes.  Lanes at the
// wave's edges shift in 0 (such columns only feed discarded halo columns).
// For C < 4 bytes above C-1 of the result are not meaningful.
template <int C>
__device__ __forceinline__ uint32_t cols_from_left(uint32_t w) {
    const uint32_t xl =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
    if constexpr (C == 4) return __builtin_amdgcn_alignbit(w, xl, 24u);
    else return (w << 8) | (xl >> (8 * (C - 1)));
}
template <int C>
__device__ __forceinline__ uint32_t cols_from_right(uint32_t w) {
    const uint32_t xr =
        (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
    if constexpr (C == 4) return __builtin_amdgcn_alignbit(xr, w, 8u);
    else return (w >> 8) | (xr << (8 * (C - 1)));
}

// The set columns of a mask word (bytes 0/1) as bits 0..C-1.
__device__ __forceinline__ uint32_t col_nibble(uint32_t mw) {
    const uint32_t t = mw | (mw >> 7);
    return (t | (t >> 14)) & 0xfu;
}

// Keeps a value's computation in the current basic block: the DPP move
// that feeds it can then be folded into it (the compiler folds a move only
// into uses in its own block, and would otherwise sink some of these uses
// past the deferred stores' branches).
__device__ __forceinline__ void keep_here(float& v) { asm volatile("" : "+v"(v)); }

__device__ __forceinline__ float max3f(float a, float b, float c) {
    return __builtin_fmaxf(__builtin_fmaxf(a, b), c);
}

// A uniform pointer plus a per-lane 32-bit unsigned byte offset (the
// listing's scattered stores).
template <class T, class B>
__device__ __forceinline__ gptr<T> at_off(gptr<B> base, uint32_t byte_off) {
    return (gptr<T>)((gptr<char>)base + byte_off);
}

// Rows [row0, row0 + rows) of a pitched plane as a buffer resource: each
// access is the resource (scalar registers), a per-lane byte offset within
// the row (a vector register fixed for the tile) and the row's byte offset
// (a scalar register), so no address arithmetic runs per lane.  The
// resource's extent ends at element `width` of the last row: an access
// outside it reads 0 / is dropped instead of touching other memory.
struct RowSpan {
    __amdgpu_buffer_rsrc_t r;
    int row0;
    uint32_t pitch_bytes;
    __device__ __forceinline__ RowSpan(const void* base, int row0_, int rows,
                                       int64_t pitch_elems, int elem_bytes, int width) {
        row0 = row0_;
        pitch_bytes = (uint32_t)(pitch_elems * elem_bytes);
        const char* p = (const char*)base + (int64_t)row0_ * pitch_elems * elem_bytes;
        const uint32_t extent =
            (uint32_t)(rows - 1) * pitch_bytes + (uint32_t)width * (uint32_t)elem_bytes;
        // Word 3 of a gfx9 buffer resource: 32-bit data format, the rest 0.
        r = __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)extent, 0x00020000);
    }
    __device__ __forceinline__ uint32_t soff(int row) const {
        return (uint32_t)(row - row0) * pitch_bytes;
    }
};

template <int C>
__device__ __forceinline__ void span_load(const RowSpan& sp, int row, uint32_t voff,
                                          float (&dst)[C]) {
    if constexpr (C == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 v = __builtin_bit_cast(
            f4, __builtin_amdgcn_raw_buffer_load_b128(sp.r, voff, sp.soff(row), 0));
        dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
    } else if constexpr (C == 2) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = __builtin_bit_cast(
            f2, __builtin_amdgcn_raw_buffer_load_b64(sp.r, voff, sp.soff(row), 0));
        dst[0] = v.x; dst[1] = v.y;
    } else {
        dst[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(sp.r, voff, sp.soff(row), 0));
    }
}
__device__ __forceinline__ float span_load1(const RowSpan& sp, int row, uint32_t voff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(sp.r, voff, sp.soff(row), 0));
}
template <int C>
__device__ __forceinline__ void span_store(const RowSpan& sp, int row, uint32_t voff,
                                           const float (&val)[C]) {
    if constexpr (C == 4) {
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
        const u4 v = {__float_as_uint(val[0]), __float_as_uint(val[1]),
                      __float_as_uint(val[2]), __float_as_uint(val[3])};
        __builtin_amdgcn_raw_buffer_store_b128(v, sp.r, voff, sp.soff(row), 0);
    } else if constexpr (C == 2) {
        typedef uint32_t u2 __attribute__((ext_vector_type(2)));
        const u2 v = {__float_as_uint(val[0]), __float_as_uint(val[1])};
        __builtin_amdgcn_raw_buffer_store_b64(v, sp.r, voff, sp.soff(row), 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val[0]), sp.r, voff,
                                              sp.soff(row), 0);
    }
}

// Replace the values of columns outside [0, W) with column 0's / W-1's.
// Columns come in whole lanes on the left (the strip starts at a multiple
// of C), so the left fix is per lane; on the right, column W-1 is element
// `el` of lane `ln` (both wave-uniform): every element of that lane is read
// and one picked with scalar selects.  (Picking the element first with
// selects on the vector side lets the compiler index the lane's C values
// as an array in scratch memory, a load and a full memory wait per row.)
template <int C, int HL, int SW>
__device__ __forceinline__ void fix_cols(float (&x)[C], int x0, int xs,
                                         int cbase, int W) {
    if (x0 == 0) {
        // Column 0 sits in lane HL/C, element 0.
        const float v0 = __int_as_float(
            __builtin_amdgcn_readlane(__float_as_int(x[0]), HL / C));
#pragma unroll
        for (int e = 0; e < C; ++e)
            if (cbase < 0) x[e] = v0;
    }
    if (xs + SW > W) {
        const int cw = W - 1 - xs;
        const int ln = cw / C, el = cw - ln * C;
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

// Run one tile: output columns [x0, x0+OW) x rows [y0, y0+ty), clipped to
// the image; ty is a multiple of kSweepRowStep.  BX / BY: the tile's input
// window crosses a column / row border of the image; BX also serves images
// whose rows are not aligned for the vector accesses (it reads and writes
// one element at a time).  thr2 is used by
// SM_MASK and SM_SPEC only.  gmax accumulates G^2 over real image pixels
// of the tile (per lane; the caller reduces).  sp: SM_SPEC's list of the
// pixels it set; entries beyond sp->cap are counted but not written.
// up_req: sweep the tile bottom to top (tiles whose rows lie inside the
// image only; others always sweep down).  Every stage is symmetric under
// the flip -- the blur's pairs and the n+s sums add commutatively and gy
// only changes sign before it is squared -- so both directions give the
// same bits.  Neighbouring bands that sweep in opposite directions read
// their shared halo rows at the same time (both at the start, or both at
// the end of their sweeps), so the second read finds them in L2.
// BL (with !BX, C = 4): the tile's only column border is the image's left
// edge, and its rows are aligned: the vector path runs, and the lane just
// left of column 0 -- the only outside lane whose values reach an output --
// has its input samples, its B and its L replaced by column 0's (the
// clamped-coordinate rule per stage), 6 operations per row instead of the
// border variant's per-element loads and column fixes.  BR (with !BX,
// C = 4, W a multiple of 4): likewise for a tile whose only column border
// is the image's right edge: lanes right of column W-1 read columns
// W-4..W-1, and the first of them (the only one whose values reach an
// output) has its samples, B and L replaced by column W-1's; lanes right
// of the edge neither write nor count toward the max.
template <int KS, int C, int MODE, bool BX, bool BY, bool BL = false, bool BR = false,
          bool BA = false, bool BQ = false>
__device__ __forceinline__ void sweep_body(const ImgArgs& a, const Taps& tp,
                                           int x0, int y0, int ty, float thr2,
                                           float& gmax, SpecTile* sp, bool up_req) {
    using S = SweepShape<KS, C, MODE>;
    constexpr int R = S::R, HY = S::HY, HL = S::HL, SW = S::SW, OW = S::OW;
    constexpr int NP = S::NP, P = S::P, PF = S::PF;

#ifdef HX_TAPS_IN_VGPRS
    // The blur taps in vector registers (frees scalar registers).
    Taps tv;
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        float g = tp.g[i];
        asm("" : "+v"(g));
        tv.g[i] = g;
    }
#else
    // The blur taps stay in scalar registers (kernel arguments): each fma
    // takes one as its scalar operand, which leaves the vector registers
    // to the row rings.
    const Taps& tv = tp;
#endif

    const int lane = lane_id();
    const int H = a.H, W = a.W;
    const int NS = ty + 2 * HY;
    // Step t of the sweep reads input row row_at(t).
    const bool up = !BY && up_req;
    const int dir = up ? -1 : 1;
    const int vfirst = up ? y0 + ty - 1 + HY : y0 - HY;
    auto row_at = [&](int t) { return vfirst + dir * t; };
    const int xs = x0 - HL;
    const int cbase = xs + C * lane;
    // Byte offsets of the lane's first column in an input / mask row.  Only
    // lanes inside the image (or, in the border variants, with clamped
    // columns) ever access memory through them.
    static_assert(!BL || (!BX && C == 4 && (S::HL == 4 || S::HL == 8)),
                  "BL: one or two lanes left of column 0");
    static_assert(!BR || (!BX && C == 4), "BR: whole lanes right of column W-1");
    static_assert(!BA || (!BX && (!BR || BQ) && C == 4 && (MODE == SM_MASK || MODE == SM_SPEC)),
                  "BA: vector rows with mask rows that are not word aligned");
    static_assert(C != 4 || (S::HL % 4 == 0 && S::OW % 4 == 0),
                  "a lane's first column is a multiple of 4 from the row start");
    static_assert(!BQ || (BR && MODE != SM_STORE && MODE != SM_BG && MODE != SM_BGL),
                  "BQ: a right edge inside a lane");
    // BL: lanes left of column 0 read columns 0..C-1, BR: lanes right of
    // column W-1 read columns W-C..W-1 (their own values are replaced or
    // unused), so every access stays inside the image.
    const uint32_t off_in = (BL && cbase < 0)        ? 0u
                            : (BR && cbase + C > W) ? (uint32_t)(W - C) * 4u
                                                    : (uint32_t)cbase * 4u;
    const bool edge_lane = BL && lane == HL / C - 1;
    // BQ (W not a multiple of 4): the straddling lane holds columns
    // W-wr..W-wr+3, of which the first wr are inside the image; the lane
    // after it plays the edge lane's part.
    const int wr = W & 3;
    const bool strad = BQ && (cbase < W) && (cbase + C > W);
    const bool edge_lane_r = BR && (BQ ? (cbase >= W) & (cbase < W + C) : cbase == W);
    const uint32_t off_m = (uint32_t)cbase;
    const int ylim = min(y0 + ty, H);
    const bool lane_out = (cbase >= x0) & (cbase < x0 + OW) &
                          (!BR || (BQ ? cbase < W : cbase + C <= W));
    // Lanes whose every column has a valid G^2 (its neighbourhood lies in
    // the strip); outside the border variants those are all real pixels.
    const bool gvalid = (cbase >= xs + R + 1) & (cbase + C <= xs + SW - R - 1) &
                        (!BR || (BQ ? cbase < W : cbase + C <= W)) & (!BL || cbase >= 0);
    bool ecol[C];
#pragma unroll
    for (int e = 0; e < C; ++e) ecol[e] = lane_out & (cbase + e < W);
    // The lanes that own output columns, as a mask (interior tiles); with
    // BQ the straddling lane is apart (it writes single bytes).
    const lmask out_lanes = __ballot(lane_out & (!BQ || cbase + C <= W));
    const bool strad_out = BQ && lane_out && strad;
    const lmask strad_lanes = BQ ? __ballot(strad_out) : 0;
    // BQ: the straddling lane's per-column selections (wr is uniform):
    // samples from the loaded columns W-4..W-1, and the columns at and past
    // W that take column W-1's B and L (fixB[e]) or carry no G^2 (gkill[e]).
    bool s0v1 = false, s0v2 = false, s0v3 = false, s1v2 = false, s1v3 = false;
    bool fixB[C], gkill[C];
#pragma unroll
    for (int e = 0; e < C; ++e) {
        fixB[e] = strad && (e > 0) && (wr == e);
        gkill[e] = strad && (e >= wr);
    }
    if constexpr (BQ) {
        s0v1 = strad && wr == 3;
        s0v2 = strad && wr == 2;
        s0v3 = strad && wr == 1;
        s1v2 = strad && wr == 3;
        s1v3 = strad && wr <= 2;
    }
    // Border variants: the lanes that may write their mask row as one word
    // (all C columns inside the image, word-aligned mask rows).
    const bool mask_words = (C == 4) && ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) &&
                            ((a.mp % 4) == 0);
    const lmask word_lanes = mask_words ? __ballot(lane_out & (cbase + C <= W)) : 0;

    // The tile's input rows (clamped into the image), output rows.
    const int in0 = BY ? max(y0 - HY, 0) : y0 - HY;
    const int in1 = BY ? min(y0 + ty + HY, H) : y0 + ty + HY;
    const RowSpan src(a.src, in0, in1 - in0, a.sp, 4, W);
    const int nout = max(ylim - y0, 1);
    constexpr bool WRITES_MASK = MODE == SM_MASK || MODE == SM_SPEC;
    constexpr bool WRITES_F = MODE == SM_STORE || MODE == SM_BG || MODE == SM_BGL;
    constexpr bool WRITES_G = MODE == SM_BG || MODE == SM_BGL;
    const RowSpan msk(WRITES_MASK ? (const void*)a.mask : (const void*)a.src, y0, nout,
                      WRITES_MASK ? a.mp : 0, 1, W);
    // BA: the low two address bits of the tile's first mask row (a lane's
    // word then starts at those bits plus the row's offset, since its first
    // column is a multiple of 4).
    const uint32_t mlo =
        BA ? (uint32_t)(reinterpret_cast<uintptr_t>(a.mask) + (uint64_t)y0 * (uint64_t)a.mp) & 3u
           : 0u;
    const RowSpan fo(WRITES_F ? (const void*)a.fout : (const void*)a.src, y0, nout,
                     WRITES_F ? a.op : 0, 4, W);
    const RowSpan go(WRITES_G ? (const void*)a.g2 : (const void*)a.src, y0, nout,
                     WRITES_G ? a.op : 0, 4, W);

    auto load_row = [&](int v, float (&dst)[C]) {
        const int row = BY ? clampi(v, 0, H - 1) : v;
        if constexpr (!BX) {
            span_load<C>(src, row, off_in, dst);
            if constexpr (BL) {
                // The edge lane loaded columns 0..C-1: its samples of
                // columns -C..-1 are column 0's.
#pragma unroll
                for (int e = 1; e < C; ++e) dst[e] = edge_lane ? dst[0] : dst[e];
            }
            if constexpr (BR) {
                // The right edge lane loaded columns W-C..W-1: its samples
                // of columns W..W+C-1 are column W-1's.
#pragma unroll
                for (int e = 0; e < C - 1; ++e) dst[e] = edge_lane_r ? dst[C - 1] : dst[e];
            }
            if constexpr (BQ) {
                // The straddling lane loaded columns W-4..W-1: column
                // W-wr+e is loaded column min(4-wr+e, 3).
                const float v1 = dst[1], v2 = dst[2], v3 = dst[3];
                dst[0] = s0v3 ? v3 : (s0v2 ? v2 : (s0v1 ? v1 : dst[0]));
                dst[1] = s1v3 ? v3 : (s1v2 ? v2 : dst[1]);
                dst[2] = strad ? v3 : dst[2];
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                dst[e] = span_load1(src, row, 4u * (uint32_t)clampi(cbase + e, 0, W - 1));
        }
    };
    auto store_f = [&](const RowSpan& dst, int row, const float (&val)[C]) {
        if constexpr (!BX) {
            if (__builtin_amdgcn_inverse_ballot_w64(out_lanes)) span_store<C>(dst, row, off_in, val);
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ecol[e])
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(val[e]), dst.r,
                                                          off_in + 4u * e, dst.soff(row), 0);
        }
    };

    float pf[P][C];   // prefetched input rows
    float bh[P][C];   // horizontal blur rows
    float bb[P][C];   // B rows
    float ew[P][C];   // B(x-1) + B(x+1)
    float sy[P][C];   // Sobel sy
    uint32_t ho[P];   // per L row, byte e: the 3-wide window at column e
    uint32_t ha[P];   // holds an L > 0 (ho) / holds only L > 0 (ha), 0/1
    float g2d[C];     // G^2 of the row waiting for its Z
    uint32_t tbd = 0; // its threshold bytes (0xff where G^2 > thr2)
    float gacc = 0.0f;
    // The output row of stage D is written one step later, after the next
    // row's horizontal blur (flush_out): its stores are guarded by the lanes
    // that own output columns and, for SM_SPEC, the listing is a branch
    // taken only when the row set a bit.  Each of those ends a basic block;
    // deferring them keeps a row's integer work of stage D in one block with
    // the next row's float work, and the two overlap.
    // Pending: the row (vzl, valid if pv), its mask word (mwl) or pass-1
    // codes (cdl), and for SM_SPEC the lanes that set a bit (bal) with
    // their G^2 (g2l).
    bool pv = false;
    int vzl = 0;
    uint32_t mwl = 0;
    lmask bal = 0;      // SM_SPEC: the lanes of the pending row that set one
    float cdl[C];
    float g2l[C];
#pragma unroll
    for (int e = 0; e < C; ++e) {
        cdl[e] = 0.0f;
        g2l[e] = 0.0f;
    }
    // The lane's columns inside the image, as 0xff bytes (border variants).
    uint32_t emw = 0;
#pragma unroll
    for (int e = 0; e < C; ++e) emw |= ecol[e] ? (0xffu << (8 * e)) : 0u;
    auto flush_out = [&]() {
        if constexpr (S::NEED_Z) {
            if (pv) {
                if constexpr (MODE == SM_STORE) {
                    store_f(fo, vzl, cdl);
                } else {
                    if constexpr (!BX && C == 4 && !BA) {
                        if (__builtin_amdgcn_inverse_ballot_w64(out_lanes))
                            __builtin_amdgcn_raw_buffer_store_b32(mwl, msk.r, off_m,
                                                                  msk.soff(vzl), 0);
                    } else if constexpr (BA) {
                        // Mask rows that are not word aligned: the row's
                        // alignment is the same for every lane, so the
                        // word goes out as naturally aligned pieces (one
                        // word, two halves, or byte + half + byte).
                        const uint32_t so = msk.soff(vzl);
                        const uint32_t rem = (mlo + so) & 3u;
                        if (__builtin_amdgcn_inverse_ballot_w64(out_lanes)) {
                            if (rem == 0u) {
                                __builtin_amdgcn_raw_buffer_store_b32(mwl, msk.r, off_m, so, 0);
                            } else if (rem == 2u) {
                                __builtin_amdgcn_raw_buffer_store_b16(
                                    (unsigned short)(mwl & 0xffffu), msk.r, off_m, so, 0);
                                __builtin_amdgcn_raw_buffer_store_b16(
                                    (unsigned short)(mwl >> 16), msk.r, off_m + 2u, so, 0);
                            } else {
                                __builtin_amdgcn_raw_buffer_store_b8(
                                    (unsigned char)(mwl & 0xffu), msk.r, off_m, so, 0);
                                __builtin_amdgcn_raw_buffer_store_b16(
                                    (unsigned short)((mwl >> 8) & 0xffffu), msk.r, off_m + 1u,
                                    so, 0);
                                __builtin_amdgcn_raw_buffer_store_b8(
                                    (unsigned char)(mwl >> 24), msk.r, off_m + 3u, so, 0);
                            }
                        }
                    } else {
                        // Whole words for the lanes whose C columns are all
                        // inside the image (when mask rows are word
                        // aligned), single bytes for the rest.
                        if (__builtin_amdgcn_inverse_ballot_w64(word_lanes)) {
                            __builtin_amdgcn_raw_buffer_store_b32(mwl, msk.r, off_m,
                                                                  msk.soff(vzl), 0);
                        } else {
#pragma unroll
                            for (int e = 0; e < C; ++e)
                                if (ecol[e])
                                    __builtin_amdgcn_raw_buffer_store_b8(
                                        (uint8_t)((mwl >> (8 * e)) & 1u), msk.r, off_m + e,
                                        msk.soff(vzl), 0);
                        }
                    }
                    if constexpr (BQ) {
                        // The straddling lane: its wr columns inside the
                        // image, one byte each.
                        if (strad_out) {
                            const uint32_t so = msk.soff(vzl);
                            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)(mwl & 0xffu),
                                                                 msk.r, off_m, so, 0);
                            if (wr > 1)
                                __builtin_amdgcn_raw_buffer_store_b8(
                                    (unsigned char)((mwl >> 8) & 0xffu), msk.r, off_m + 1u, so, 0);
                            if (wr > 2)
                                __builtin_amdgcn_raw_buffer_store_b8(
                                    (unsigned char)((mwl >> 16) & 0xffu), msk.r, off_m + 2u, so, 0);
                        }
                    }
                }
                if constexpr (MODE == SM_SPEC) {
                    // The lanes that set a bit in the row, packed in lane
                    // order after the tile's earlier entries: their C values
                    // of G^2, and row | lane | set columns.
                    if (bal) {
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        const uint32_t idx = sp->n + below;
                        if (__builtin_amdgcn_inverse_ballot_w64(bal) & (idx < sp->cap)) {
                            const gptr<VecF<C>> q =
                                at_off<VecF<C>>(as_global(sp->code), idx * (uint32_t)(4 * C));
#pragma unroll
                            for (int e = 0; e < C; ++e) q->v[e] = g2l[e];
                            *at_off<int32_t>(as_global(sp->row), idx * 4u) =
                                (int32_t)(((uint32_t)(vzl - y0) << 10) |
                                          ((uint32_t)lane << 4) | col_nibble(mwl));
                        }
                        sp->n += (uint32_t)__builtin_popcountll(bal);
                    }
                }
                pv = false;
            }
        }
    };

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
        const int v = row_at(s);
        if constexpr (LD == 1) load_row(row_at(s + PF), pf[(J + PF) % P]);
        // LD == 2: past the tile's last input row the prefetch repeats that
        // row (its value is never used): every step loads, so the memory
        // wait before a row's use counts only the loads issued after it.
        if constexpr (LD == 2) load_row(row_at(min(s + PF, NS - 1)), pf[(J + PF) % P]);

        // ---- A: horizontal blur of input row v
        {
            float ext[C + 2 * R];
            static_for([&](auto kt) {
                constexpr int kk = decltype(kt)::value - R;
                constexpr int q = kk >= 0 ? kk / C : -((-kk + C - 1) / C);
                ext[kk + R] = lane_fetch<q>(pf[J][kk - q * C]);
            }, std::make_integer_sequence<int, C + 2 * R>{});
#pragma unroll
            for (int e = 0; e < C; ++e) {
                // The pairs that take a neighbouring lane's sample stay in
                // this block, where that sample's DPP move folds into them.
                float pair[R];
#pragma unroll
                for (int i = 1; i <= R; ++i) {
                    pair[i - 1] = blur_pair<KS>(&ext[e], i);
                    if (e - i < 0 || e + i >= C) keep_here(pair[i - 1]);
                }
                bh[J][e] = blur_from_pairs<KS>(ext[e + R], pair, tv);
            }
        }
        // The previous row's output, here: its branches then separate float
        // work of this row only, and no DPP move of stages B and C is split
        // from its use (a move whose use lies in another block cannot be
        // folded into it).
        flush_out();

        // ---- B: vertical blur, row vb = v - R
        if constexpr (DB) {
            const int vb = v - dir * R;
            float b[C];
#pragma unroll
            for (int e = 0; e < C; ++e) {
                float col[KS];
#pragma unroll
                for (int i = 0; i < KS; ++i) col[i] = bh[(J - 2 * R + i + 4 * P) % P][e];
                b[e] = blur_chain<KS>(col, tv);
            }
            if constexpr (BY) {
                if (vb >= H) {
#pragma unroll
                    for (int e = 0; e < C; ++e) b[e] = bb[J1][e];
                }
            }
            if constexpr (BX) fix_cols<C, HL, SW>(b, x0, xs, cbase, W);
            if constexpr (BL) {
                const float b0 = lane_fetch<1>(b[0]);
                b[C - 1] = edge_lane ? b0 : b[C - 1];
            }
            if constexpr (BR && !BQ) {
                const float bw = lane_fetch<-1>(b[C - 1]);
                b[0] = edge_lane_r ? bw : b[0];
            }
            if constexpr (BQ) {
                // Column W of the straddling lane takes column W-1's B.
#pragma unroll
                for (int e = 1; e < C; ++e) b[e] = fixB[e] ? b[e - 1] : b[e];
            }
            const float bl0 = lane_fetch<-1>(b[C - 1]);
            const float br0 = lane_fetch<1>(b[0]);
#pragma unroll
            for (int e = 0; e < C; ++e) {
                const float l = e > 0 ? b[e - 1] : bl0;
                const float r = e < C - 1 ? b[e + 1] : br0;
                bb[J][e] = b[e];
                ew[J][e] = l + r;
                if (e == 0 || e == C - 1) keep_here(ew[J][e]);
                sy[J][e] = sobel_sy(ew[J][e], b[e]);
            }
            if constexpr (BY) {
                if (vb == 0) {  // the row above the image is row 0
#pragma unroll
                    for (int e = 0; e < C; ++e) {
                        bb[J1][e] = bb[J][e];
                        sy[J1][e] = sy[J][e];
                    }
                }
            }
        }

        // ---- C: L and G^2 of row vl = v - R - 1
        if constexpr (DC) {
            const int vl = v - dir * (R + 1);
            // ns and vs down each column; gx from the neighbouring
            // columns' vs (the outer ones from the adjacent lanes).
            float ns[C], vs[C], g2[C];
#pragma unroll
            for (int e = 0; e < C; ++e) {
                ns[e] = bb[J2][e] + bb[J][e];
                vs[e] = sobel_vs(ns[e], bb[J1][e]);
            }
            const float vsl0 = lane_fetch<-1>(vs[C - 1]);
            const float vsr0 = lane_fetch<1>(vs[0]);
#pragma unroll
            for (int e = 0; e < C; ++e)
                g2[e] = sobel_g2(e > 0 ? vs[e - 1] : vsl0, e < C - 1 ? vs[e + 1] : vsr0,
                                 sy[J2][e], sy[J][e]);
            keep_here(g2[0]);
            if constexpr (C > 1) keep_here(g2[C - 1]);
            if constexpr (S::DO_MAX) {
                if constexpr (!BX && !BY) {
                    // Every row of an interior tile is a real pixel row and
                    // max is idempotent: no per-row masking needed.
                    if constexpr (BQ) {
#pragma unroll
                        for (int e = 1; e < C; ++e) g2[e] = gkill[e] ? 0.0f : g2[e];
                    }
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
                    store_f(fo, vl, bb[J1]);
                    store_f(go, vl, g2);
                }
            }
            if constexpr (S::NEED_L) {
                float l[C];
#pragma unroll
                for (int e = 0; e < C; ++e)
                    l[e] = lap_from(ns[e], ew[J1][e], bb[J1][e]);
                if constexpr (MODE == SM_BGL) {
                    if (row_out) {
                        store_f(fo, vl, l);
                        store_f(go, vl, g2);
                    }
                }
                if constexpr (S::NEED_Z) {
                    if constexpr (BX) fix_cols<C, HL, SW>(l, x0, xs, cbase, W);
                    if constexpr (BL) {
                        const float l0 = lane_fetch<1>(l[0]);
                        l[C - 1] = edge_lane ? l0 : l[C - 1];
                    }
                    if constexpr (BR && !BQ) {
                        const float lw = lane_fetch<-1>(l[C - 1]);
                        l[0] = edge_lane_r ? lw : l[0];
                    }
                    if constexpr (BQ) {
#pragma unroll
                        for (int e = 1; e < C; ++e) l[e] = fixB[e] ? l[e - 1] : l[e];
                    }
                    // Z needs only the sign of L: 1 if L > 0 (L's bits,
                    // read as a signed integer, are >= 1; -0 reads as
                    // INT_MIN), one byte per column.
                    uint32_t sb[C];
#pragma unroll
                    for (int e = 0; e < C; ++e) sb[e] = pos_bit(l[e]);
                    const uint32_t sw = col_bytes<C>(sb);
                    const uint32_t sl = cols_from_left<C>(sw), sr = cols_from_right<C>(sw);
                    ho[J] = sw | sl | sr;
                    ha[J] = sw & sl & sr;
                    if constexpr (BY) {
                        if (vl >= H) {
                            ho[J] = ho[J1];
                            ha[J] = ha[J1];
                        }
                        if (vl == 0) {
                            ho[J1] = ho[J];
                            ha[J1] = ha[J];
                        }
                    }
                    // ---- D: Z of row vz = vl - 1, and the output
                    if constexpr (DD) {
                        const int vz = vl - dir;
                        if (!BY || ((vz >= y0) & (vz < ylim))) {
                            // Over the three rows: the window holds an L > 0
                            // and not only L > 0.
                            const uint32_t any = ho[J2] | ho[J1] | ho[J];
                            const uint32_t all = ha[J2] & ha[J1] & ha[J];
                            if constexpr (MODE == SM_STORE) {
                                const uint32_t zw = any & ~all;
#pragma unroll
                                for (int e = 0; e < C; ++e)
                                    cdl[e] = pass1_code((zw >> (8 * e)) & 1u, g2d[e]);
                            } else {
                                static_assert(C <= 4, "one mask byte per column in a word");
                                // Mask byte e = Z and G^2 > thr2: 0 or 1.
                                uint32_t mw = any & ~all & tbd;
                                if constexpr (BX || BQ) mw &= emw;
                                mwl = mw;
                                if constexpr (MODE == SM_SPEC) {
                                    bal = __ballot(mw != 0u);
                                    if constexpr (!BX) bal &= out_lanes | strad_lanes;
#pragma unroll
                                    for (int e = 0; e < C; ++e) g2l[e] = g2d[e];
                                }
                            }
                            vzl = vz;
                            pv = true;
                        }
                    }
#pragma unroll
                    for (int e = 0; e < C; ++e) g2d[e] = g2[e];
                    if constexpr (MODE == SM_MASK || MODE == SM_SPEC) {
                        // The row's threshold: the sign of thr2 - G^2 is set
                        // exactly when G^2 > thr2 (a difference of finite
                        // values is 0 only when they are equal, and then +0).
                        float t[C];
#pragma unroll
                        for (int e = 0; e < C; ++e) t[e] = thr2 - g2[e];
                        tbd = col_sign_bytes<C>(t);
                    }
                }
            }
        }
    };

    // Prefetch, then the pipeline fill with compile-time stage flags.
#pragma unroll
    for (int j = 0; j < PF; ++j) load_row(row_at(j), pf[j]);
    static_for([&](auto st) {
        constexpr int s = decltype(st)::value;
        step(IC<s % P>{}, IC<(s >= 2 * R)>{}, IC<(s >= 2 * R + 2)>{},
             IC<(s >= 2 * R + 4)>{}, IC<1>{}, s);
    }, std::make_integer_sequence<int, NP>{});
    static_assert(NP + PF <= NP + kSweepRowStep, "the fill prefetches within the tile");
    // Steady state: every stage active, ty steps in groups of P.  With
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
    flush_out();
    if constexpr (!BX && !BY) gacc = gvalid ? gacc : 0.0f;
    gmax = __builtin_fmaxf(gmax, gacc);
}

template <int KS, int C, int MODE>
__device__ __forceinline__ void sweep_tile(const ImgArgs& a, const Taps& tp,
                                           int x0, int y0, int ty, float thr2,
                                           float& gmax, SpecTile* sp = nullptr,
                                           bool up = false) {
    using S = SweepShape<KS, C, MODE>;
    // A tile must start inside the image: its row spans are built from
    // the rows it covers there.
    if (y0 >= a.H || x0 >= a.W) return;
    const int xs = x0 - S::HL;
    // A tile that reaches the image's bottom runs only the rows the image
    // still has, rounded up to the row step (its output rows are the same;
    // a full-height sweep would compute up to ty - 8 rows of clamped rows).
    ty = min(ty, (a.H - y0 + kSweepRowStep - 1) / kSweepRowStep * kSweepRowStep);
    // Vector rows.  Input rows that start on 4C-byte boundaries always take
    // them; with C = 4, in the modes that write no float plane, rows that
    // start on a word boundary do too (a 16-byte load needs only a 4-byte
    // aligned address; such a row only touches one more cache line per
    // wave).  Mask rows that are not word aligned take the BA variant,
    // which stores each lane's mask word as aligned pieces.
    constexpr bool WRITES_MASK = MODE == SM_MASK || MODE == SM_SPEC;
    constexpr bool WRITES_F = MODE == SM_STORE || MODE == SM_BG || MODE == SM_BGL;
    const bool src_al = ((reinterpret_cast<uintptr_t>(a.src) % (4 * C)) == 0) & ((a.sp % C) == 0);
    const bool vec_ok = (C == 4 && !WRITES_F) ? (reinterpret_cast<uintptr_t>(a.src) % 4) == 0
                                              : src_al;
    const bool mask_al = ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) & ((a.mp % 4) == 0);
    constexpr bool kHasBA = C == 4 && WRITES_MASK;
    // The common case first: the tile's window lies inside the image and
    // its rows are aligned (the same choice the checks below make for it,
    // reached without evaluating them).
    {
        const bool by0 = (y0 - S::HY < 0) | (y0 + ty + S::HY > a.H);
        if ((xs >= 0) & (xs + S::SW <= a.W) & src_al & (!WRITES_MASK || (C == 4 && mask_al)) &
            !by0) {
            sweep_body<KS, C, MODE, false, false>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
            return;
        }
    }
    const bool mask_vec = !WRITES_MASK || C == 4;
    const bool ba = kHasBA && !mask_al;
    const bool bx = (xs < 0) | (xs + S::SW > a.W) | !vec_ok | !mask_vec;
    // Left border only, vector rows: the vector path with the edge lane's
    // values fixed (C = 4 and a left halo of one lane, k <= 5, or two, k = 7:
    // only the lane just left of column 0 reaches an output, since no stage
    // reaches further than 3 columns and B and L at column -1 are fixed).
    constexpr bool kHasBL = C == 4 && (S::HL == 4 || S::HL == 8);
    const bool bl = kHasBL && (xs < 0) & (xs + S::SW <= a.W) & vec_ok & mask_vec;
    // Right border only, 4C-byte aligned input rows, word-aligned mask rows
    // and a width that is a multiple of 4.
    constexpr bool kHasBR = C == 4;
    const bool br = kHasBR && (xs >= 0) & (xs + S::SW > a.W) & ((a.W % C) == 0) & src_al &
                    (!WRITES_MASK || mask_al);
    // Right border only, vector rows, W not a multiple of 4 (BQ): the
    // straddling lane and the lane after it must both lie in the strip.
    constexpr bool kHasBQ = C == 4 && !WRITES_F;
    const bool bq = kHasBQ && (xs >= 0) & (xs + S::SW > a.W) & ((a.W % C) != 0) &
                    (a.W - (a.W % C) + 2 * C <= xs + S::SW) & vec_ok & mask_vec;
    const bool by = (y0 - S::HY < 0) | (y0 + ty + S::HY > a.H);
    if constexpr (kHasBQ) {
        if (bq) {
            if (!ba) {
                if (!by)
                    sweep_body<KS, C, MODE, false, false, false, true, false, true>(
                        a, tp, x0, y0, ty, thr2, gmax, sp, up);
                else
                    sweep_body<KS, C, MODE, false, true, false, true, false, true>(
                        a, tp, x0, y0, ty, thr2, gmax, sp, up);
            } else if constexpr (kHasBA) {
                if (!by)
                    sweep_body<KS, C, MODE, false, false, false, true, true, true>(
                        a, tp, x0, y0, ty, thr2, gmax, sp, up);
                else
                    sweep_body<KS, C, MODE, false, true, false, true, true, true>(
                        a, tp, x0, y0, ty, thr2, gmax, sp, up);
            }
            return;
        }
    }
    // Both borders in one strip (an image narrower than the strip, modes
    // that write no float plane): the left edge lane's fixes and the
    // right edge's together; they touch different lanes once W >= 2C.
    if constexpr (kHasBL && kHasBQ) {
        const bool bn = (xs < 0) & (xs + S::SW > a.W) & (a.W >= 2 * C) & vec_ok & mask_vec;
        if (bn) {
            if ((a.W % C) == 0) {
                if (src_al & (!WRITES_MASK || mask_al) & (a.W + C <= xs + S::SW)) {
                    if (!by)
                        sweep_body<KS, C, MODE, false, false, true, true>(a, tp, x0, y0, ty, thr2,
                                                                          gmax, sp, up);
                    else
                        sweep_body<KS, C, MODE, false, true, true, true>(a, tp, x0, y0, ty, thr2,
                                                                         gmax, sp, up);
                    return;
                }
            } else if (a.W - (a.W % C) + 2 * C <= xs + S::SW) {
                if (!ba) {
                    if (!by)
                        sweep_body<KS, C, MODE, false, false, true, true, false, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                    else
                        sweep_body<KS, C, MODE, false, true, true, true, false, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                } else if constexpr (kHasBA) {
                    if (!by)
                        sweep_body<KS, C, MODE, false, false, true, true, true, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                    else
                        sweep_body<KS, C, MODE, false, true, true, true, true, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                }
                return;
            }
        }
    }
    if constexpr (kHasBL) {
        if (bl) {
            if constexpr (kHasBA) {
                if (ba) {
                    if (!by)
                        sweep_body<KS, C, MODE, false, false, true, false, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                    else
                        sweep_body<KS, C, MODE, false, true, true, false, true>(
                            a, tp, x0, y0, ty, thr2, gmax, sp, up);
                    return;
                }
            }
            if (!by)
                sweep_body<KS, C, MODE, false, false, kHasBL>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
            else
                sweep_body<KS, C, MODE, false, true, kHasBL>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
            return;
        }
    }
    if constexpr (kHasBR) {
        if (br) {
            if (!by)
                sweep_body<KS, C, MODE, false, false, false, kHasBR>(a, tp, x0, y0, ty, thr2,
                                                                     gmax, sp, up);
            else
                sweep_body<KS, C, MODE, false, true, false, kHasBR>(a, tp, x0, y0, ty, thr2,
                                                                    gmax, sp, up);
            return;
        }
    }
    if constexpr (kHasBA) {
        if (!bx & ba) {
            if (!by)
                sweep_body<KS, C, MODE, false, false, false, false, true>(a, tp, x0, y0, ty, thr2,
                                                                          gmax, sp, up);
            else
                sweep_body<KS, C, MODE, false, true, false, false, true>(a, tp, x0, y0, ty, thr2,
                                                                         gmax, sp, up);
            return;
        }
    }
    if (!bx & !by)
        sweep_body<KS, C, MODE, false, false>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
    else if (!bx)
        sweep_body<KS, C, MODE, false, true>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
    else if (!by)
        sweep_body<KS, C, MODE, true, false>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
    else
        sweep_body<KS, C, MODE, true, true>(a, tp, x0, y0, ty, thr2, gmax, sp, up);
}

}  // namespace hx
