// k_srad.hip -- SRAD (speckle reducing anisotropic diffusion), the second
// stencil + sum-reduction workload (Evaluation; Use and Impact of
// Schedules: its loops fused and its sums turned into a three-level
// reduction tree).  Per iteration, with the whole image as the region of
// interest and clamped neighbours:
//   q0^2 = var(J) / mean(J)^2                    (two sums over the image)
//   c    = 1 / (1 + (q^2 - q0^2) / (q0^2 (1 + q0^2))), clamped to [0, 1],
//          q^2 from the four differences dN, dS, dW, dE of each pixel
//   J'   = J + lambda/4 (c dN + c_S dS + c dW + c_E dE)
//
// Every kernel is a register sweep: a wave64 owns a strip of 256 columns
// (4 per lane, 16-byte loads) and a band of kBH rows, and walks the band
// top to bottom keeping the last rows in registers; west / east
// neighbours come from the adjacent lane by DPP, and the strip's outer
// neighbours from one extra load per row.  Loads run kRing rows ahead.
// Workgroups (4 waves, 4 adjacent strips) are numbered so that each XCD
// takes a contiguous range of bands: the rows and columns two bands or
// strips share are then fetched once into that XCD's L2.
//
// Two forms, bit-identical to each other:
//   unfused  k_srad_sweep<kCoeff> writes c; <kUpdate> reads it, writes J'
//   fused    k_srad_sweep<kFused> computes c in registers one row ahead
//            of the update: c never reaches HBM.
// c is the paper's expression multiplied through by (4 J + sum d)^2, which
// for positive images is the same function and needs one reciprocal:
//   q^2 = (8 sum d^2 - (sum d)^2) / (sum of the four neighbours)^2.
// The sums of J' for the next iteration are folded with one pixel map:
// per lane in row order (level 1, fp64), xor-shuffled across the wave and
// added over the workgroup's 4 waves in a fixed order (level 2), and the
// next kernel's every workgroup adds all the workgroup pairs in a fixed
// order before its sweep (level 3) -- no separate statistics kernel, and
// the same bits for both forms and every run.
#include <hip/hip_runtime.h>

#include "srad_kernels.h"

namespace hx {
namespace {

#ifndef HX_SRAD_BH
#define HX_SRAD_BH 32
#endif
#ifndef HX_SRAD_RING
#define HX_SRAD_RING 4
#endif
constexpr int kSW = 256;          // strip width: 64 lanes x 4 columns
constexpr int kBH = HX_SRAD_BH;   // band height
constexpr int kRing = HX_SRAD_RING;   // rows the fused sweep loads ahead
static_assert(kBH >= 1 && kBH <= 63, "kBH + 1 rows of east c must fit one VGPR");
static_assert(kRing % 4 == 0, "the fused sweep's 4-row window must divide the ring");
enum { kFused = 0, kCoeff = 1, kUpdate = 2, kSums = 3 };

typedef float v4f __attribute__((ext_vector_type(4)));

struct SradArgs {
    const float* J;      // input plane of this iteration
    float* out;          // J' (fused, update) or c (coeff)
    const float* c;      // c plane (update)
    int64_t pin, pout, pc;
    const double* prev;  // workgroup partial pairs of the sums of J (fused, coeff)
    double* part;        // this kernel's workgroup partial pairs (fused, update, sums)
    double* q_log;       // nullable: q0^2 of iteration `it`
    int H, W, nstrips, nitems, nprev, it;
    float step;          // lambda / 4
    int vin, vout, vc;   // rows of J / out / c are 16-byte aligned
};

__device__ __forceinline__ int clampi_s(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Workgroup b runs on XCD b % 8; give each XCD a contiguous range.
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Lane l takes lane l-1's v (lane 0 keeps `old`) / lane l+1's v (lane 63
// keeps `old`).
__device__ __forceinline__ float from_west(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(
        __float_as_int(old), __float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_east(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(
        __float_as_int(old), __float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, false));
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// c of a pixel of value j with neighbours n, s, w, e (one fixed order).
// K = 1 / (q0 (1 + q0)); lo = 1 when q0^2 <= 0 (c = 1 then), else 0.
__device__ __forceinline__ float srad_c(float j, float n, float s, float w, float e,
                                        float q0, float K, float lo) {
    const float dN = n - j, dS = s - j, dW = w - j, dE = e - j;
    const float t = (n + s) + (w + e);                  // 4 j + sum d
    const float s1 = fmaf(-4.0f, j, t);                 // sum d
    const float s2 = fmaf(dN, dN, fmaf(dS, dS, fmaf(dW, dW, dE * dE)));
    const float num = fmaf(-s1, s1, 8.0f * s2);         // q^2 = num / t^2
    const float p = t * t;
    const float den = fmaf(fmaf(-q0, p, num), K, p);    // t^2 (1 + (q^2 - q0) K)
    return __builtin_amdgcn_fmed3f(p * __builtin_amdgcn_rcpf(den), lo, 1.0f);
}

// J' of a pixel.  At the last row / column the clamped neighbour equals
// the pixel, so dS / dE is +0 and c_S / c_E (any value in [0, 1]) drops
// out: the sweeps need not clamp them.
__device__ __forceinline__ float srad_new(float j, float n, float s, float w, float e,
                                          float c, float cS, float cE, float step) {
    const float dN = n - j, dS = s - j, dW = w - j, dE = e - j;
    const float D = fmaf(c, dN, fmaf(cS, dS, fmaf(c, dW, cE * dE)));
    return fmaf(step, D, j);
}

// One loaded row of a strip: 4 columns per lane plus one outer value
// (lane 0: column x0 - 1, every other lane: column x0 + 256; clamped).
struct Raw {
    float v[4];
    float ex;
};
struct Row {
    float v[4];
    float w, e;   // neighbours of columns 0 and 3
};
struct Pair {
    Raw j, c;
};

// Element i of a row whose base is uniform: a 32-bit byte offset from a
// scalar base (the global_load saddr form, no 64-bit vector address).
template <class T>
__device__ __forceinline__ T& at(const float* row, uint32_t i) {
    return *(T*)((const char*)row + (i << 2));
}

// The wave's strip and band.  FULL: the strip lies inside the image and
// every plane it touches has 16-byte-aligned rows.
struct Strip {
    int x0, y0, y1, H, W, lane;
};

template <bool FULL>
__device__ __forceinline__ Raw load_row(const float* P, int64_t pitch, int r, const Strip& g) {
    const float* row = P + (int64_t)clampi_s(r, 0, g.H - 1) * pitch;
    const uint32_t x = (uint32_t)(g.x0 + 4 * g.lane);
    Raw o;
    if constexpr (FULL) {
        const v4f t = at<const v4f>(row, x);
        o.v[0] = t.x;
        o.v[1] = t.y;
        o.v[2] = t.z;
        o.v[3] = t.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            o.v[k] = at<const float>(row, x + k < (uint32_t)g.W ? x + k : (uint32_t)(g.W - 1));
    }
    const int xe = g.lane == 0 ? (g.x0 > 0 ? g.x0 - 1 : 0)
                               : (g.x0 + kSW < g.W ? g.x0 + kSW : g.W - 1);
    o.ex = at<const float>(row, (uint32_t)xe);
    return o;
}

template <bool FULL>
__device__ __forceinline__ void store_row(float* P, int64_t pitch, int y, const Strip& g,
                                          const float (&v)[4]) {
    float* row = P + (int64_t)y * pitch;
    const uint32_t x = (uint32_t)(g.x0 + 4 * g.lane);
    if constexpr (FULL) {
        v4f t;
        t.x = v[0];
        t.y = v[1];
        t.z = v[2];
        t.w = v[3];
        at<v4f>(row, x) = t;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (x + k < (uint32_t)g.W) at<float>(row, x + k) = v[k];
    }
}

__device__ __forceinline__ Row with_nb(const Raw& r) {
    Row o;
#pragma unroll
    for (int k = 0; k < 4; ++k) o.v[k] = r.v[k];
    o.w = from_west(r.ex, r.v[3]);
    o.e = from_east(r.ex, r.v[0]);
    return o;
}
__device__ __forceinline__ float west_of(const Row& r, int k) { return k ? r.v[k - 1] : r.w; }
__device__ __forceinline__ float east_of(const Row& r, int k) { return k < 3 ? r.v[k + 1] : r.e; }

// Sums of the row's pixels (level 1: fp64, row order, column order);
// columns past the image add zero, which leaves the sums' bits unchanged.
template <bool FULL>
__device__ __forceinline__ void accumulate(const float (&v)[4], const Strip& g, double& s,
                                           double& s2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float f = v[k];
        if constexpr (!FULL) f = g.x0 + 4 * g.lane + k < g.W ? f : 0.0f;
        const double d = (double)f;
        s += d;
        s2 = __builtin_fma(d, d, s2);
    }
}

// Rows t = 0 .. n-1 of a sweep: load(t) fetches row t, pro(row, t) takes
// the first P rows (t a constant after unrolling) and step(row, t) every
// later one.  Loads run R rows ahead; past the last row they fetch it
// again (in bounds, unused).  The R-row groups of the main loop are
// unconditional, so a register window whose length divides R rotates
// without copies.  Requires n >= P.
template <int P, int R, class LoadF, class ProF, class StepF>
__device__ __forceinline__ void sweep_rows(int n, LoadF&& load, ProF&& pro, StepF&& step) {
    using T = decltype(load(0));
    T head[P], ring[R];
#pragma unroll
    for (int t = 0; t < P; ++t) head[t] = load(t);
#pragma unroll
    for (int k = 0; k < R; ++k) ring[k] = load(P + k < n ? P + k : n - 1);
#pragma unroll
    for (int t = 0; t < P; ++t) pro(head[t], t);
    int s = P;
    for (; s + R <= n; s += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T in = ring[k];
            const int nx = s + k + R;
            ring[k] = load(nx < n ? nx : n - 1);
            step(in, s + k);
        }
    }
#pragma unroll
    for (int k = 0; k < R - 1; ++k)
        if (s + k < n) step(ring[k], s + k);
}

// The four sweeps.  q0, K, lo: the iteration's constants (fused, coeff).
template <bool FULL>
__device__ __forceinline__ void sweep_sums(const SradArgs& a, const Strip& g, double& s,
                                           double& s2) {
    auto load = [&](int t) { return load_row<FULL>(a.J, a.pin, g.y0 + t, g); };
    auto take = [&](const Raw& in, int) { accumulate<FULL>(in.v, g, s, s2); };
    sweep_rows<1, 4>(g.y1 - g.y0, load, take, take);
}

// J rows y0-1 .. y1; at row t >= 2, c of image row y0 + t - 2.
template <bool FULL>
__device__ __forceinline__ void sweep_coeff(const SradArgs& a, const Strip& g, float q0,
                                            float K, float lo) {
    Row j0{}, j1{}, j2{};
    auto load = [&](int t) { return load_row<FULL>(a.J, a.pin, g.y0 - 1 + t, g); };
    auto push = [&](const Raw& in) {
        j2 = j1;
        j1 = j0;
        j0 = with_nb(in);
    };
    sweep_rows<2, 6>(
        g.y1 - g.y0 + 2, load, [&](const Raw& in, int) { push(in); },
        [&](const Raw& in, int t) {
            push(in);
            float c[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                c[k] = srad_c(j1.v[k], j2.v[k], j0.v[k], west_of(j1, k), east_of(j1, k), q0,
                              K, lo);
            store_row<FULL>(a.out, a.pout, g.y0 + t - 2, g, c);
        });
}

// J and c rows y0-1 .. y1; at row t >= 2, J' of image row y0 + t - 2.
template <bool FULL>
__device__ __forceinline__ void sweep_update(const SradArgs& a, const Strip& g, double& s,
                                             double& s2) {
    Row j0{}, j1{}, j2{};
    float c0[4] = {}, c1[4] = {}, c0e = 0.0f, c1e = 0.0f;
    auto load = [&](int t) {
        return Pair{load_row<FULL>(a.J, a.pin, g.y0 - 1 + t, g),
                    load_row<FULL>(a.c, a.pc, g.y0 - 1 + t, g)};
    };
    auto push = [&](const Pair& in) {
        j2 = j1;
        j1 = j0;
        j0 = with_nb(in.j);
#pragma unroll
        for (int k = 0; k < 4; ++k) c1[k] = c0[k];
        c1e = c0e;
#pragma unroll
        for (int k = 0; k < 4; ++k) c0[k] = in.c.v[k];
        c0e = from_east(in.c.ex, in.c.v[0]);
    };
    sweep_rows<2, 6>(
        g.y1 - g.y0 + 2, load, [&](const Pair& in, int) { push(in); },
        [&](const Pair& in, int t) {
            push(in);
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[k] = srad_new(j1.v[k], j2.v[k], j0.v[k], west_of(j1, k), east_of(j1, k),
                                c1[k], c0[k], k < 3 ? c1[k + 1] : c1e, a.step);
            store_row<FULL>(a.out, a.pout, g.y0 + t - 2, g, v);
            accumulate<FULL>(v, g, s, s2);
        });
}

// Fused.  J rows y0-1 .. y1+1; at row t >= 2, c of image row y0 + t - 2
// (into c1, the previous c1 moving to c2); at t >= 3, J' of row y0 + t - 3.
template <bool FULL>
__device__ __forceinline__ void sweep_fused(const SradArgs& a, const Strip& g, float q0,
                                            float K, float lo, double& s, double& s2) {
    const int H = g.H, W = g.W;
    // c of the column right of the strip, rows y0 .. y1, one row per lane.
    float ce = 0.0f;
    if (g.x0 + kSW < W && g.lane <= g.y1 - g.y0) {
        const int y = clampi_s(g.y0 + g.lane, 0, H - 1), xe = g.x0 + kSW;
        const float* r = a.J + (int64_t)y * a.pin;
        const float* rn = a.J + (int64_t)(y > 0 ? y - 1 : 0) * a.pin;
        const float* rs = a.J + (int64_t)(y + 1 < H ? y + 1 : H - 1) * a.pin;
        ce = srad_c(r[xe], rn[xe], rs[xe], r[xe - 1], r[xe + 1 < W ? xe + 1 : W - 1], q0, K,
                    lo);
    }
    Row j0{}, j1{}, j2{}, j3{};
    float c1[4] = {}, c2[4] = {}, c1e = 0.0f, c2e = 0.0f;
    auto load = [&](int t) { return load_row<FULL>(a.J, a.pin, g.y0 - 1 + t, g); };
    auto push = [&](const Raw& in, int t) {
        j3 = j2;
        j2 = j1;
        j1 = j0;
        j0 = with_nb(in);
        if (t >= 2) {
#pragma unroll
            for (int k = 0; k < 4; ++k) c2[k] = c1[k];
            c2e = c1e;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                c1[k] = srad_c(j1.v[k], j2.v[k], j0.v[k], west_of(j1, k), east_of(j1, k), q0,
                               K, lo);
            const float cx =
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ce), t - 2));
            c1e = from_east(cx, c1[0]);
        }
    };
    sweep_rows<3, kRing>(g.y1 - g.y0 + 3, load, push, [&](const Raw& in, int t) {
        push(in, t);
        float v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = srad_new(j2.v[k], j3.v[k], j1.v[k], west_of(j2, k), east_of(j2, k), c2[k],
                            c1[k], k < 3 ? c2[k + 1] : c2e, a.step);
        store_row<FULL>(a.out, a.pout, g.y0 + t - 3, g, v);
        accumulate<FULL>(v, g, s, s2);
    });
}

}  // namespace

template <int MODE>
__global__ __launch_bounds__(256) void k_srad_sweep(SradArgs a) {
    __shared__ double sh[2][4];
    // The wave index is uniform: readfirstlane lets the compiler keep the
    // strip, band and row addresses in scalar registers.
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    float q0 = 0.0f, K = 0.0f, lo = 1.0f;
    if constexpr (MODE == kFused || MODE == kCoeff) {
        // Level 3 of the previous sums: every workgroup folds all pairs.
        double s = 0.0, s2 = 0.0;
        for (int i = threadIdx.x; i < a.nprev; i += 256) {
            s += a.prev[2 * i];
            s2 += a.prev[2 * i + 1];
        }
        s = wave_sum_d(s);
        s2 = wave_sum_d(s2);
        if (lane == 0) {
            sh[0][wave] = s;
            sh[1][wave] = s2;
        }
        __syncthreads();
        const double S = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        const double S2 = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
        const double npix = (double)a.H * (double)a.W;
        const double mean = S / npix;
        const double var = S2 / npix - mean * mean;
        const double q = var / (mean * mean);
        if (blockIdx.x == 0 && threadIdx.x == 0 && a.q_log) a.q_log[a.it] = q;
        q0 = (float)q;
        const bool flat = !(q0 > 0.0f);
        K = flat ? 0.0f : (float)(1.0 / (q * (1.0 + q)));
        lo = flat ? 1.0f : 0.0f;
        __syncthreads();   // sh is reused below
    }
    double s = 0.0, s2 = 0.0;
    const int item = xcd_block(blockIdx.x, gridDim.x) * 4 + wave;
    if (item < a.nitems) {
        Strip g;
        g.x0 = (item % a.nstrips) * kSW;
        g.y0 = (item / a.nstrips) * kBH;
        g.y1 = g.y0 + kBH < a.H ? g.y0 + kBH : a.H;
        g.H = a.H;
        g.W = a.W;
        g.lane = lane;
        const bool inside = g.x0 + kSW <= a.W;
        if constexpr (MODE == kSums) {
            if (inside && a.vin) sweep_sums<true>(a, g, s, s2);
            else sweep_sums<false>(a, g, s, s2);
        } else if constexpr (MODE == kCoeff) {
            if (inside && a.vin && a.vout) sweep_coeff<true>(a, g, q0, K, lo);
            else sweep_coeff<false>(a, g, q0, K, lo);
        } else if constexpr (MODE == kUpdate) {
            if (inside && a.vin && a.vc && a.vout) sweep_update<true>(a, g, s, s2);
            else sweep_update<false>(a, g, s, s2);
        } else {
            if (inside && a.vin && a.vout) sweep_fused<true>(a, g, q0, K, lo, s, s2);
            else sweep_fused<false>(a, g, q0, K, lo, s, s2);
        }
    }
    if constexpr (MODE != kCoeff) {
        s = wave_sum_d(s);
        s2 = wave_sum_d(s2);
        if (lane == 0) {
            sh[0][wave] = s;
            sh[1][wave] = s2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.part[2 * blockIdx.x] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
            a.part[2 * blockIdx.x + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
        }
    }
}

int64_t srad_blocks(int64_t H, int64_t W) {
    const int64_t items = ((W + kSW - 1) / kSW) * ((H + kBH - 1) / kBH);
    return (items + 3) / 4;
}

hipError_t launch_srad(const float* J, float* Jb, int64_t pj, int64_t pb, float* cbuf,
                       int64_t pc, double* partials, double* q_log, int H, int W, int niter,
                       float lambda, bool fused, hipStream_t s) {
    const int nstrips = (W + kSW - 1) / kSW;
    const int nitems = nstrips * ((H + kBH - 1) / kBH);
    const int nblocks = (nitems + 3) / 4;
    auto aligned = [](const void* p, int64_t pitch) {
        return ((uintptr_t)p % 16 == 0) && (pitch % 4 == 0);
    };
    SradArgs a{};
    a.H = H;
    a.W = W;
    a.nstrips = nstrips;
    a.nitems = nitems;
    a.nprev = nblocks;
    a.step = 0.25f * lambda;
    a.q_log = q_log;
    a.J = J;
    a.pin = pj;
    a.vin = aligned(J, pj);
    a.part = partials;
    hipLaunchKernelGGL(k_srad_sweep<kSums>, dim3(nblocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    const float* cur = J;
    int64_t pcur = pj;
    for (int it = 0; it < niter && e == hipSuccess; ++it) {
        // Iteration it reads `cur` and the sums in half it % 2 of the
        // partials, and writes the other plane and the other half.
        float* nxt = (cur == J) ? Jb : const_cast<float*>(J);
        const int64_t pnxt = (cur == J) ? pb : pj;
        a.it = it;
        a.J = cur;
        a.pin = pcur;
        a.vin = aligned(cur, pcur);
        a.prev = partials + 2 * (int64_t)nblocks * (it % 2);
        a.part = partials + 2 * (int64_t)nblocks * ((it + 1) % 2);
        if (fused) {
            a.out = nxt;
            a.pout = pnxt;
            a.vout = aligned(nxt, pnxt);
            hipLaunchKernelGGL(k_srad_sweep<kFused>, dim3(nblocks), dim3(256), 0, s, a);
        } else {
            SradArgs ac = a;
            ac.out = cbuf;
            ac.pout = pc;
            ac.vout = aligned(cbuf, pc);
            hipLaunchKernelGGL(k_srad_sweep<kCoeff>, dim3(nblocks), dim3(256), 0, s, ac);
            SradArgs au = a;
            au.c = cbuf;
            au.pc = pc;
            au.vc = aligned(cbuf, pc);
            au.out = nxt;
            au.pout = pnxt;
            au.vout = aligned(nxt, pnxt);
            hipLaunchKernelGGL(k_srad_sweep<kUpdate>, dim3(nblocks), dim3(256), 0, s, au);
        }
        e = hipGetLastError();
        cur = nxt;
        pcur = pnxt;
    }
    return e;
}

}  // namespace hx
