// hx_device.h -- per-pixel arithmetic of the EDGE stages, shared by every
// kernel variant (depth-1 stage kernels, register sweeps, the persistent
// batch kernel).  Each output value is produced by exactly one fixed
// sequence of fp32 operations defined here, so every schedule yields
// bit-identical B, L, G^2, Z, max and mask.  Code is compiled with
// -ffp-contract=off: the only fused multiply-adds are the explicit fmaf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hx {

constexpr int kMaxK = 15;

// 1-D Gaussian taps, rounded to fp32 from the fp64 normalised weights.
struct Taps {
    float g[kMaxK];
};

// Horizontal or vertical pass of the separable blur over k samples
// v[0..k-1] (v[r] is the centre, r = k/2; the taps are symmetric): the
// centre's product, then for i = 1..r the pair v[r-i] + v[r+i] times its
// tap, added in that order by fma.  Each output costs k operations, and a
// sample from a neighbouring lane only ever enters an addition.
template <int K>
__device__ __forceinline__ float blur_pair(const float* v, int i) {
    return v[K / 2 - i] + v[K / 2 + i];
}
template <int K>
__device__ __forceinline__ float blur_from_pairs(float centre, const float* pair,
                                                 const Taps& t) {
    constexpr int R = K / 2;
    float acc = t.g[R] * centre;
#pragma unroll
    for (int i = 1; i <= R; ++i) acc = fmaf(t.g[R + i], pair[i - 1], acc);
    return acc;
}
template <int K>
__device__ __forceinline__ float blur_chain(const float* v, const Taps& t) {
    float pair[K / 2 > 0 ? K / 2 : 1];
#pragma unroll
    for (int i = 1; i <= K / 2; ++i) pair[i - 1] = blur_pair<K>(v, i);
    return blur_from_pairs<K>(v[K / 2], pair, t);
}

// Pairwise sums that both the Laplacian and the Sobel stage reuse.
//   ew = B(x-1) + B(x+1)                      (same row)
//   ns = B(y-1) + B(y+1)                      (same column)
__device__ __forceinline__ float lap_from(float ns, float ew, float c) {
    // ((n + s) + (e + w)) - 4c; 4c is exact, so one rounding of the sum.
    return fmaf(-4.0f, c, ns + ew);
}

// Sobel as two smoothings and two differences:
//   sy = ew + 2 B(x)          along a row (ew = B(x-1) + B(x+1)),
//   vs = ns + 2 B(y)          down a column (ns = B(y-1) + B(y+1)),
//   gx = vs(x+1) - vs(x-1),   gy = sy(y+1) - sy(y-1),
//   G^2 = gx^2 + gy^2 (the sweep never takes the square root).
// The sums ew and ns are the Laplacian's, so each is formed once.
__device__ __forceinline__ float sobel_sy(float ew, float c) {
    return fmaf(2.0f, c, ew);
}
__device__ __forceinline__ float sobel_vs(float ns, float c) {
    return fmaf(2.0f, c, ns);
}
__device__ __forceinline__ float sobel_g2(float vsl, float vsr, float syu, float syd) {
    const float gx = vsr - vsl;
    const float gy = syd - syu;
    return fmaf(gx, gx, gy * gy);
}

// Zero crossing from the 3x3 max and min of L: the window holds a value
// > 0 and a value <= 0.  Exact (no rounding), so its order is free.
__device__ __forceinline__ bool zero_cross(float lmax, float lmin) {
    return (lmax > 0.0f) & !(lmin > 0.0f);
}

// Pass-1 store code: G^2 where Z = 1, else -1 (never above a threshold).
__device__ __forceinline__ float pass1_code(bool z, float g2) {
    return z ? g2 : -1.0f;
}

// Threshold on G^2: tau = theta * sqrt(M2), compare G^2 > tau^2.
__device__ __forceinline__ float thr2_from(uint32_t m2bits, float theta) {
    float m = __builtin_sqrtf(__uint_as_float(m2bits));
    float tau = theta * m;
    return tau * tau;
}
__device__ __forceinline__ float max_from(uint32_t m2bits) {
    return __builtin_sqrtf(__uint_as_float(m2bits));
}

// G^2 >= +0 always, so its IEEE bits order like unsigned integers and a
// device-scope integer atomic max is an exact float max.
__device__ __forceinline__ void atomic_max_g2(uint32_t* slot, float g2) {
    atomicMax(slot, __float_as_uint(g2));
}

// Pointers read from a descriptor table are generic to the compiler;
// casting them to the global address space lets it emit global (not flat)
// loads and stores with a scalar base address.
template <class T>
using gptr = T __attribute__((address_space(1)))*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
    return (gptr<T>)p;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Max over the 64 lanes of a wave (xor butterfly); every lane gets it.
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Map a workgroup index so that each of the 8 XCDs (which receive
// workgroups round-robin) walks a contiguous range of tiles: neighbouring
// tiles then share halo rows through the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    const int per = nblocks / 8, rem = nblocks % 8;
    const int xcd = bid % 8, loc = bid / 8;
    return xcd < rem ? xcd * (per + 1) + loc
                     : rem * (per + 1) + (xcd - rem) * per + loc;
}

}  // namespace hx
