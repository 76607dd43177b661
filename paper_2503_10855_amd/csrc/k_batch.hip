// k_batch.hip -- a whole batch of images of any sizes in one graph launch:
// an outer fork over images whose inner fork factors differ per image,
// flattened into two lists of work items.
//
//   reset   zeroes each image's max slot;
//   pass 1  one item = one sweep tile (one wave) of one image: STORE writes
//           the pass-1 code of its pixels, RECOMPUTE computes blur + Sobel
//           only; both fold the tile's G^2 maximum into the image's slot;
//   pass 2  one item = a run of rows (STORE: code -> mask) or one sweep tile
//           (RECOMPUTE: every stage -> mask) of one image.
// SPECULATE adds pass 0 (one item = one 8-row sampled band tile: blur +
// Sobel -> a lower bound of the max), runs every stage in pass 1 (mask
// against the bound's threshold, plus the list of pixels it set), and
// re-decides only the listed pixels in pass 2 (one item = one pass-1 tile).
// Pass 2 starts after pass 1 has finished (a kernel boundary), so every max
// is final when it is read; no workgroup ever waits for another one.  Each
// wave takes the item of its index (the host sizes each grid to its pass's
// item count; were a grid smaller, its waves would stride over the rest).
// The item lists live in the descriptor table, so the kernels read every
// size from it and a captured graph is replayed as long as the batch's
// item counts are unchanged.
#include <hip/hip_runtime.h>

#include "../../include/hx.h"
#include "sweep_impl.h"
#include "thresh_impl.h"

namespace hx {

#ifndef HX_BATCH_C
#define HX_BATCH_C 4
#endif
#ifndef HX_BATCH_TY
#define HX_BATCH_TY 64
#endif
#ifndef HX_SWEEP_WAVES
#define HX_SWEEP_WAVES 3
#endif
#ifndef HX_SWEEP_WAVES_SMALL_K
#define HX_SWEEP_WAVES_SMALL_K HX_SWEEP_WAVES
#endif
#ifndef HX_BATCH_WG_WAVES
#define HX_BATCH_WG_WAVES 1
#endif
constexpr int kBC = HX_BATCH_C;    // columns per lane of the batch sweep
constexpr int kBTY = HX_BATCH_TY;  // default rows per sweep tile
// Waves per workgroup of the pass kernels.  One: a wave slot freed by a
// finished tile takes the next item at once, where a 4-wave workgroup
// waits for room for all four; with calls in flight on several streams
// that lets one call's last partial round of tiles overlap the next call.
constexpr int kWG = HX_BATCH_WG_WAVES;
// Waves per SIMD the sweep kernels are compiled for (their register cap):
// the 7-tap blur's longer row ring needs more registers than k <= 5.
constexpr int sweep_waves(int ks) { return ks <= 5 ? HX_SWEEP_WAVES_SMALL_K : HX_SWEEP_WAVES; }

int batch_sweep_c() { return kBC; }
int batch_sweep_ty() { return kBTY; }
int batch_wg_waves() { return kWG; }

__host__ __device__ inline int p2_rows(int64_t W) {
    const int64_t r = 4096 / (W > 0 ? W : 1);
    return r < 1 ? 1 : (r > (1 << 20) ? (1 << 20) : (int)r);
}
int batch_p2_rows(int64_t W) { return p2_rows(W); }

size_t batch_table_bytes(int n, int64_t n1, int64_t n2, int64_t n0) {
    return sizeof(BatchHeader) + (size_t)n * sizeof(ImgArgs) +
           (size_t)(n1 + n2 + n0) * sizeof(BatchItem);
}

int64_t batch_sample_items(int ks, int64_t H, int64_t W) {
    const SweepGeom g{ks, kBC, kSampleRows};
    const int st = sample_stride(H);
    return g.strips(W) * ((H + st - 1) / st);
}

// The bound's threshold is scaled down by this factor so that it stays at
// or below the true max's threshold even if the square root were not
// monotone to the last ulp; it only lists a few more pixels.
constexpr float kSpecSafety = 0.99999f;

struct TableView {
    BatchHeader hdr;
    const ImgArgs* imgs;
    const BatchItem* items1;
    const BatchItem* items2;
    const BatchItem* items0;
};

__device__ __forceinline__ TableView view(const uint8_t* __restrict__ table) {
    TableView v;
    v.hdr = *reinterpret_cast<const BatchHeader*>(table);
    v.imgs = reinterpret_cast<const ImgArgs*>(table + sizeof(BatchHeader));
    v.items1 = reinterpret_cast<const BatchItem*>(v.imgs + v.hdr.n_images);
    v.items2 = v.items1 + v.hdr.n_items1;
    v.items0 = v.items2 + v.hdr.n_items2;
    return v;
}

__global__ void k_batch_reset(const uint8_t* __restrict__ table, uint32_t* slots) {
    const int n = reinterpret_cast<const BatchHeader*>(table)->n_images;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        slots[i] = 0;
}

// Index of this wave among all waves of the grid (XCD-contiguous).
__device__ __forceinline__ int global_wave() {
    return __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * kWG +
                                          (int)(threadIdx.x >> 6));
}

// SPECULATE pass 0: G^2 on the sampled bands, folded into the images'
// bounds under the current epoch.  Any pixel's G^2 is at most the image's
// max, so each then holds a lower bound of it.  The first item of each
// image also clears the image's max slot (pass 1 folds into it after this
// kernel), so SPECULATE needs no reset kernel.
template <int KS>
__global__ __launch_bounds__(64 * kWG) __attribute__((amdgpu_waves_per_eu(sweep_waves(KS))))
void k_batch_p0(const uint8_t* __restrict__ table, Taps tp) {
    using S = SweepShape<KS, kBC, SM_MAXONLY>;
    const TableView tv = view(table);
    const int nw = gridDim.x * kWG;
    const uint64_t ep = (uint64_t)*as_global(tv.hdr.epoch) << 32;
    for (int k = global_wave(); k < tv.hdr.n_items0; k += nw) {
        const BatchItem it = tv.items0[k];
        const ImgArgs a = tv.imgs[it.image];
        if (it.local == 0 && lane_id() == 0) *as_global(a.slot) = 0u;
        const int nstrips = (a.W + S::OW - 1) / S::OW;
        float gmax = 0.0f;
        sweep_tile<KS, kBC, SM_MAXONLY>(a, tp, (it.local % nstrips) * S::OW,
                                         (it.local / nstrips) * sample_stride(a.H), kSampleRows,
                                         0.0f, gmax);
        gmax = wave_max(gmax);
        if (lane_id() == 0)
            atomicMax(tv.hdr.bound + it.image,
                      (unsigned long long)(ep | __float_as_uint(gmax)));
    }
}

template <int KS, int PASS>
__device__ __forceinline__ void batch_p1_body(const uint8_t* __restrict__ table,
                                              const Taps& tp) {
    constexpr int M1 = PASS == HX_PASS_STORE       ? SM_STORE
                       : PASS == HX_PASS_SPECULATE ? SM_SPEC
                                                   : SM_MAXONLY;
    using S = SweepShape<KS, kBC, M1>;
    const TableView tv = view(table);
    const int nw = gridDim.x * kWG;
    for (int k = global_wave(); k < tv.hdr.n_items1; k += nw) {
        const BatchItem it = tv.items1[k];
        const ImgArgs a = tv.imgs[it.image];
        const int nstrips = (a.W + S::OW - 1) / S::OW;
        float gmax = 0.0f;
        float thr2 = 0.0f;
        SpecTile sp{nullptr, nullptr, 0u, 0u};
        if constexpr (PASS == HX_PASS_SPECULATE) {
            // Pass 0 finished before this kernel began, and nothing writes
            // the bounds meanwhile.  (Reading the image's slot, which the
            // other tiles keep raising, measured much slower: each read
            // waits behind this wave's own atomic on the same address.)
            const uint64_t bv = as_global(tv.hdr.bound)[it.image];
            const uint32_t lb2 = (uint32_t)(bv >> 32) == *as_global(tv.hdr.epoch)
                                     ? (uint32_t)bv : 0u;
            thr2 = thr2_from(lb2, tv.hdr.theta) * kSpecSafety;
            const int64_t base = (int64_t)a.list_base + (int64_t)it.local * a.list_cap;
            sp.code = tv.hdr.cand_code + base * kBC;
            sp.row = tv.hdr.cand_row + base;
            sp.cap = a.list_cap;
        }
        // Odd bands sweep upwards (their halo rows are then read while the
        // neighbouring bands read them too).
        const int band = it.local / nstrips;
        sweep_tile<KS, kBC, M1>(a, tp, (it.local % nstrips) * S::OW, band * a.ty, a.ty, thr2,
                                gmax, &sp, (band & 1) != 0);
        if constexpr (PASS == HX_PASS_SPECULATE)
            if (lane_id() == 0) as_global(tv.hdr.cand_n)[k] = sp.n;
        gmax = wave_max(gmax);
        if (lane_id() == 0) atomic_max_g2(a.slot, gmax);
    }
}

// The sweep kernels are capped at three waves per SIMD (at most 168
// registers): left alone, the scheduler keeps more rows in flight and
// the kernels fall to two waves per SIMD, which measured slower.
template <int KS, int PASS>
__global__ __launch_bounds__(64 * kWG) __attribute__((amdgpu_waves_per_eu(sweep_waves(KS))))
void k_batch_p1(const uint8_t* __restrict__ table, Taps tp) {
    batch_p1_body<KS, PASS>(table, tp);
}

template <int KS>
__global__ __launch_bounds__(64 * kWG) __attribute__((amdgpu_waves_per_eu(sweep_waves(KS))))
void k_batch_p1s(const uint8_t* __restrict__ table, Taps tp) {
    batch_p1_body<KS, HX_PASS_SPECULATE>(table, tp);
}

// Pass 2's mask-only sweep (RECOMPUTE, SPECULATE overflow) keeps the
// three-wave cap at every k: at four it spills.
template <int KS, int PASS>
__global__ __launch_bounds__(64 * kWG) __attribute__((amdgpu_waves_per_eu(HX_SWEEP_WAVES)))
void k_batch_p2(const uint8_t* __restrict__ table, Taps tp) {
    using S = SweepShape<KS, kBC, SM_MASK>;
    const TableView tv = view(table);
    const int nw = gridDim.x * kWG;
    const int lane = lane_id();
    for (int k = global_wave(); k < tv.hdr.n_items2; k += nw) {
        const BatchItem it = tv.items2[k];
        const ImgArgs a = tv.imgs[it.image];
        // SPECULATE: the tile's entry count, loaded beside the max.
        int n_listed = 0;
        if constexpr (PASS == HX_PASS_SPECULATE) n_listed = (int)as_global(tv.hdr.cand_n)[k];
        const uint32_t m2 = *as_global(a.slot);
        const float thr2 = thr2_from(m2, tv.hdr.theta);
        if (it.local == 0 && lane == 0 && a.dmax) *as_global(a.dmax) = max_from(m2);
        if constexpr (PASS == HX_PASS_STORE) {
            const int rb = p2_rows(a.W);
            const int r0 = it.local * rb;
            const int r1 = min(a.H, r0 + rb);
            const int wq = (a.W + 3) / 4;
            const bool mvec = ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) &
                              ((a.mp % 4) == 0);
            for (int y = r0; y < r1; ++y)
                for (int q = lane; q < wq; q += 64) threshold4(a, y, q * 4, thr2, mvec);
        } else if constexpr (PASS == HX_PASS_SPECULATE) {
            // Re-decide the pixels pass 1 listed for this tile, now that
            // the max is final.
            const int nstrips = (a.W + S::OW - 1) / S::OW;
            const int x0 = (it.local % nstrips) * S::OW;
            const int y0 = (it.local / nstrips) * a.ty;
            const int n = n_listed;
            // The last reader of this batch's bounds has finished: advance
            // the epoch for the next batch on this context.
            if (k == 0 && lane == 0) *as_global(tv.hdr.epoch) += 1u;
            if ((uint32_t)n > a.list_cap) {
                // The tile set more pixels than its share of the listing
                // holds (its list is incomplete): redo the whole tile's mask
                // against the true threshold.
                float unused = 0.0f;
                sweep_tile<KS, kBC, SM_MASK>(a, tp, x0, y0, a.ty, thr2, unused);
                continue;
            }
            const bool mvec = ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) &
                              ((a.mp % 4) == 0);
            const int64_t base = (int64_t)a.list_base + (int64_t)it.local * a.list_cap;
            for (int t = lane; t < n; t += 64) {
                const int64_t idx = base + t;
                const gptr<const VecF<kBC>> q =
                    (gptr<const VecF<kBC>>)(as_global(tv.hdr.cand_code) + idx * kBC);
                const uint32_t rw = (uint32_t)as_global(tv.hdr.cand_row)[idx];
                const int y = y0 + (int)(rw >> 10);
                const int cbase = x0 - S::HL + kBC * (int)((rw >> 4) & 63u);
                const gptr<uint8_t> rp = as_global(a.mask) + (int64_t)y * a.mp + cbase;
                // Pass 1 set every listed pixel to 1 and left the others of
                // the lane-row at 0.  Only a listed pixel at or below the
                // true threshold changes (to 0): the lane-row is rewritten,
                // as one aligned word when it lies inside the image, only
                // if one did.  Those are few when the bound is close to the
                // max, and scattered partial writes are what this pass
                // spends its time on.
                // Both loads are unconditional, so they are in flight
                // together (a short-circuit test would load each value
                // behind its own wait).
                float g2v[kBC];
#pragma unroll
                for (int e = 0; e < kBC; ++e) g2v[e] = q->v[e];
                uint32_t w = 0, was = 0;
#pragma unroll
                for (int e = 0; e < kBC; ++e) {
                    const uint32_t listed = (rw >> e) & 1u;
                    was |= listed << (8 * e);
                    w |= (listed & (uint32_t)(g2v[e] > thr2)) << (8 * e);
                }
                if (w != was) {
                    if (kBC == 4 && mvec && cbase + 4 <= a.W) {
                        *(gptr<uint32_t>)rp = w;
                    } else {
#pragma unroll
                        for (int e = 0; e < kBC; ++e)
                            if (((was ^ w) >> (8 * e)) & 1u) rp[e] = 0;
                    }
                }
            }
        } else {
            const int nstrips = (a.W + S::OW - 1) / S::OW;
            float unused = 0.0f;
            const int band = it.local / nstrips;
            sweep_tile<KS, kBC, SM_MASK>(a, tp, (it.local % nstrips) * S::OW, band * a.ty, a.ty,
                                         thr2, unused, nullptr, (band & 1) != 0);
        }
    }
}

hipError_t launch_batch_reset(const void* d_table, uint32_t* slots, int max_images,
                              hipStream_t s) {
    int grid = (max_images + 255) / 256;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_batch_reset, dim3(grid), dim3(256), 0, s,
                       (const uint8_t*)d_table, slots);
    return hipGetLastError();
}

static const void* batch_kernel_ptr(int ks, int pass, int phase) {
#define HX_B(K)                                                                      \
    if (ks == K) {                                                                   \
        if (phase == 0)                                                              \
            return pass == HX_PASS_SPECULATE ? (const void*)k_batch_p0<K> : nullptr; \
        if (pass == HX_PASS_STORE)                                                   \
            return phase == 1 ? (const void*)k_batch_p1<K, HX_PASS_STORE>            \
                              : (const void*)k_batch_p2<K, HX_PASS_STORE>;           \
        if (pass == HX_PASS_RECOMPUTE)                                               \
            return phase == 1 ? (const void*)k_batch_p1<K, HX_PASS_RECOMPUTE>        \
                              : (const void*)k_batch_p2<K, HX_PASS_RECOMPUTE>;       \
        if (pass == HX_PASS_SPECULATE)                                               \
            return phase == 1 ? (const void*)k_batch_p1s<K>                          \
                              : (const void*)k_batch_p2<K, HX_PASS_SPECULATE>;       \
    }
    HX_B(3) HX_B(5) HX_B(7)
#undef HX_B
    return nullptr;
}


hipError_t launch_batch_phase(int ks, int pass_mode, int phase, const void* d_table,
                              const Taps& t, int grid, hipStream_t s) {
    const void* k = batch_kernel_ptr(ks, pass_mode, phase);
    if (!k || grid < 1) return hipErrorInvalidValue;
    const uint8_t* tab = (const uint8_t*)d_table;
    Taps tc = t;
    void* args[] = {(void*)&tab, (void*)&tc};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * kWG), args, 0, s);
}

}  // namespace hx
