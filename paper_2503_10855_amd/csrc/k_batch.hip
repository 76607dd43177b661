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
// Pass 2 starts after pass 1 has finished (a kernel boundary), so every max
// is final when it is read; no workgroup ever waits for another one.  Each
// persistent wave strides over its pass's item list; the item lists live in
// the descriptor table, so one captured graph serves every batch
// composition.
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
constexpr int kBC = HX_BATCH_C;    // columns per lane of the batch sweep
constexpr int kBTY = HX_BATCH_TY;  // rows per sweep tile

int batch_sweep_c() { return kBC; }
int batch_sweep_ty() { return kBTY; }

__host__ __device__ inline int p2_rows(int64_t W) {
    const int64_t r = 4096 / (W > 0 ? W : 1);
    return r < 1 ? 1 : (r > (1 << 20) ? (1 << 20) : (int)r);
}
int batch_p2_rows(int64_t W) { return p2_rows(W); }

size_t batch_table_bytes(int n, int64_t n1, int64_t n2) {
    return sizeof(BatchHeader) + (size_t)n * sizeof(ImgArgs) +
           (size_t)(n1 + n2) * sizeof(BatchItem);
}

struct TableView {
    BatchHeader hdr;
    const ImgArgs* imgs;
    const BatchItem* items1;
    const BatchItem* items2;
};

__device__ __forceinline__ TableView view(const uint8_t* __restrict__ table) {
    TableView v;
    v.hdr = *reinterpret_cast<const BatchHeader*>(table);
    v.imgs = reinterpret_cast<const ImgArgs*>(table + sizeof(BatchHeader));
    v.items1 = reinterpret_cast<const BatchItem*>(v.imgs + v.hdr.n_images);
    v.items2 = v.items1 + v.hdr.n_items1;
    return v;
}

__global__ void k_batch_reset(const uint8_t* __restrict__ table, uint32_t* slots) {
    const int n = reinterpret_cast<const BatchHeader*>(table)->n_images;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        slots[i] = 0;
}

// Index of this wave among all waves of the grid (XCD-contiguous).
__device__ __forceinline__ int global_wave() {
    return __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 +
                                          (int)(threadIdx.x >> 6));
}

template <int KS, int PASS>
__global__ __launch_bounds__(256) void k_batch_p1(const uint8_t* __restrict__ table,
                                                  Taps tp) {
    constexpr int M1 = PASS == HX_PASS_STORE ? SM_STORE : SM_MAXONLY;
    using S = SweepShape<KS, kBC, kBTY, M1>;
    const TableView tv = view(table);
    const int nw = gridDim.x * 4;
    for (int k = global_wave(); k < tv.hdr.n_items1; k += nw) {
        const BatchItem it = tv.items1[k];
        const ImgArgs a = tv.imgs[it.image];
        const int nstrips = (a.W + S::OW - 1) / S::OW;
        float gmax = 0.0f;
        sweep_tile<KS, kBC, kBTY, M1>(a, tp, (it.local % nstrips) * S::OW,
                                      (it.local / nstrips) * kBTY, 0.0f, gmax);
        gmax = wave_max(gmax);
        if (lane_id() == 0) atomic_max_g2(a.slot, gmax);
    }
}

template <int KS, int PASS>
__global__ __launch_bounds__(256) void k_batch_p2(const uint8_t* __restrict__ table,
                                                  Taps tp) {
    using S = SweepShape<KS, kBC, kBTY, SM_MASK>;
    const TableView tv = view(table);
    const int nw = gridDim.x * 4;
    const int lane = lane_id();
    for (int k = global_wave(); k < tv.hdr.n_items2; k += nw) {
        const BatchItem it = tv.items2[k];
        const ImgArgs a = tv.imgs[it.image];
        const uint32_t m2 = *a.slot;
        const float thr2 = thr2_from(m2, tv.hdr.theta);
        if (it.local == 0 && lane == 0 && a.dmax) *a.dmax = max_from(m2);
        if constexpr (PASS == HX_PASS_STORE) {
            const int rb = p2_rows(a.W);
            const int r0 = it.local * rb;
            const int r1 = min(a.H, r0 + rb);
            const int wq = (a.W + 3) / 4;
            const bool mvec = ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) &
                              ((a.mp % 4) == 0);
            for (int y = r0; y < r1; ++y)
                for (int q = lane; q < wq; q += 64) threshold4(a, y, q * 4, thr2, mvec);
        } else {
            const int nstrips = (a.W + S::OW - 1) / S::OW;
            float unused = 0.0f;
            sweep_tile<KS, kBC, kBTY, SM_MASK>(a, tp, (it.local % nstrips) * S::OW,
                                               (it.local / nstrips) * kBTY, thr2, unused);
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
#define HX_B(K)                                                                        \
    if (ks == K) {                                                                     \
        if (phase == 1)                                                                \
            return pass == HX_PASS_STORE ? (const void*)k_batch_p1<K, HX_PASS_STORE>      \
                                         : (const void*)k_batch_p1<K, HX_PASS_RECOMPUTE>; \
        return pass == HX_PASS_STORE ? (const void*)k_batch_p2<K, HX_PASS_STORE>          \
                                     : (const void*)k_batch_p2<K, HX_PASS_RECOMPUTE>;      \
    }
    HX_B(3) HX_B(5) HX_B(7)
#undef HX_B
    return nullptr;
}

int batch_grid_size(int device, int ks, int pass_mode, int phase) {
    const void* k = batch_kernel_ptr(ks, pass_mode, phase);
    if (!k) return 0;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_batch_phase(int ks, int pass_mode, int phase, const void* d_table,
                              const Taps& t, int grid, hipStream_t s) {
    const void* k = batch_kernel_ptr(ks, pass_mode, phase);
    if (!k || grid < 1) return hipErrorInvalidValue;
    const uint8_t* tab = (const uint8_t*)d_table;
    Taps tc = t;
    void* args[] = {(void*)&tab, (void*)&tc};
    return hipLaunchKernel(k, dim3(grid), dim3(256), args, 0, s);
}

}  // namespace hx
