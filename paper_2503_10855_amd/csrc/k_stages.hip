// k_stages.hip -- the unfused (fusion depth 1) stage kernels, the second
// kernels of fusion depths 2 and 3, the threshold kernels and small
// helpers.  One kernel per fork over pixels, in the form the paper's EDGE
// schedule used (no fusion; Use and Impact of Schedules, transform table).
// Per-pixel arithmetic comes from hx_device.h, identical to the sweeps.
#include <hip/hip_runtime.h>

#include "../../include/hx.h"
#include "hx_kernels.h"
#include "thresh_impl.h"

namespace hx {

namespace {

// Pixel tile of a 256-thread workgroup: TW x TH pixels, thread (tx, ty0)
// handles column tx of rows ty0, ty0 + 256/TW, ...
struct TileMap {
    int tw, th;
    int tiles_x, tiles_y;
};

__device__ __forceinline__ bool tile_px(const TileMap& m, int k, int W, int H,
                                        int& x, int& y) {
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = bid % m.tiles_x, by = bid / m.tiles_x;
    const int rows_per = 256 / m.tw;
    x = bx * m.tw + (int)(threadIdx.x % m.tw);
    y = by * m.th + (int)(threadIdx.x / m.tw) + k * rows_per;
    return (x < W) & (y < H) & ((int)(threadIdx.x / m.tw) + k * rows_per < m.th);
}

__device__ __forceinline__ int reps(const TileMap& m) {
    const int rows_per = 256 / m.tw;
    return (m.th + rows_per - 1) / rows_per;
}

// B of each pixel from its clamped KS x KS window: the horizontal chain of
// each window row, then the vertical chain of the results (the sweeps'
// order, so the same bits).  KS is a template argument so the window lives
// in registers.
template <int KS>
__global__ __launch_bounds__(256) void k_blur(ImgArgs a, StageBufs b, Taps t, TileMap m) {
    constexpr int r = KS / 2;
    for (int k = 0; k < reps(m); ++k) {
        int x, y;
        if (!tile_px(m, k, a.W, a.H, x, y)) continue;
        int xs[KS];
#pragma unroll
        for (int j = 0; j < KS; ++j) xs[j] = clampi(x - r + j, 0, a.W - 1);
        float col[KS];
#pragma unroll
        for (int i = 0; i < KS; ++i) {
            const float* rp = a.src + (int64_t)clampi(y - r + i, 0, a.H - 1) * a.sp;
            float row[KS];
#pragma unroll
            for (int j = 0; j < KS; ++j) row[j] = rp[xs[j]];
            col[i] = blur_chain<KS>(row, t);
        }
        b.B[(int64_t)y * b.op + x] = blur_chain<KS>(col, t);
    }
}

__device__ __forceinline__ float at(const float* X, int64_t op, int y, int x,
                                    int H, int W) {
    return X[(int64_t)clampi(y, 0, H - 1) * op + clampi(x, 0, W - 1)];
}

__device__ __forceinline__ float lap_at(const float* B, int64_t op, int y,
                                        int x, int H, int W) {
    const float ns = at(B, op, y - 1, x, H, W) + at(B, op, y + 1, x, H, W);
    const float ew = at(B, op, y, x - 1, H, W) + at(B, op, y, x + 1, H, W);
    return lap_from(ns, ew, at(B, op, y, x, H, W));
}

__global__ __launch_bounds__(256) void k_laplacian(ImgArgs a, StageBufs b,
                                                  TileMap m) {
    for (int k = 0; k < reps(m); ++k) {
        int x, y;
        if (!tile_px(m, k, a.W, a.H, x, y)) continue;
        b.L[(int64_t)y * b.op + x] = lap_at(b.B, b.op, y, x, a.H, a.W);
    }
}

__global__ __launch_bounds__(256) void k_zero_cross(ImgArgs a, StageBufs b,
                                                   const float* L, TileMap m) {
    for (int k = 0; k < reps(m); ++k) {
        int x, y;
        if (!tile_px(m, k, a.W, a.H, x, y)) continue;
        float mx = -__builtin_inff(), mn = __builtin_inff();
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const float v = at(L, b.op, y + dy, x + dx, a.H, a.W);
                mx = __builtin_fmaxf(mx, v);
                mn = __builtin_fminf(mn, v);
            }
        b.Z[(int64_t)y * b.op + x] = zero_cross(mx, mn) ? 1 : 0;
    }
}

// Depth 2's second kernel for 64 x 16 output tiles: B of the tile and a
// 2-pixel halo is staged in LDS once, L of the tile and a 1-pixel halo is
// computed into LDS once per pixel, and Z reads its 3 x 3 window from LDS
// (instead of 9 Laplacians of 5 global loads each per pixel).  Every LDS
// cell holds the stage's value at the clamped image position, so the same
// operands reach lap_from and zero_cross as in the depth-1 Laplacian and
// zero-crossing kernels: the same bits.
constexpr int kLzW = 64, kLzH = 16;
__global__ __launch_bounds__(256) void k_lap_zero_cross_lds(ImgArgs a, StageBufs b,
                                                           TileMap m) {
    constexpr int BW = kLzW + 4, BH = kLzH + 4, LW = kLzW + 2, LH = kLzH + 2;
    __shared__ float sB[BH][BW];
    __shared__ float sL[LH][LW];
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (bid % m.tiles_x) * kLzW, y0 = (bid / m.tiles_x) * kLzH;
    const int H = a.H, W = a.W;
    // B at clamped (y0 - 2 + r, x0 - 2 + c).
    for (int i = threadIdx.x; i < BH * BW; i += 256) {
        const int r = i / BW, c = i - r * BW;
        sB[r][c] = b.B[(int64_t)clampi(y0 - 2 + r, 0, H - 1) * b.op + clampi(x0 - 2 + c, 0, W - 1)];
    }
    __syncthreads();
    // L at clamped (y0 - 1 + r, x0 - 1 + c); its B neighbours at clamped
    // positions, found in sB at (image row - (y0 - 2), image col - (x0 - 2)).
    for (int i = threadIdx.x; i < LH * LW; i += 256) {
        const int r = i / LW, c = i - r * LW;
        const int y = clampi(y0 - 1 + r, 0, H - 1), x = clampi(x0 - 1 + c, 0, W - 1);
        const int ry = y - (y0 - 2), rx = x - (x0 - 2);
        const int rn = clampi(y - 1, 0, H - 1) - (y0 - 2), rs = clampi(y + 1, 0, H - 1) - (y0 - 2);
        const int cw = clampi(x - 1, 0, W - 1) - (x0 - 2), ce = clampi(x + 1, 0, W - 1) - (x0 - 2);
        const float ns = sB[rn][rx] + sB[rs][rx];
        const float ew = sB[ry][cw] + sB[ry][ce];
        sL[r][c] = lap_from(ns, ew, sB[ry][rx]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLzH * kLzW; i += 256) {
        const int ly = i / kLzW, lx = i - ly * kLzW;
        const int y = y0 + ly, x = x0 + lx;
        if (y >= H || x >= W) continue;
        float mx = -__builtin_inff(), mn = __builtin_inff();
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const float v = sL[clampi(y + dy, 0, H - 1) - (y0 - 1)]
                                  [clampi(x + dx, 0, W - 1) - (x0 - 1)];
                mx = __builtin_fmaxf(mx, v);
                mn = __builtin_fminf(mn, v);
            }
        b.Z[(int64_t)y * b.op + x] = zero_cross(mx, mn) ? 1 : 0;
    }
}

__device__ __forceinline__ float g2_at(const float* B, int64_t op, int y,
                                       int x, int H, int W) {
    // sy on the rows above and below, vs on the columns left and right, each
    // from B at clamped positions.
    float sy[2], vs[2];
    for (int d = 0; d < 2; ++d) {
        const int yy = y - 1 + 2 * d, xx = x - 1 + 2 * d;
        sy[d] = sobel_sy(at(B, op, yy, x - 1, H, W) + at(B, op, yy, x + 1, H, W),
                         at(B, op, yy, x, H, W));
        vs[d] = sobel_vs(at(B, op, y - 1, xx, H, W) + at(B, op, y + 1, xx, H, W),
                         at(B, op, y, xx, H, W));
    }
    return sobel_g2(vs[0], vs[1], sy[0], sy[1]);
}

// reduce: HX_REDUCE_TREE folds the max in here (wave shuffle + atomic);
// the other modes reduce the stored G^2 plane afterwards.
__global__ __launch_bounds__(256) void k_sobel(ImgArgs a, StageBufs b,
                                              TileMap m, int reduce) {
    float mx = 0.0f;
    for (int k = 0; k < reps(m); ++k) {
        int x, y;
        if (!tile_px(m, k, a.W, a.H, x, y)) continue;
        const float g2 = g2_at(b.B, b.op, y, x, a.H, a.W);
        b.G2[(int64_t)y * b.op + x] = g2;
        mx = __builtin_fmaxf(mx, g2);
    }
    if (reduce == HX_REDUCE_TREE) {
        // Wave maxima by shuffles, the workgroup's 4 through LDS, one
        // device-scope atomic per workgroup (every atomic of the kernel
        // lands on the image's one slot, so fewer is faster).
        __shared__ float wm[4];
        mx = wave_max(mx);
        if (lane_id() == 0) wm[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0)
            atomic_max_g2(a.slot, __builtin_fmaxf(__builtin_fmaxf(wm[0], wm[1]),
                                                  __builtin_fmaxf(wm[2], wm[3])));
    }
}

// First level of the TWO_LEVEL tree (the reduction_tree schedule: chunk the
// reduction over kTreeThreads threads, each starting from the identity):
// thread t folds the G^2 values t, t + N, t + 2N, ... of the plane, in
// order, into partial[t].
__global__ __launch_bounds__(256) void k_chunk_max(ImgArgs a, const float* G2, int64_t op,
                                                  float* partial) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)a.H * op;
    float mx = 0.0f;
    for (int64_t i = t; i < n; i += kTreeThreads)
        if (i % op < a.W) mx = __builtin_fmaxf(mx, G2[i]);
    partial[t] = mx;
}

// Second level: one thread combines the partials in order (the fission of
// the chunked loop into a parallel and a serial fork).
__global__ void k_combine_partials(ImgArgs a, const float* partial, int64_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float mx = 0.0f;
    for (int64_t i = 0; i < n; ++i) mx = __builtin_fmaxf(mx, partial[i]);
    *a.slot = __float_as_uint(mx);
}

// SEQUENTIAL: one thread scans every G^2 value (no reduction tree).
__global__ void k_sequential_max(ImgArgs a, const float* G2, int64_t op) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float mx = 0.0f;
    for (int y = 0; y < a.H; ++y)
        for (int x = 0; x < a.W; ++x) mx = __builtin_fmaxf(mx, G2[(int64_t)y * op + x]);
    *a.slot = __float_as_uint(mx);
}

__global__ __launch_bounds__(256) void k_threshold_zg(ImgArgs a, StageBufs b,
                                                     float theta, TileMap m) {
    const uint32_t m2 = *a.slot;
    const float thr2 = thr2_from(m2, theta);
    if (a.dmax && blockIdx.x == 0 && threadIdx.x == 0) *a.dmax = max_from(m2);
    for (int k = 0; k < reps(m); ++k) {
        int x, y;
        if (!tile_px(m, k, a.W, a.H, x, y)) continue;
        const int64_t i = (int64_t)y * b.op + x;
        a.mask[(int64_t)y * a.mp + x] = (b.Z[i] && (b.G2[i] > thr2)) ? 1 : 0;
    }
}

// Pass 2 of STORE on one image: code -> mask, 4 pixels per thread.
__global__ __launch_bounds__(256) void k_threshold_code(ImgArgs a, float theta,
                                                        uint32_t* zero_next) {
    const uint32_t m2 = *a.slot;
    const float thr2 = thr2_from(m2, theta);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (a.dmax) *a.dmax = max_from(m2);
        if (zero_next) *zero_next = 0u;  // the next per-image call's max slot
    }
    const int wq = (a.W + 3) / 4;
    const bool mvec = ((reinterpret_cast<uintptr_t>(a.mask) % 4) == 0) & ((a.mp % 4) == 0);
    const int64_t total = (int64_t)wq * a.H;
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * 256) {
        const int y = (int)(g / wq);
        const int x = (int)(g - (int64_t)y * wq) * 4;
        threshold4(a, y, x, thr2, mvec);
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_write_max(ImgArgs a) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && a.dmax) *a.dmax = max_from(*a.slot);
}

__global__ __launch_bounds__(256) void k_export(ImgArgs a, StageBufs b,
                                               float* dB, float* dL,
                                               uint8_t* dZ, float* dG) {
    const int64_t n = (int64_t)a.H * a.W;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256) {
        const int y = (int)(i / a.W), x = (int)(i - (int64_t)y * a.W);
        const int64_t j = (int64_t)y * b.op + x;
        if (dB) dB[i] = b.B[j];
        if (dL) dL[i] = b.L[j];
        if (dZ) dZ[i] = b.Z[j];
        if (dG) dG[i] = __builtin_sqrtf(b.G2[j]);
    }
}

TileMap make_map(const ImgArgs& a, int tw, int th) {
    TileMap m;
    m.tw = tw;
    m.th = th;
    m.tiles_x = (a.W + tw - 1) / tw;
    m.tiles_y = (a.H + th - 1) / th;
    return m;
}

int grid_of(const TileMap& m) { return m.tiles_x * m.tiles_y; }

int stream_grid(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3(stream_grid(n, 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_blur(const ImgArgs& a, const StageBufs& b, const Taps& t,
                       int ks, int tw, int th, hipStream_t s) {
    const TileMap m = make_map(a, tw, th);
    const dim3 g(grid_of(m)), blk(256);
    switch (ks) {
        case 1: hipLaunchKernelGGL(k_blur<1>, g, blk, 0, s, a, b, t, m); break;
        case 3: hipLaunchKernelGGL(k_blur<3>, g, blk, 0, s, a, b, t, m); break;
        case 5: hipLaunchKernelGGL(k_blur<5>, g, blk, 0, s, a, b, t, m); break;
        case 7: hipLaunchKernelGGL(k_blur<7>, g, blk, 0, s, a, b, t, m); break;
        case 9: hipLaunchKernelGGL(k_blur<9>, g, blk, 0, s, a, b, t, m); break;
        case 11: hipLaunchKernelGGL(k_blur<11>, g, blk, 0, s, a, b, t, m); break;
        case 13: hipLaunchKernelGGL(k_blur<13>, g, blk, 0, s, a, b, t, m); break;
        case 15: hipLaunchKernelGGL(k_blur<15>, g, blk, 0, s, a, b, t, m); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_laplacian(const ImgArgs& a, const StageBufs& b, int tw,
                            int th, hipStream_t s) {
    const TileMap m = make_map(a, tw, th);
    hipLaunchKernelGGL(k_laplacian, dim3(grid_of(m)), dim3(256), 0, s, a, b, m);
    return hipGetLastError();
}

hipError_t launch_zero_cross(const ImgArgs& a, const StageBufs& b,
                             const float* Lsrc, int tw, int th, hipStream_t s) {
    const TileMap m = make_map(a, tw, th);
    hipLaunchKernelGGL(k_zero_cross, dim3(grid_of(m)), dim3(256), 0, s, a, b, Lsrc, m);
    return hipGetLastError();
}

hipError_t launch_lap_zero_cross(const ImgArgs& a, const StageBufs& b, int tw,
                                 int th, hipStream_t s) {
    if (tw != kLzW || th != kLzH) return hipErrorInvalidValue;  // its one tile shape
    const TileMap m = make_map(a, tw, th);
    hipLaunchKernelGGL(k_lap_zero_cross_lds, dim3(grid_of(m)), dim3(256), 0, s, a, b, m);
    return hipGetLastError();
}

hipError_t launch_sobel_max(const ImgArgs& a, const StageBufs& b, int tw,
                            int th, int reduce_mode, hipStream_t s) {
    const TileMap m = make_map(a, tw, th);
    hipLaunchKernelGGL(k_sobel, dim3(grid_of(m)), dim3(256), 0, s, a, b, m, reduce_mode);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (reduce_mode == HX_REDUCE_TWO_LEVEL) {
        hipLaunchKernelGGL(k_chunk_max, dim3(kTreeThreads / 256), dim3(256), 0, s, a,
                           (const float*)b.G2, b.op, b.partial);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_combine_partials, dim3(1), dim3(64), 0, s, a,
                           (const float*)b.partial, (int64_t)kTreeThreads);
        e = hipGetLastError();
    } else if (reduce_mode == HX_REDUCE_SEQUENTIAL) {
        hipLaunchKernelGGL(k_sequential_max, dim3(1), dim3(64), 0, s, a,
                           (const float*)b.G2, b.op);
        e = hipGetLastError();
    }
    return e;
}

hipError_t launch_threshold_zg(const ImgArgs& a, const StageBufs& b,
                               float theta, int tw, int th, hipStream_t s) {
    const TileMap m = make_map(a, tw, th);
    hipLaunchKernelGGL(k_threshold_zg, dim3(grid_of(m)), dim3(256), 0, s, a, b, theta, m);
    return hipGetLastError();
}

hipError_t launch_threshold_code(const ImgArgs& a, float theta, hipStream_t s,
                                 uint32_t* zero_next) {
    const int64_t work = (int64_t)((a.W + 3) / 4) * a.H;
    hipLaunchKernelGGL(k_threshold_code, dim3(stream_grid(work, 256 * 4)), dim3(256), 0, s,
                       a, theta, zero_next);
    return hipGetLastError();
}

hipError_t launch_write_max(const ImgArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_write_max, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_export_stages(const ImgArgs& a, const StageBufs& b,
                                float* dB, float* dL, uint8_t* dZ, float* dG,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_export, dim3(stream_grid((int64_t)a.H * a.W, 256 * 8)), dim3(256),
                       0, s, a, b, dB, dL, dZ, dG);
    return hipGetLastError();
}

}  // namespace hx
