// hx_kernels.h -- argument blocks and launchers of the HIP kernels.
// Internal to libhx.so (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hx_device.h"

namespace hx {

// Sweep modes: which stages the register sweep computes and what it writes.
enum SweepMode : int {
    SM_STORE = 0,    // every stage -> pass-1 code (G^2 if Z else -1) + max
    SM_MAXONLY = 1,  // blur + Sobel -> max only
    SM_MASK = 2,     // every stage -> mask (reads the finished max)
    SM_BG = 3,       // blur + Sobel -> B, G^2, max
    SM_BGL = 4,      // blur + Sobel + Laplacian -> L, G^2, max
    SM_SPEC = 5,     // every stage -> mask against a lower-bound threshold,
                     // the list of pixels it set (SpecTile), and the max
};

// Where one SM_SPEC tile lists the pixels whose mask bit it set.  One
// entry per (row, lane) that set a bit, packed in row then lane order:
// code[] holds G^2 of the lane's C pixels of that row, and row[] packs
// (row offset from the tile top) << 10 | lane << 4 | a bit per column
// that was set.  n counts the tile's entries (the same in every lane).
struct SpecTile {
    float* code;     // C floats per entry
    int32_t* row;
    uint32_t n;
    uint32_t cap;    // entries the tile may write; n may exceed it
};

// One image as the kernels see it.  Pitches are in elements of the
// respective buffer.  fout: pass-1 code (STORE), B (BG) or L (BGL);
// g2: G^2 (BG, BGL).  fout/g2 rows use pitch `op`, which is a multiple of
// 4 floats with 16-byte aligned rows.
struct ImgArgs {
    const float* src;
    int64_t sp;
    uint8_t* mask;
    int64_t mp;
    float* fout;
    float* g2;
    int64_t op;
    uint32_t* slot;   // max G^2 bits of this image
    float* dmax;      // optional: receives M = sqrt(max G^2)
    int32_t H, W;
    // Batched SPECULATE: the image's pass-1 tile t lists its pixels in
    // entries [list_base + t * list_cap, list_base + (t + 1) * list_cap).
    uint32_t list_base, list_cap;
    // Batched calls: rows per sweep tile of this image (a multiple of 8).
    int32_t ty;
};

// Geometry of a register-sweep tile (one wave64): C input columns per lane,
// TY output rows; KS the blur size.
struct SweepGeom {
    int ks, c, ty;
    int halo() const { return ks / 2 + 2; }
    int hl() const { return ((halo() + c - 1) / c) * c; }
    int sw() const { return 64 * c; }
    int ow() const { return ((sw() - hl() - halo()) / c) * c; }
    int64_t strips(int64_t W) const { return (W + ow() - 1) / ow(); }
    int64_t bands(int64_t H) const { return (H + ty - 1) / ty; }
    int64_t tiles(int64_t H, int64_t W) const { return strips(W) * bands(H); }
};

// Is (ks, c, ty) one of the compiled sweep shapes?
bool sweep_supported(int ks, int c, int ty);

// ---- per-image launchers (return hipSuccess or the launch error) -------
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_sweep(int mode, int ks, int c, int ty, const ImgArgs& a,
                        const Taps& t, float theta, hipStream_t s);
// Pass 2 of STORE: code -> mask, and M into dmax.
// zero_next (nullable): a word the kernel sets to 0 (the slot of the next
// per-image call, which no wave of this kernel reads).
hipError_t launch_threshold_code(const ImgArgs& a, float theta, hipStream_t s,
                                 uint32_t* zero_next = nullptr);
// Write M into a.dmax from a.slot (one thread).
hipError_t launch_write_max(const ImgArgs& a, hipStream_t s);

// Depth-1 stage kernels (tile tw x th pixels per 256-thread workgroup).
struct StageBufs {
    float* B;        // dense-pitched H x op
    float* L;
    float* G2;
    uint8_t* Z;      // pitch op bytes
    float* partial;  // TWO_LEVEL: kTreeThreads partial maxima
    int64_t op;
};
// Threads of the first level of the TWO_LEVEL max reduction.
constexpr int kTreeThreads = 4096;
hipError_t launch_blur(const ImgArgs& a, const StageBufs& b, const Taps& t,
                       int ks, int tw, int th, hipStream_t s);
hipError_t launch_laplacian(const ImgArgs& a, const StageBufs& b, int tw,
                            int th, hipStream_t s);
hipError_t launch_zero_cross(const ImgArgs& a, const StageBufs& b,
                             const float* Lsrc, int tw, int th, hipStream_t s);
// reduce_mode: HX_REDUCE_* from hx.h.  For TWO_LEVEL and SEQUENTIAL this
// also launches the final combining kernel.
hipError_t launch_sobel_max(const ImgArgs& a, const StageBufs& b, int tw,
                            int th, int reduce_mode, hipStream_t s);
// Depth-2 second kernel: L from B, then Z (64 x 16 tiles only).
hipError_t launch_lap_zero_cross(const ImgArgs& a, const StageBufs& b, int tw,
                                 int th, hipStream_t s);
// Final threshold of depths 1-3: (Z, G^2, max) -> mask, M into dmax.
hipError_t launch_threshold_zg(const ImgArgs& a, const StageBufs& b,
                               float theta, int tw, int th, hipStream_t s);
// Test hook: G = sqrt(G^2) and B, L, Z copied out densely (pitch W).
hipError_t launch_export_stages(const ImgArgs& a, const StageBufs& b,
                                float* dB, float* dL, uint8_t* dZ, float* dG,
                                hipStream_t s);

// ---- batched launch ----------------------------------------------------
// Device descriptor table of one batched call: BatchHeader, then n_images
// ImgArgs, then n_items1 pass-1 items, then n_items2 pass-2 items.
struct BatchItem {
    int32_t image;   // index into the ImgArgs array
    int32_t local;   // pass 1: sweep tile; pass 2: row run (STORE) or tile
};
struct BatchHeader {
    int32_t n_images;
    int32_t n_items1;
    int32_t n_items2;
    int32_t pass_mode;  // HX_PASS_STORE / RECOMPUTE / SPECULATE
    float theta;
    int32_t n_items0;   // SPECULATE: sampled-band items of pass 0
    int32_t pad[2];
    // SPECULATE: the listed pixels of pass-1 item k (a tile of image i)
    // occupy the image's entries for that tile (ImgArgs::list_base and
    // list_cap) of cand_code / cand_row, and cand_n[k] counts them; a tile
    // that set more pixels than its capacity is redone whole by pass 2.
    float* cand_code;
    int32_t* cand_row;
    uint32_t* cand_n;
    // SPECULATE: per-image lower bounds of max G^2, written by pass 0 and
    // only read by pass 1 (whose own maxima go to the images' slots).  A
    // bound is (epoch << 32) | bits of G^2: pass 0 folds values of the
    // current epoch with a 64-bit max, so a bound left by an earlier batch
    // needs no clearing (its epoch is lower); pass 2 advances the epoch.
    unsigned long long* bound;
    uint32_t* epoch;
};

size_t batch_table_bytes(int n_images, int64_t n_items1, int64_t n_items2,
                         int64_t n_items0);
// SPECULATE: pass-0 band geometry (8 sampled rows at the top of every
// sample_stride(H) rows: every H/32 rows clamped to [192, 256], but at
// least four bands in an image shorter than 768 rows) and the listed-pixel
// capacity of one pass-1 item, in entries.  Denser samples raise the bound
// (fewer pixels for pass 2); thinner ones cost pass 0 less.
constexpr int kSampleRows = 8;
__host__ __device__ inline int sample_stride(int64_t H) {
    const int64_t f = H / 32 < 192 ? 192 : (H / 32 > 256 ? 256 : H / 32);
    const int64_t q = H / 4 < 8 ? 8 : H / 4;
    return (int)(f < q ? f : q);
}
int64_t batch_sample_items(int ks, int64_t H, int64_t W);
// SPECULATE: listed-pixel capacity of each pass-1 tile of an image with
// `tiles` tiles: one entry per 16 of the image's pixels, spread evenly.
inline uint32_t spec_tile_cap(int64_t H, int64_t W, int64_t tiles) {
    return (uint32_t)((H * W) / (16 * tiles));
}
int batch_sweep_c();   // columns per lane of the batch sweep
int batch_wg_waves();  // waves per workgroup of the batch pass kernels
int batch_sweep_ty();  // rows per batch sweep tile
// Rows per pass-2 item of the STORE threshold for width W.
int batch_p2_rows(int64_t W);
// Zero the first n (read from the table) max slots; grid sized for
// max_images.  SPECULATE batches do not need it (pass 0 clears them).
hipError_t launch_batch_reset(const void* d_table, uint32_t* slots,
                              int max_images, hipStream_t s);
// One pass (phase 0, 1 or 2) over the table's item list on `grid`
// workgroups of four waves.  Phase 0 exists for SPECULATE only.
hipError_t launch_batch_phase(int ks, int pass_mode, int phase,
                              const void* d_table, const Taps& t, int grid,
                              hipStream_t s);

}  // namespace hx
