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
// Two forms, bit-identical to each other:
//   unfused  k_srad_coeff writes c; k_srad_update reads it and writes J'
//   fused    k_srad_fused stages a J tile (with a 2-pixel halo) and its c
//            tile in LDS and writes J' directly: c never reaches HBM.
// Both updates fold the sums of J' for the next iteration with the same
// pixel-to-thread map: thread (per 32x64 tile, 256 threads) -> 8 pixels,
// summed in fp64 in a fixed order (level 1), xor-shuffled across the wave
// (level 2), one partial pair per wave; k_srad_stats folds the partials in
// a fixed order in one workgroup (level 3).  Sums are therefore the same
// bits for both forms and every run.
#include <hip/hip_runtime.h>

#include "../../include/hx.h"
#include "hx_kernels.h"

namespace hx {
namespace {

constexpr int kTH = 32, kTW = 64;  // output tile: rows x columns

__device__ __forceinline__ int clampi_s(int v, int lo, int hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// c of one pixel from its value and differences (one fixed order).
__device__ __forceinline__ float srad_c(float j, float dN, float dS, float dW, float dE,
                                        float q0sqr) {
    const float g2 = (dN * dN + dS * dS + dW * dW + dE * dE) / (j * j);
    const float l = (dN + dS + dW + dE) / j;
    const float num = 0.5f * g2 - (l * l) * 0.0625f;
    const float den = 1.0f + 0.25f * l;
    const float qsqr = num / (den * den);
    if (!(q0sqr > 0.0f)) return 1.0f;
    float c = 1.0f / (1.0f + (qsqr - q0sqr) / (q0sqr * (1.0f + q0sqr)));
    c = c < 0.0f ? 0.0f : c;
    c = c > 1.0f ? 1.0f : c;
    return c;
}

__device__ __forceinline__ float srad_new(float j, float dN, float dS, float dW, float dE,
                                          float c, float cS, float cE, float step) {
    const float D = c * dN + cS * dS + c * dW + cE * dE;
    return j + step * D;
}

// Level 2: fp64 sums across the wave (xor butterfly), result in every lane.
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct SradImg {
    const float* J;    // input of this iteration
    float* out;        // output of this iteration (J' or c)
    int64_t pin, pout; // row pitches (elements)
    int H, W;
};

__device__ __forceinline__ int tiles_x(int W) { return (W + kTW - 1) / kTW; }

// The pixels of thread t in tile (ty0, tx0): column tx0 + t % 64, rows
// ty0 + t / 64 + 4 k, k = 0..7.
__device__ __forceinline__ void emit_partials(double s, double s2, double* partials) {
    s = wave_sum_d(s);
    s2 = wave_sum_d(s2);
    if ((threadIdx.x & 63) == 0) {
        const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
        partials[2 * w] = s;
        partials[2 * w + 1] = s2;
    }
}

}  // namespace

// Sums of the initial image (same map as the updates).
__global__ __launch_bounds__(256) void k_srad_sums(SradImg a, double* partials) {
    const int tx = blockIdx.x % tiles_x(a.W), ty = blockIdx.x / tiles_x(a.W);
    const int x = tx * kTW + (threadIdx.x & 63);
    double s = 0.0, s2 = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int y = ty * kTH + (threadIdx.x >> 6) + 4 * k;
        if (y < a.H && x < a.W) {
            const double v = a.J[(int64_t)y * a.pin + x];
            s += v;
            s2 += v * v;
        }
    }
    emit_partials(s, s2, partials);
}

// Level 3: one workgroup folds n partial pairs into q0^2 (written to q and,
// if q_log, to q_log[it]).
__global__ __launch_bounds__(256) void k_srad_stats(const double* partials, int64_t n,
                                                    double npix, float* q, double* q_log,
                                                    int it) {
    __shared__ double ls[256], ls2[256];
    double s = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        s += partials[2 * i];
        s2 += partials[2 * i + 1];
    }
    ls[threadIdx.x] = s;
    ls2[threadIdx.x] = s2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            ls[threadIdx.x] += ls[threadIdx.x + o];
            ls2[threadIdx.x] += ls2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = ls[0] / npix;
        const double var = ls2[0] / npix - mean * mean;
        const double q0 = var / (mean * mean);
        *q = (float)q0;
        if (q_log) q_log[it] = q0;
    }
}

// Unfused, first loop: c of every pixel.
__global__ __launch_bounds__(256) void k_srad_coeff(SradImg a, const float* q) {
    const float q0 = *q;
    const int tx = blockIdx.x % tiles_x(a.W), ty = blockIdx.x / tiles_x(a.W);
    const int x = tx * kTW + (threadIdx.x & 63);
    if (x >= a.W) return;
    const int xw = x > 0 ? x - 1 : 0, xe = x + 1 < a.W ? x + 1 : a.W - 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int y = ty * kTH + (threadIdx.x >> 6) + 4 * k;
        if (y >= a.H) break;
        const float* r = a.J + (int64_t)y * a.pin;
        const float j = r[x];
        const float dN = a.J[(int64_t)(y > 0 ? y - 1 : 0) * a.pin + x] - j;
        const float dS = a.J[(int64_t)(y + 1 < a.H ? y + 1 : a.H - 1) * a.pin + x] - j;
        const float dW = r[xw] - j;
        const float dE = r[xe] - j;
        a.out[(int64_t)y * a.pout + x] = srad_c(j, dN, dS, dW, dE, q0);
    }
}

// Unfused, second loop: J' from J and c, plus the sums of J'.
__global__ __launch_bounds__(256) void k_srad_update(SradImg a, const float* c, int64_t pc,
                                                     float step, double* partials) {
    const int tx = blockIdx.x % tiles_x(a.W), ty = blockIdx.x / tiles_x(a.W);
    const int x = tx * kTW + (threadIdx.x & 63);
    double s = 0.0, s2 = 0.0;
    if (x < a.W) {
        const int xw = x > 0 ? x - 1 : 0, xe = x + 1 < a.W ? x + 1 : a.W - 1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int y = ty * kTH + (threadIdx.x >> 6) + 4 * k;
            if (y >= a.H) break;
            const int ys = y + 1 < a.H ? y + 1 : a.H - 1;
            const float* r = a.J + (int64_t)y * a.pin;
            const float j = r[x];
            const float dN = a.J[(int64_t)(y > 0 ? y - 1 : 0) * a.pin + x] - j;
            const float dS = a.J[(int64_t)ys * a.pin + x] - j;
            const float dW = r[xw] - j;
            const float dE = r[xe] - j;
            const float cc = c[(int64_t)y * pc + x];
            const float cS = c[(int64_t)ys * pc + x];
            const float cE = c[(int64_t)y * pc + xe];
            const float v = srad_new(j, dN, dS, dW, dE, cc, cS, cE, step);
            a.out[(int64_t)y * a.pout + x] = v;
            s += (double)v;
            s2 += (double)v * (double)v;
        }
    }
    emit_partials(s, s2, partials);
}

// Fused: the J tile with its halo and the c tile live in LDS.
__global__ __launch_bounds__(256) void k_srad_fused(SradImg a, const float* q, float step,
                                                    double* partials) {
    // J rows y0-1 .. y0+kTH+1, columns x0-1 .. x0+kTW+1 (clamped); c rows
    // y0 .. y0+kTH, columns x0 .. x0+kTW (the tile plus its south and east
    // neighbours).
    constexpr int JR = kTH + 3, JC = kTW + 3, CR = kTH + 1, CC = kTW + 1;
    __shared__ float sJ[JR][JC];
    __shared__ float sC[CR][CC];
    const float q0 = *q;
    const int tx = blockIdx.x % tiles_x(a.W), ty = blockIdx.x / tiles_x(a.W);
    const int x0 = tx * kTW, y0 = ty * kTH;
    for (int i = threadIdx.x; i < JR * JC; i += 256) {
        const int r = i / JC, cidx = i - r * JC;
        const int y = clampi_s(y0 - 1 + r, 0, a.H - 1);
        const int x = clampi_s(x0 - 1 + cidx, 0, a.W - 1);
        sJ[r][cidx] = a.J[(int64_t)y * a.pin + x];
    }
    __syncthreads();
    // c at J-tile position (r, cidx) = image pixel (y0 + r - 1, x0 + cidx - 1)
    // for r, cidx in 1 .. kTH+1 / kTW+1.  A pixel outside the image takes
    // the clamped pixel's c: the clamped neighbours read the same J values,
    // so computing it from the J tile at the clamped position gives it.
    for (int i = threadIdx.x; i < CR * CC; i += 256) {
        const int r = i / CC, cidx = i - r * CC;
        const int y = clampi_s(y0 + r, 0, a.H - 1), x = clampi_s(x0 + cidx, 0, a.W - 1);
        const int ry = y - y0 + 1, rx = x - x0 + 1;  // in the J tile
        const float j = sJ[ry][rx];
        const float vN = y > 0 ? sJ[ry - 1][rx] : j;
        const float vS = y + 1 < a.H ? sJ[ry + 1][rx] : j;
        const float vW = x > 0 ? sJ[ry][rx - 1] : j;
        const float vE = x + 1 < a.W ? sJ[ry][rx + 1] : j;
        sC[r][cidx] = srad_c(j, vN - j, vS - j, vW - j, vE - j, q0);
    }
    __syncthreads();
    const int lx = threadIdx.x & 63;
    const int x = x0 + lx;
    double s = 0.0, s2 = 0.0;
    if (x < a.W) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int ly = (threadIdx.x >> 6) + 4 * k;
            const int y = y0 + ly;
            if (y >= a.H) break;
            const float j = sJ[ly + 1][lx + 1];
            const float vN = y > 0 ? sJ[ly][lx + 1] : j;
            const float vS = y + 1 < a.H ? sJ[ly + 2][lx + 1] : j;
            const float vW = x > 0 ? sJ[ly + 1][lx] : j;
            const float vE = x + 1 < a.W ? sJ[ly + 1][lx + 2] : j;
            const float cc = sC[ly][lx];
            const float cS = sC[y + 1 < a.H ? ly + 1 : ly][lx];
            const float cE = sC[ly][x + 1 < a.W ? lx + 1 : lx];
            const float v = srad_new(j, vN - j, vS - j, vW - j, vE - j, cc, cS, cE, step);
            a.out[(int64_t)y * a.pout + x] = v;
            s += (double)v;
            s2 += (double)v * (double)v;
        }
    }
    emit_partials(s, s2, partials);
}

int64_t srad_tiles(int64_t H, int64_t W) {
    return ((W + kTW - 1) / kTW) * ((H + kTH - 1) / kTH);
}

hipError_t launch_srad(const float* J, float* Jb, int64_t pj, int64_t pb, float* cbuf,
                       int64_t pc, double* partials, float* q, double* q_log, int H, int W,
                       int niter, float lambda, bool fused, hipStream_t s) {
    const int64_t tiles = srad_tiles(H, W);
    const int64_t nparts = tiles * 4;
    const double npix = (double)H * (double)W;
    const float step = 0.25f * lambda;
    SradImg a0{J, nullptr, pj, 0, H, W};
    hipLaunchKernelGGL(k_srad_sums, dim3((unsigned)tiles), dim3(256), 0, s, a0, partials);
    hipError_t e = hipGetLastError();
    const float* cur = J;
    int64_t pcur = pj;
    for (int it = 0; it < niter && e == hipSuccess; ++it) {
        hipLaunchKernelGGL(k_srad_stats, dim3(1), dim3(256), 0, s, (const double*)partials,
                           nparts, npix, q, q_log, it);
        // Iteration it reads `cur` and writes the other buffer.
        float* nxt = (cur == J) ? Jb : const_cast<float*>(J);
        const int64_t pnxt = (cur == J) ? pb : pj;
        if (fused) {
            SradImg a{cur, nxt, pcur, pnxt, H, W};
            hipLaunchKernelGGL(k_srad_fused, dim3((unsigned)tiles), dim3(256), 0, s, a,
                               (const float*)q, step, partials);
        } else {
            SradImg ac{cur, cbuf, pcur, pc, H, W};
            hipLaunchKernelGGL(k_srad_coeff, dim3((unsigned)tiles), dim3(256), 0, s, ac,
                               (const float*)q);
            SradImg au{cur, nxt, pcur, pnxt, H, W};
            hipLaunchKernelGGL(k_srad_update, dim3((unsigned)tiles), dim3(256), 0, s, au,
                               (const float*)cbuf, pc, step, partials);
        }
        e = hipGetLastError();
        cur = nxt;
        pcur = pnxt;
    }
    return e;
}

}  // namespace hx
