/*
 * hxo.h -- the oracle for the EDGE edge-detection pipeline.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load this
 * library.  It shares no source, header, table or helper with the HIP path
 * under paper_2503_10855_amd/csrc, and it imports nothing from it.
 *
 * What it computes.  The paper (Evaluation, the EDGE benchmark; Use and
 * Impact of Schedules, the max_gradient reduction) names EDGE as a pipeline
 * of nested parallel loops (fork-joins, "Representing Parallelism with
 * Fork-Joins") ending in a large max reduction, but never spells out its
 * stages.  The stage list below is the reading adopted for this repository:
 *
 *   O1  g[i] = exp(-i^2 / (2 sigma^2)), i in [-r, r], r = (k-1)/2,
 *       normalised so that sum g = 1; the 2-D kernel is w[i][j] = g[i] g[j].
 *   O2  every stage reads its input at clamped coordinates
 *       (clamp(y, 0, H-1), clamp(x, 0, W-1)).
 *   O3  B(y,x) = sum_{i,j} w[i][j] I(y+i, x+j)        (direct 2-D sum)
 *   O4  L = ((B(y-1,x) + B(y+1,x)) + (B(y,x-1) + B(y,x+1))) - 4 B(y,x)
 *   O5  S = [L > 0];  Z = max_{3x3} S - min_{3x3} S   (in {0,1})
 *   O6  gx = sum_dy c_dy (B(y+dy,x+1) - B(y+dy,x-1)),
 *       gy = sum_dx c_dx (B(y+1,x+dx) - B(y-1,x+dx)),  c = (1,2,1);
 *       G = sqrt(gx^2 + gy^2)
 *   O7  M = max over all pixels of G                 (the monoid reduction)
 *   O8  tau = theta * M;  mask = 1 iff Z == 1 and G > tau   (strict)
 *
 * All arithmetic is double precision on the fp32 input (promoted exactly).
 * Every routine is a plain loop over the definition: no blocking, no
 * separable factorisation, no reordering.
 *
 * Errors: every routine returns 0 on success and -1 on an invalid argument
 * (null pointer, H or W < 1, pitch < W, even or non-positive ksize,
 * sigma <= 0).  Nothing is allocated by the caller-facing routines except
 * hxo_edge_detect, which allocates its own temporaries when the caller
 * passes NULL for a stage buffer, and frees them before returning.
 */
#ifndef HXO_H
#define HXO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* O1: fill g[0..k-1] with the normalised sampled Gaussian (index i-r). */
int hxo_gauss_weights(int32_t ksize, double sigma, double* g);

/* O2+O3: I is fp32, row-major with row pitch `pitch` elements; B is dense
 * H*W doubles. */
int hxo_blur(const float* I, int64_t H, int64_t W, int64_t pitch,
             int32_t ksize, double sigma, double* B);

/* O4: B and L dense H*W. */
int hxo_laplacian(const double* B, int64_t H, int64_t W, double* L);

/* O5: L dense H*W doubles -> Z dense H*W bytes in {0,1}. */
int hxo_zero_crossing(const double* L, int64_t H, int64_t W, uint8_t* Z);

/* O6: B dense -> G dense (the magnitude, after the square root). */
int hxo_sobel(const double* B, int64_t H, int64_t W, double* G);

/* O7: max over n >= 1 values; returns the maximum (NaN if n < 1). */
double hxo_max(const double* G, int64_t n);

/* O8: mask[y*mask_pitch + x] = (Z[y*W+x] == 1 && G[y*W+x] > tau). */
int hxo_threshold(const uint8_t* Z, const double* G, int64_t H, int64_t W,
                  double tau, uint8_t* mask, int64_t mask_pitch);

/* O1..O8 for one image.  mask has row pitch mask_pitch bytes.  *M_out
 * receives M (may be NULL).  B, L, Z, G are optional dense H*W outputs of
 * the intermediate stages (NULL = not wanted). */
int hxo_edge_detect(const float* I, int64_t H, int64_t W, int64_t pitch,
                    int32_t ksize, double sigma, double theta,
                    uint8_t* mask, int64_t mask_pitch, double* M_out,
                    double* B, double* L, uint8_t* Z, double* G);

/* The same for n independent images, one image per worker thread, used
 * only to time the oracle as a CPU baseline.  Results are identical to n
 * calls of hxo_edge_detect.  nthreads < 1 means 1. */
int hxo_edge_detect_many(int32_t n, const float* const* I, const int64_t* H,
                         const int64_t* W, const int64_t* pitch,
                         int32_t ksize, double sigma, double theta,
                         uint8_t* const* mask, const int64_t* mask_pitch,
                         double* M_out, int32_t nthreads);

#ifdef __cplusplus
}
#endif

#endif /* HXO_H */
