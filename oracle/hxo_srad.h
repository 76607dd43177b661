/*
 * hxo_srad.h -- the oracle for SRAD (speckle reducing anisotropic
 * diffusion), the second stencil + sum-reduction workload.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (same rules as hxo.h: only
 * the tests, the smoke check and the benchmark's CPU-baseline leg load it;
 * it shares nothing with the HIP path).
 *
 * The paper evaluates SRAD from the Rodinia suite (Evaluation) and says
 * only that its schedules fuse two large loops and turn its large sum
 * reductions into a three-level reduction tree (Use and Impact of
 * Schedules).  The iteration below is the published SRAD update as Rodinia
 * states it, read with the whole image as the region of interest:
 *
 *   S1  N = H W, mean = (sum J) / N, var = (sum J^2) / N - mean^2,
 *       q0^2 = var / mean^2                       (two sum reductions)
 *   S2  with clamped neighbours (row y-1 -> max(y-1, 0), etc.):
 *       dN = J(y-1,x) - J(y,x), dS = J(y+1,x) - J(y,x),
 *       dW = J(y,x-1) - J(y,x), dE = J(y,x+1) - J(y,x);
 *       g2 = (dN^2 + dS^2 + dW^2 + dE^2) / J^2,  l = (dN + dS + dW + dE) / J;
 *       q^2 = (g2 / 2 - l^2 / 16) / (1 + l / 4)^2;
 *       c = 1 / (1 + (q^2 - q0^2) / (q0^2 (1 + q0^2))), clamped to [0, 1];
 *       c = 1 when q0^2 <= 0 (a flat image, where every d is 0 anyway;
 *       the one-pass variance of a flat image rounds to 0 or just below)
 *   S3  D = c(y,x) dN + c(y+1,x) dS + c(y,x) dW + c(y,x+1) dE  (clamped),
 *       J' = J + (lambda / 4) D
 *
 * Every pixel of S2 and S3 reads the J of the previous iteration.  All
 * arithmetic is double precision; J is kept in double between iterations.
 * Inputs must be finite and > 0 (S2 divides by J).
 *
 * Errors: 0 on success, -1 on an invalid argument (null pointer, H or W
 * < 1, pitch < W, niter < 0).
 */
#ifndef HXO_SRAD_H
#define HXO_SRAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* S1 on a dense H*W double image: q0^2 (and mean, var if non-NULL). */
int hxo_srad_stats(const double* J, int64_t H, int64_t W, double* q0sqr, double* mean,
                   double* var);

/* S2 on a dense H*W double image with the given q0^2: c, dense H*W. */
int hxo_srad_coeff(const double* J, int64_t H, int64_t W, double q0sqr, double* c);

/* S3: J' from J and c (dense H*W each). */
int hxo_srad_update(const double* J, const double* c, int64_t H, int64_t W, double lambda,
                    double* Jout);

/* niter iterations of S1..S3 on an fp32 image (row pitch `pitch`); the
 * result goes to Jout (dense H*W doubles); q0sqr (nullable, niter doubles)
 * receives each iteration's q0^2. */
int hxo_srad(const float* J0, int64_t H, int64_t W, int64_t pitch, int32_t niter,
             double lambda, double* Jout, double* q0sqr);

#ifdef __cplusplus
}
#endif

#endif
