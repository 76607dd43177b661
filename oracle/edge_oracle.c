/*
 * edge_oracle.c -- plain, slow, obviously-correct CPU definition of the EDGE
 * pipeline.  TEST INFRASTRUCTURE ONLY (see hxo.h for who may use it and for
 * the stage definitions O1..O8).  Double precision throughout; every stage
 * is a direct loop over its definition.
 */
#include "hxo.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

/* O1: sampled Gaussian, normalised to unit sum. */
int hxo_gauss_weights(int32_t ksize, double sigma, double* g) {
    if (!g || ksize < 1 || (ksize % 2) == 0 || !(sigma > 0.0)) return -1;
    int32_t r = ksize / 2;
    double sum = 0.0;
    for (int32_t i = -r; i <= r; ++i) {
        g[i + r] = exp(-(double)(i * i) / (2.0 * sigma * sigma));
        sum += g[i + r];
    }
    for (int32_t i = 0; i < ksize; ++i) g[i] /= sum;
    return 0;
}

/* O2 + O3: direct 2-D weighted sum over the clamped k x k window. */
int hxo_blur(const float* I, int64_t H, int64_t W, int64_t pitch,
             int32_t ksize, double sigma, double* B) {
    if (!I || !B || H < 1 || W < 1 || pitch < W) return -1;
    double g[64];
    if (ksize > 63 || hxo_gauss_weights(ksize, sigma, g) != 0) return -1;
    int32_t r = ksize / 2;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int32_t i = -r; i <= r; ++i) {
                for (int32_t j = -r; j <= r; ++j) {
                    double w = g[i + r] * g[j + r];
                    int64_t yy = clampi(y + i, 0, H - 1);
                    int64_t xx = clampi(x + j, 0, W - 1);
                    acc += w * (double)I[yy * pitch + xx];
                }
            }
            B[y * W + x] = acc;
        }
    }
    return 0;
}

/* Read a dense H x W double image at clamped coordinates (O2). */
static double at(const double* X, int64_t H, int64_t W, int64_t y, int64_t x) {
    return X[clampi(y, 0, H - 1) * W + clampi(x, 0, W - 1)];
}

/* O4: 5-point Laplacian, summed pairwise as written in the definition. */
int hxo_laplacian(const double* B, int64_t H, int64_t W, double* L) {
    if (!B || !L || H < 1 || W < 1) return -1;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            double ns = at(B, H, W, y - 1, x) + at(B, H, W, y + 1, x);
            double ew = at(B, H, W, y, x - 1) + at(B, H, W, y, x + 1);
            L[y * W + x] = (ns + ew) - 4.0 * at(B, H, W, y, x);
        }
    }
    return 0;
}

/* O5: S = [L > 0]; Z = 1 iff the clamped 3x3 window holds both values. */
int hxo_zero_crossing(const double* L, int64_t H, int64_t W, uint8_t* Z) {
    if (!L || !Z || H < 1 || W < 1) return -1;
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            int smax = 0, smin = 1;
            for (int dy = -1; dy <= 1; ++dy) {
                for (int dx = -1; dx <= 1; ++dx) {
                    int s = at(L, H, W, y + dy, x + dx) > 0.0 ? 1 : 0;
                    if (s > smax) smax = s;
                    if (s < smin) smin = s;
                }
            }
            Z[y * W + x] = (uint8_t)(smax - smin);
        }
    }
    return 0;
}

/* O6: unnormalised Sobel pair and its L2 magnitude. */
int hxo_sobel(const double* B, int64_t H, int64_t W, double* G) {
    if (!B || !G || H < 1 || W < 1) return -1;
    static const double c[3] = {1.0, 2.0, 1.0};
    for (int64_t y = 0; y < H; ++y) {
        for (int64_t x = 0; x < W; ++x) {
            double gx = 0.0, gy = 0.0;
            for (int d = -1; d <= 1; ++d) {
                gx += c[d + 1] * (at(B, H, W, y + d, x + 1) - at(B, H, W, y + d, x - 1));
                gy += c[d + 1] * (at(B, H, W, y + 1, x + d) - at(B, H, W, y - 1, x + d));
            }
            G[y * W + x] = sqrt(gx * gx + gy * gy);
        }
    }
    return 0;
}

/* O7: sequential max, in increasing index order. */
double hxo_max(const double* G, int64_t n) {
    if (!G || n < 1) return NAN;
    double m = G[0];
    for (int64_t i = 1; i < n; ++i)
        if (G[i] > m) m = G[i];
    return m;
}

/* O8: strict threshold on G, gated by the zero-crossing flag. */
int hxo_threshold(const uint8_t* Z, const double* G, int64_t H, int64_t W,
                  double tau, uint8_t* mask, int64_t mask_pitch) {
    if (!Z || !G || !mask || H < 1 || W < 1 || mask_pitch < W) return -1;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x)
            mask[y * mask_pitch + x] =
                (Z[y * W + x] == 1 && G[y * W + x] > tau) ? 1 : 0;
    return 0;
}

int hxo_edge_detect(const float* I, int64_t H, int64_t W, int64_t pitch,
                    int32_t ksize, double sigma, double theta,
                    uint8_t* mask, int64_t mask_pitch, double* M_out,
                    double* B, double* L, uint8_t* Z, double* G) {
    if (!I || !mask || H < 1 || W < 1 || pitch < W || mask_pitch < W) return -1;
    size_t n = (size_t)H * (size_t)W;
    double* b = B ? B : (double*)malloc(n * sizeof(double));
    double* l = L ? L : (double*)malloc(n * sizeof(double));
    uint8_t* z = Z ? Z : (uint8_t*)malloc(n);
    double* g = G ? G : (double*)malloc(n * sizeof(double));
    int rc = -1;
    if (b && l && z && g &&
        hxo_blur(I, H, W, pitch, ksize, sigma, b) == 0 &&
        hxo_laplacian(b, H, W, l) == 0 &&
        hxo_zero_crossing(l, H, W, z) == 0 &&
        hxo_sobel(b, H, W, g) == 0) {
        double M = hxo_max(g, (int64_t)n);
        double tau = theta * M;
        rc = hxo_threshold(z, g, H, W, tau, mask, mask_pitch);
        if (M_out) *M_out = M;
    }
    if (!B) free(b);
    if (!L) free(l);
    if (!Z) free(z);
    if (!G) free(g);
    return rc;
}

typedef struct {
    int32_t first, step, n;
    const float* const* I;
    const int64_t *H, *W, *pitch, *mask_pitch;
    int32_t ksize;
    double sigma, theta;
    uint8_t* const* mask;
    double* M;
    int rc;
} many_job;

static void* many_worker(void* arg) {
    many_job* j = (many_job*)arg;
    j->rc = 0;
    for (int32_t i = j->first; i < j->n; i += j->step) {
        if (hxo_edge_detect(j->I[i], j->H[i], j->W[i], j->pitch[i], j->ksize,
                            j->sigma, j->theta, j->mask[i], j->mask_pitch[i],
                            j->M ? &j->M[i] : NULL, NULL, NULL, NULL, NULL) != 0)
            j->rc = -1;
    }
    return NULL;
}

int hxo_edge_detect_many(int32_t n, const float* const* I, const int64_t* H,
                         const int64_t* W, const int64_t* pitch,
                         int32_t ksize, double sigma, double theta,
                         uint8_t* const* mask, const int64_t* mask_pitch,
                         double* M_out, int32_t nthreads) {
    if (n < 0 || !I || !H || !W || !pitch || !mask || !mask_pitch) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > n) nthreads = n > 0 ? n : 1;
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    many_job* jobs = (many_job*)calloc((size_t)nthreads, sizeof(many_job));
    if (!th || !jobs) { free(th); free(jobs); return -1; }
    for (int32_t t = 0; t < nthreads; ++t) {
        many_job j = {t, nthreads, n, I, H, W, pitch, mask_pitch, ksize,
                      sigma, theta, mask, M_out, 0};
        jobs[t] = j;
    }
    int rc = 0;
    int32_t started = 0;
    for (int32_t t = 1; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, many_worker, &jobs[t]) != 0) break;
        ++started;
    }
    many_worker(&jobs[0]);
    for (int32_t t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    /* Jobs that could not get a thread run here, serially. */
    for (int32_t t = started + 1; t < nthreads; ++t) many_worker(&jobs[t]);
    for (int32_t t = 0; t < nthreads; ++t)
        if (jobs[t].rc != 0) rc = -1;
    free(th);
    free(jobs);
    return rc;
}
