/*
 * srad_oracle.c -- plain fp64 loops over the SRAD definitions S1..S3 of
 * hxo_srad.h.  Test infrastructure only.
 */
#include "hxo_srad.h"

#include <stdlib.h>
#include <string.h>

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

static double at(const double* X, int64_t H, int64_t W, int64_t y, int64_t x) {
    return X[clampi(y, 0, H - 1) * W + clampi(x, 0, W - 1)];
}

/* S1 */
int hxo_srad_stats(const double* J, int64_t H, int64_t W, double* q0sqr, double* mean,
                   double* var) {
    if (!J || !q0sqr || H < 1 || W < 1) return -1;
    double s = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < H * W; ++i) {
        s += J[i];
        s2 += J[i] * J[i];
    }
    const double n = (double)(H * W);
    const double m = s / n;
    const double v = s2 / n - m * m;
    *q0sqr = v / (m * m);
    if (mean) *mean = m;
    if (var) *var = v;
    return 0;
}

/* S2 */
int hxo_srad_coeff(const double* J, int64_t H, int64_t W, double q0sqr, double* c) {
    if (!J || !c || H < 1 || W < 1) return -1;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            const double j = J[y * W + x];
            const double dN = at(J, H, W, y - 1, x) - j;
            const double dS = at(J, H, W, y + 1, x) - j;
            const double dW = at(J, H, W, y, x - 1) - j;
            const double dE = at(J, H, W, y, x + 1) - j;
            const double g2 = (dN * dN + dS * dS + dW * dW + dE * dE) / (j * j);
            const double l = (dN + dS + dW + dE) / j;
            const double num = 0.5 * g2 - (l * l) / 16.0;
            const double den = 1.0 + 0.25 * l;
            const double qsqr = num / (den * den);
            double cv = 1.0;
            if (q0sqr > 0.0) {
                cv = 1.0 / (1.0 + (qsqr - q0sqr) / (q0sqr * (1.0 + q0sqr)));
                if (cv < 0.0) cv = 0.0;
                if (cv > 1.0) cv = 1.0;
            }
            c[y * W + x] = cv;
        }
    return 0;
}

/* S3 */
int hxo_srad_update(const double* J, const double* c, int64_t H, int64_t W, double lambda,
                    double* Jout) {
    if (!J || !c || !Jout || H < 1 || W < 1) return -1;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            const double j = J[y * W + x];
            const double dN = at(J, H, W, y - 1, x) - j;
            const double dS = at(J, H, W, y + 1, x) - j;
            const double dW = at(J, H, W, y, x - 1) - j;
            const double dE = at(J, H, W, y, x + 1) - j;
            const double cc = c[y * W + x];
            const double D = cc * dN + at(c, H, W, y + 1, x) * dS + cc * dW +
                             at(c, H, W, y, x + 1) * dE;
            Jout[y * W + x] = j + 0.25 * lambda * D;
        }
    return 0;
}

int hxo_srad(const float* J0, int64_t H, int64_t W, int64_t pitch, int32_t niter,
             double lambda, double* Jout, double* q0sqr) {
    if (!J0 || !Jout || H < 1 || W < 1 || pitch < W || niter < 0) return -1;
    const size_t n = (size_t)(H * W);
    double* J = (double*)malloc(sizeof(double) * n);
    double* c = (double*)malloc(sizeof(double) * n);
    if (!J || !c) {
        free(J);
        free(c);
        return -1;
    }
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) J[y * W + x] = (double)J0[y * pitch + x];
    for (int32_t it = 0; it < niter; ++it) {
        double q = 0.0;
        hxo_srad_stats(J, H, W, &q, NULL, NULL);
        if (q0sqr) q0sqr[it] = q;
        hxo_srad_coeff(J, H, W, q, c);
        hxo_srad_update(J, c, H, W, lambda, Jout);
        memcpy(J, Jout, sizeof(double) * n);
    }
    memcpy(Jout, J, sizeof(double) * n);
    free(J);
    free(c);
    return 0;
}
