/*
 * Photometric losses. TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Paper Sec. 3: photometric L1 plus D-SSIM between rendered and target images.
 * Sec. 5.1.2, Eqs. 7-10: D-SSIM = 1 - SSIM with
 *   SSIM = (2 mu1 mu2 + C1)(2 tau12 + C2) / ((mu1^2 + mu2^2 + C1)(tau1^2 + tau2^2 + C2)),
 * the moments being inner products of local patches with a 2D Gaussian kernel.
 * Readings (the paper names MS-SSIM but writes the single-scale formula): an
 * 11x11 window of the sampled Gaussian with sigma = 1.5, normalised to sum 1,
 * centred on each pixel, zero outside the image; C1 = 0.01^2, C2 = 0.03^2;
 * both losses are means over every (view, channel, row, column), and
 *   L = w_l1 * L1 + w_dssim * (1 - mean SSIM).
 * The gradient of |x| at 0 is taken as 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ora.h"

#define WIN 11
#define HALF 5
#define SIGMA 1.5
#define SSIM_C1 (0.01 * 0.01)
#define SSIM_C2 (0.03 * 0.03)

static void window(double w[WIN][WIN])
{
    double s = 0.0;
    for (int i = 0; i < WIN; ++i)
        for (int j = 0; j < WIN; ++j) {
            const double u = i - HALF, v = j - HALF;
            w[i][j] = exp(-(u * u + v * v) / (2.0 * SIGMA * SIGMA));
            s += w[i][j];
        }
    for (int i = 0; i < WIN; ++i)
        for (int j = 0; j < WIN; ++j) w[i][j] /= s;
}

typedef struct {
    double mu1, mu2, m11, m22, m12;
} moments;

static moments local_moments(int W, int H, const double* a, const double* b, int x, int y, double w[WIN][WIN])
{
    moments m = {0, 0, 0, 0, 0};
    for (int i = 0; i < WIN; ++i) {
        const int yy = y + i - HALF;
        if (yy < 0 || yy >= H) continue;
        for (int j = 0; j < WIN; ++j) {
            const int xx = x + j - HALF;
            if (xx < 0 || xx >= W) continue;
            const double p = a[(int64_t)yy * W + xx], q = b[(int64_t)yy * W + xx], k = w[i][j];
            m.mu1 += k * p;
            m.mu2 += k * q;
            m.m11 += k * p * p;
            m.m22 += k * q * q;
            m.m12 += k * p * q;
        }
    }
    return m;
}

/* SSIM value and its partial derivatives with respect to mu1, m11 = E[a^2], m12 = E[ab] */
static double ssim_terms(moments m, double* d_mu1, double* d_m11, double* d_m12)
{
    const double s11 = m.m11 - m.mu1 * m.mu1, s22 = m.m22 - m.mu2 * m.mu2, s12 = m.m12 - m.mu1 * m.mu2;
    const double A1 = 2 * m.mu1 * m.mu2 + SSIM_C1, A2 = 2 * s12 + SSIM_C2;
    const double B1 = m.mu1 * m.mu1 + m.mu2 * m.mu2 + SSIM_C1, B2 = s11 + s22 + SSIM_C2;
    const double S = A1 * A2 / (B1 * B2);
    if (d_mu1) {
        *d_mu1 = 2 * m.mu2 * (A2 - A1) / (B1 * B2) - 2 * m.mu1 * S * (1.0 / B1 - 1.0 / B2);
        *d_m11 = -S / B2;
        *d_m12 = 2 * A1 / (B1 * B2);
    }
    return S;
}

int ora_ssim_map(int32_t W, int32_t H, const double* a, const double* b, double* out)
{
    double w[WIN][WIN];
    window(w);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) out[(int64_t)y * W + x] = ssim_terms(local_moments(W, H, a, b, x, y, w), 0, 0, 0);
    return 0;
}

int ora_loss(const ora_cams* c, const double* const* img, const double* const* tgt, double w_l1, double w_dssim,
             double* loss, double* const* dl_dimg)
{
    double N = 0.0;
    for (int v = 0; v < c->B; ++v) N += 3.0 * c->wh[2 * v] * c->wh[2 * v + 1];
    double w[WIN][WIN];
    window(w);
    double l1 = 0.0, ssum = 0.0;
    for (int v = 0; v < c->B; ++v) {
        const int W = c->wh[2 * v], H = c->wh[2 * v + 1];
        const int64_t HW = (int64_t)H * W;
        for (int ch = 0; ch < 3; ++ch) {
            const double* a = img[v] + ch * HW;
            const double* b = tgt[v] + ch * HW;
            double* g = dl_dimg ? dl_dimg[v] + ch * HW : NULL;
            double l1_c = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : l1_c)
            for (int64_t i = 0; i < HW; ++i) {
                const double d = a[i] - b[i];
                l1_c += fabs(d);
                if (g) g[i] = w_l1 * ((d > 0) - (d < 0)) / N;
            }
            l1 += l1_c;
            if (w_dssim == 0.0) continue;
            double* dmu = (double*)malloc(sizeof(double) * 3 * HW);
            double *d11 = dmu + HW, *d12 = dmu + 2 * HW;
            double s_c = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s_c)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    const int64_t i = (int64_t)y * W + x;
                    s_c += ssim_terms(local_moments(W, H, a, b, x, y, w), &dmu[i], &d11[i], &d12[i]);
                }
            ssum += s_c;
            if (g) {
                /* dL/da(q) = -w_dssim/N sum_p w(q-p) [dS/dmu1(p) + 2 a(q) dS/dm11(p) + b(q) dS/dm12(p)] */
#pragma omp parallel for schedule(static)
                for (int y = 0; y < H; ++y)
                    for (int x = 0; x < W; ++x) {
                        double s0 = 0, s1 = 0, s2 = 0;
                        for (int i = 0; i < WIN; ++i) {
                            const int yy = y - (i - HALF);
                            if (yy < 0 || yy >= H) continue;
                            for (int j = 0; j < WIN; ++j) {
                                const int xx = x - (j - HALF);
                                if (xx < 0 || xx >= W) continue;
                                const int64_t p = (int64_t)yy * W + xx;
                                s0 += w[i][j] * dmu[p];
                                s1 += w[i][j] * d11[p];
                                s2 += w[i][j] * d12[p];
                            }
                        }
                        const int64_t q = (int64_t)y * W + x;
                        g[q] += -w_dssim / N * (s0 + 2.0 * a[q] * s1 + b[q] * s2);
                    }
            }
            free(dmu);
        }
    }
    *loss = w_l1 * l1 / N + w_dssim * (1.0 - ssum / N);
    return 0;
}
