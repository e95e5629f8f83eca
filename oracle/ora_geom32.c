/*
 * Single-precision decision geometry (oracle side). TEST INFRASTRUCTURE ONLY.
 *
 * The rasterizer's binning decisions -- does a Gaussian take part in a view,
 * which tiles does it cover, what is its 32-bit depth key -- are functions of
 * single-precision arithmetic in the kernel. To compare binning bit for bit,
 * the oracle takes these decisions in single precision with the operation
 * sequence written out below (every multiply and add is its own rounding;
 * fused multiply-adds appear only where fmaf() is written; division and square
 * root are IEEE). This file must be compiled with -ffp-contract=off. The
 * per-pixel cut and clamp tests are not taken here: the walk decides them in
 * double precision and flags the pixels where single precision could decide
 * otherwise. The single-precision projected mean and conic computed here are
 * also what the image-parity mode blends with (the kernel's geometry).
 *
 * Paper passages: Sec. 3 (covariance R S S^T R^T, EWA projection of mean and
 * covariance); Appendix "Rasterization in multi-view training" (frustum culling,
 * duplication per covered tile, depth in the sort key). The paper gives no
 * formulas for culling, radius or cut; the readings used are: near plane
 * z > 0.2, dilation +0.3 px^2 on the 2D covariance diagonal,
 * pixel centres at (x+0.5, y+0.5), a pixel is covered iff power >= cut with
 * cut = max(-4.5, -ln(255 o)) (inside the 3-sigma ellipse and alpha >= 1/255,
 * the latter tested in the power domain so that no exponential enters the
 * decision), and the footprint is the pixel box of the per-axis extents of
 * that cut ellipse.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "ora.h"

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* Natural logarithm of the opacity threshold that sizes the footprint: x = 2^e m
 * with m in [sqrt(1/2), sqrt(2)], ln m = 2 atanh(s), s = (m-1)/(m+1), series to
 * s^9. It only has to be a fixed, accurate (~1e-7) function; because the
 * footprint decides binning, both sides evaluate it with this exact sequence.
 * Non-positive or NaN input gives -inf. */
float ora_ln32(float x)
{
    if (!(x > 0.0f)) return -INFINITY;
    if (x == INFINITY) return INFINITY;
    int e = 0;
    uint32_t b = f2u(x);
    if (b < 0x00800000u) {            /* subnormal: scale by 2^23 exactly */
        x = x * 8388608.0f;
        b = f2u(x);
        e = -23;
    }
    e += (int)(b >> 23) - 127;
    float m = u2f((b & 0x007fffffu) | 0x3f800000u);
    if (m > 1.41421356f) {
        m = m * 0.5f;
        e += 1;
    }
    float s = (m - 1.0f) / (m + 1.0f);
    float s2 = s * s;
    float p = 0.111111111f;
    p = fmaf(p, s2, 0.142857143f);
    p = fmaf(p, s2, 0.2f);
    p = fmaf(p, s2, 0.333333333f);
    float s_2 = s + s;
    float lnm = fmaf(s_2 * s2, p, s_2);
    return fmaf((float)e, 0.693147182f, lnm);
}

void ora_geom32_eval(const float mu[3], const float s[3], const float q[4], float o,
                     const float R[9], const float t[3], float fx, float fy, float cx, float cy,
                     int32_t W, int32_t H, ora_g32* g)
{
    memset(g, 0, sizeof(*g));
    g->participates = 0;

    /* camera-space mean */
    float tx = fmaf(R[0], mu[0], fmaf(R[1], mu[1], fmaf(R[2], mu[2], t[0])));
    float ty = fmaf(R[3], mu[0], fmaf(R[4], mu[1], fmaf(R[5], mu[2], t[1])));
    float tz = fmaf(R[6], mu[0], fmaf(R[7], mu[1], fmaf(R[8], mu[2], t[2])));
    g->depth = tz;
    g->depth_bits = f2u(tz);
    if (!(tz > 0.2f)) return;

    /* projected mean (pixels) */
    float iz = 1.0f / tz;
    float u = fx * tx;
    float w = fy * ty;
    float mx = fmaf(u, iz, cx);
    float my = fmaf(w, iz, cy);
    g->mx = mx;
    g->my = my;

    /* rotation from the normalised quaternion (w,x,y,z) */
    float n2 = fmaf(q[0], q[0], fmaf(q[1], q[1], fmaf(q[2], q[2], q[3] * q[3])));
    if (!(n2 > 0.0f)) return;
    float inv = 1.0f / sqrtf(n2);
    float qw = q[0] * inv, qx = q[1] * inv, qy = q[2] * inv, qz = q[3] * inv;
    float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    float r[9];
    r[0] = 1.0f - 2.0f * (yy + zz);
    r[1] = 2.0f * (xy - wz);
    r[2] = 2.0f * (xz + wy);
    r[3] = 2.0f * (xy + wz);
    r[4] = 1.0f - 2.0f * (xx + zz);
    r[5] = 2.0f * (yz - wx);
    r[6] = 2.0f * (xz - wy);
    r[7] = 2.0f * (yz + wx);
    r[8] = 1.0f - 2.0f * (xx + yy);

    /* M = rot * diag(s);  Sigma = M M^T (upper triangle) */
    float M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = r[3 * i + j] * s[j];
    float S00 = fmaf(M[0], M[0], fmaf(M[1], M[1], M[2] * M[2]));
    float S01 = fmaf(M[0], M[3], fmaf(M[1], M[4], M[2] * M[5]));
    float S02 = fmaf(M[0], M[6], fmaf(M[1], M[7], M[2] * M[8]));
    float S11 = fmaf(M[3], M[3], fmaf(M[4], M[4], M[5] * M[5]));
    float S12 = fmaf(M[3], M[6], fmaf(M[4], M[7], M[5] * M[8]));
    float S22 = fmaf(M[6], M[6], fmaf(M[7], M[7], M[8] * M[8]));
    float S[9] = {S00, S01, S02, S01, S11, S12, S02, S12, S22};

    /* Jacobian of the perspective projection at the camera-space mean, times the
     * world->camera rotation: T = J W (2x3) */
    float j00 = fx * iz;
    float j11 = fy * iz;
    float j02 = -(j00 * (tx * iz));
    float j12 = -(j11 * (ty * iz));
    float T0[3], T1[3];
    for (int k = 0; k < 3; ++k) {
        T0[k] = fmaf(j00, R[k], j02 * R[6 + k]);
        T1[k] = fmaf(j11, R[3 + k], j12 * R[6 + k]);
    }
    /* U = T Sigma; Sigma' = U T^T + 0.3 I */
    float U0[3], U1[3];
    for (int k = 0; k < 3; ++k) {
        U0[k] = fmaf(T0[0], S[k], fmaf(T0[1], S[3 + k], T0[2] * S[6 + k]));
        U1[k] = fmaf(T1[0], S[k], fmaf(T1[1], S[3 + k], T1[2] * S[6 + k]));
    }
    float a = fmaf(U0[0], T0[0], fmaf(U0[1], T0[1], U0[2] * T0[2])) + 0.3f;
    float b = fmaf(U0[0], T1[0], fmaf(U0[1], T1[1], U0[2] * T1[2]));
    float c = fmaf(U1[0], T1[0], fmaf(U1[1], T1[1], U1[2] * T1[2])) + 0.3f;

    float det = fmaf(a, c, -(b * b));
    if (!(det > 0.0f)) return;
    float idet = 1.0f / det;
    g->ca = c * idet;
    g->cb = -(b * idet);
    g->cc = a * idet;

    /* opacity thresholds in the power domain */
    float lc = -ora_ln32(255.0f * o);
    const float cut = (lc > -4.5f) ? lc : -4.5f;

    /* footprint: per-axis half-extents of the cut ellipse {d : -0.5 d^T conic d >= cut}, i.e.
     * sqrt(-2 cut Sigma'_xx) and sqrt(-2 cut Sigma'_yy), rounded up to whole pixels */
    float nc = -2.0f * cut;
    float rx = ceilf(sqrtf(nc * a));
    float ry = ceilf(sqrtf(nc * c));
    g->radius = rx > ry ? rx : ry;

    /* inclusive pixel box of [mx - rx, mx + rx] x [my - ry, my + ry], clipped to the image */
    float x0 = floorf(mx - rx), x1 = floorf(mx + rx);
    float y0 = floorf(my - ry), y1 = floorf(my + ry);
    float wmax = (float)(W - 1), hmax = (float)(H - 1);
    if (x0 < 0.0f) x0 = 0.0f;
    if (y0 < 0.0f) y0 = 0.0f;
    if (x1 > wmax) x1 = wmax;
    if (y1 > hmax) y1 = hmax;
    if (!(x0 <= x1) || !(y0 <= y1)) return;
    g->x0 = (int32_t)x0;
    g->x1 = (int32_t)x1;
    g->y0 = (int32_t)y0;
    g->y1 = (int32_t)y1;

    g->cut = cut;
    g->hi = ora_ln32(0.99f / o);
    g->participates = 1;
}
