/*
 * Multi-view Gaussian rasterizer, forward and backward, plain double precision.
 * TEST INFRASTRUCTURE ONLY (see ora.h).
 *
 * Forward (paper Sec. 3, Eq. 1; Appendix "Rasterization in multi-view training"):
 *   per view v and Gaussian g: camera transform, EWA projection of the mean and
 *   of Sigma = R S S^T R^T to mu' and Sigma' (+0.3 px^2 dilation), conic =
 *   Sigma'^{-1}, colour from real SH (+0.5, clamped at 0), participation and
 *   tile rectangle (single-precision decision geometry, ora_geom32.c);
 *   per (view, tile): the participating Gaussians whose rectangle covers the
 *   tile, sorted by the 64-bit key view<<48 | tile<<32 | depth bits, ties by g;
 *   per pixel: front-to-back over its tile's list, C = sum c_i alpha_i T_i,
 *   T_i = prod_{k<i} (1 - alpha_k), alpha_i = o_i exp(power_i) (0.99 when
 *   clamped), skipping Gaussians that fail the cut test, stopping before T
 *   would fall below 1e-4; output C + T_final * bg.
 * Backward: the chain rule of the above, walked back to front per pixel
 * (dC/dalpha_i = T_i (c_i - R_i), R_i = colour behind i normalised by T_{i+1}),
 * then through conic -> Sigma' -> (J, Sigma) -> camera-space mean, quaternion,
 * scale, SH, summed over views.
 * Densification statistics (Sec. 5.2, Eqs. 12-14), with positional gradients in
 * each view's normalised device coordinates (pixel gradient times (W/2, H/2)):
 *   E1 += sum_v sum_{p in v} || dL_p / d mu'_ndc ||,
 *   E2 += sum_v || sum_{p in v} dL_p / d mu'_ndc ||,
 *   count += number of views the Gaussian takes part in,
 *   E_old (comparator only) = || sum_v sum_p dL_p / d mu'_ndc ||.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "ora.h"

#define T_STOP 1e-4
#define ALPHA_CLAMP 0.99
#define DILATION 0.3

/* ------------------------------------------------------------------------- */
/* camera helpers                                                            */
/* ------------------------------------------------------------------------- */

static int cam_w(const ora_cams* c, int v) { return c->wh[2 * v]; }
static int cam_h(const ora_cams* c, int v) { return c->wh[2 * v + 1]; }
static int tiles_x(const ora_cams* c, int v) { return (cam_w(c, v) + c->tile_w - 1) / c->tile_w; }
static int tiles_y(const ora_cams* c, int v) { return (cam_h(c, v) + c->tile_h - 1) / c->tile_h; }

int64_t ora_total_tiles(const ora_cams* c)
{
    int64_t n = 0;
    for (int v = 0; v < c->B; ++v) n += (int64_t)tiles_x(c, v) * tiles_y(c, v);
    return n;
}

static int64_t tile_base(const ora_cams* c, int v)
{
    int64_t n = 0;
    for (int u = 0; u < v; ++u) n += (int64_t)tiles_x(c, u) * tiles_y(c, u);
    return n;
}

static void geom32_one(const ora_scene* s, const ora_cams* c, int v, int64_t g, ora_g32* out)
{
    float mu[3], sc[3], q[4], R[9], t[3];
    for (int k = 0; k < 3; ++k) {
        mu[k] = (float)s->means[3 * g + k];
        sc[k] = (float)s->scales[3 * g + k];
        t[k] = (float)c->t[3 * v + k];
    }
    for (int k = 0; k < 4; ++k) q[k] = (float)s->quats[4 * g + k];
    for (int k = 0; k < 9; ++k) R[k] = (float)c->R[9 * v + k];
    const double* in = c->intr + 4 * v;
    ora_geom32_eval(mu, sc, q, (float)s->opac[g], R, t, (float)in[0], (float)in[1], (float)in[2],
                    (float)in[3], cam_w(c, v), cam_h(c, v), out);
}

int ora_geom32_view(const ora_scene* s, const ora_cams* c, int32_t v, ora_g32* out)
{
    if (v < 0 || v >= c->B) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < s->P; ++g) geom32_one(s, c, v, g, &out[g]);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* double-precision projection                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    double tc[3];
    double mean2d[2];
    double qn[4], qlen;
    double rot[9], M[9], Sig[9];
    double J[6], T[6];
    double cov2d[3];
    double conic[3];
    double dir[3], dlen;
    double rgb_raw[3], rgb[3];
} proj64;

static void project64_one(const ora_scene* s, const ora_cams* c, int v, int64_t g, proj64* p)
{
    const double* R = c->R + 9 * v;
    const double* t = c->t + 3 * v;
    const double fx = c->intr[4 * v], fy = c->intr[4 * v + 1];
    const double cx = c->intr[4 * v + 2], cy = c->intr[4 * v + 3];
    const double* mu = s->means + 3 * g;
    for (int i = 0; i < 3; ++i) p->tc[i] = R[3 * i] * mu[0] + R[3 * i + 1] * mu[1] + R[3 * i + 2] * mu[2] + t[i];
    const double x = p->tc[0], y = p->tc[1], z = p->tc[2];
    p->mean2d[0] = fx * x / z + cx;
    p->mean2d[1] = fy * y / z + cy;

    const double* q = s->quats + 4 * g;
    p->qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) p->qn[k] = q[k] / p->qlen;
    const double w = p->qn[0], qx = p->qn[1], qy = p->qn[2], qz = p->qn[3];
    double* r = p->rot;
    r[0] = 1 - 2 * (qy * qy + qz * qz);
    r[1] = 2 * (qx * qy - w * qz);
    r[2] = 2 * (qx * qz + w * qy);
    r[3] = 2 * (qx * qy + w * qz);
    r[4] = 1 - 2 * (qx * qx + qz * qz);
    r[5] = 2 * (qy * qz - w * qx);
    r[6] = 2 * (qx * qz - w * qy);
    r[7] = 2 * (qy * qz + w * qx);
    r[8] = 1 - 2 * (qx * qx + qy * qy);
    const double* sc = s->scales + 3 * g;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) p->M[3 * i + j] = r[3 * i + j] * sc[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k) a += p->M[3 * i + k] * p->M[3 * j + k];
            p->Sig[3 * i + j] = a;
        }
    /* J = d mu' / d tc */
    p->J[0] = fx / z; p->J[1] = 0.0; p->J[2] = -fx * x / (z * z);
    p->J[3] = 0.0; p->J[4] = fy / z; p->J[5] = -fy * y / (z * z);
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k) {
            double a = 0;
            for (int m = 0; m < 3; ++m) a += p->J[3 * i + m] * R[3 * m + k];
            p->T[3 * i + k] = a;
        }
    double C2[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double a = 0;
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 3; ++m) a += p->T[3 * i + k] * p->Sig[3 * k + m] * p->T[3 * j + m];
            C2[2 * i + j] = a;
        }
    p->cov2d[0] = C2[0] + DILATION;
    p->cov2d[1] = C2[1];
    p->cov2d[2] = C2[3] + DILATION;
    const double det = p->cov2d[0] * p->cov2d[2] - p->cov2d[1] * p->cov2d[1];
    p->conic[0] = p->cov2d[2] / det;
    p->conic[1] = -p->cov2d[1] / det;
    p->conic[2] = p->cov2d[0] / det;

    /* colour: SH on the unit direction from the camera centre (-R^T t) to the mean */
    double cc[3];
    for (int i = 0; i < 3; ++i) cc[i] = -(R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
    double dv[3] = {mu[0] - cc[0], mu[1] - cc[1], mu[2] - cc[2]};
    p->dlen = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int i = 0; i < 3; ++i) p->dir[i] = dv[i] / p->dlen;
    const int K = ora_sh_count(s->sh_degree);
    double Y[64];
    ora_sh_basis(s->sh_degree, p->dir, Y, NULL);
    const double* sh = s->sh + (int64_t)K * 3 * g;
    for (int ch = 0; ch < 3; ++ch) {
        double a = 0.5;
        for (int k = 0; k < K; ++k) a += sh[3 * k + ch] * Y[k];
        p->rgb_raw[ch] = a;
        p->rgb[ch] = a > 0 ? a : 0.0;
    }
}

int ora_project64(const ora_scene* s, const ora_cams* c, int32_t v, double* mean2d, double* cov2d,
                  double* rgb, double* depth)
{
    if (v < 0 || v >= c->B) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < s->P; ++g) {
        proj64 p;
        project64_one(s, c, v, g, &p);
        if (mean2d) { mean2d[2 * g] = p.mean2d[0]; mean2d[2 * g + 1] = p.mean2d[1]; }
        if (cov2d) for (int k = 0; k < 3; ++k) cov2d[3 * g + k] = p.cov2d[k];
        if (rgb) for (int k = 0; k < 3; ++k) rgb[3 * g + k] = p.rgb[k];
        if (depth) depth[g] = p.tc[2];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* binning: duplicate per covered tile, sort by (tile, depth bits, g)        */
/* ------------------------------------------------------------------------- */

typedef struct {
    uint64_t key; /* view<<48 | tile<<32 | depth bits */
    uint32_t g;
} ora_pair;

static int pair_cmp(const void* a, const void* b)
{
    const ora_pair* x = (const ora_pair*)a;
    const ora_pair* y = (const ora_pair*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->g != y->g) return x->g < y->g ? -1 : 1;
    return 0;
}

typedef struct {
    ora_pair* pairs;
    int64_t n;
    uint32_t* start; /* per local tile */
    uint32_t* end;
} view_bins;

static void bin_view(const ora_cams* c, int v, const ora_g32* g32, int64_t P, view_bins* vb)
{
    const int tx_n = tiles_x(c, v), ty_n = tiles_y(c, v);
    int64_t n = 0;
    for (int64_t g = 0; g < P; ++g) {
        const ora_g32* q = &g32[g];
        if (!q->participates) continue;
        n += (int64_t)(q->x1 / c->tile_w - q->x0 / c->tile_w + 1) * (q->y1 / c->tile_h - q->y0 / c->tile_h + 1);
    }
    vb->pairs = (ora_pair*)malloc(sizeof(ora_pair) * (size_t)(n > 0 ? n : 1));
    vb->n = n;
    int64_t k = 0;
    for (int64_t g = 0; g < P; ++g) {
        const ora_g32* q = &g32[g];
        if (!q->participates) continue;
        for (int ty = q->y0 / c->tile_h; ty <= q->y1 / c->tile_h; ++ty)
            for (int tx = q->x0 / c->tile_w; tx <= q->x1 / c->tile_w; ++tx) {
                uint64_t tile = (uint64_t)ty * tx_n + tx;
                vb->pairs[k].key = ((uint64_t)v << 48) | (tile << 32) | q->depth_bits;
                vb->pairs[k].g = (uint32_t)g;
                ++k;
            }
    }
    qsort(vb->pairs, (size_t)n, sizeof(ora_pair), pair_cmp);
    const int64_t nt = (int64_t)tx_n * ty_n;
    vb->start = (uint32_t*)calloc((size_t)nt, sizeof(uint32_t));
    vb->end = (uint32_t*)calloc((size_t)nt, sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t tile = (vb->pairs[i].key >> 32) & 0xffffu;
        if (i == 0 || ((vb->pairs[i - 1].key >> 32) & 0xffffu) != tile) vb->start[tile] = (uint32_t)i;
        if (i == n - 1 || ((vb->pairs[i + 1].key >> 32) & 0xffffu) != tile) vb->end[tile] = (uint32_t)(i + 1);
    }
}

static void free_bins(view_bins* vb)
{
    free(vb->pairs);
    free(vb->start);
    free(vb->end);
}

int64_t ora_binning(const ora_scene* s, const ora_cams* c, uint64_t* keys, uint32_t* vals, int64_t cap,
                    uint32_t* ranges)
{
    ora_g32* g32 = (ora_g32*)malloc(sizeof(ora_g32) * (size_t)(s->P > 0 ? s->P : 1));
    int64_t total = 0;
    for (int v = 0; v < c->B; ++v) {
        ora_geom32_view(s, c, v, g32);
        view_bins vb;
        bin_view(c, v, g32, s->P, &vb);
        if (keys && vals) {
            for (int64_t i = 0; i < vb.n && total + i < cap; ++i) {
                keys[total + i] = vb.pairs[i].key;
                vals[total + i] = vb.pairs[i].g;
            }
        }
        if (ranges) {
            const int64_t base = tile_base(c, v);
            const int64_t nt = (int64_t)tiles_x(c, v) * tiles_y(c, v);
            for (int64_t tl = 0; tl < nt; ++tl) {
                uint32_t a = vb.start[tl], b = vb.end[tl];
                if (b == 0) a = 0;
                ranges[2 * (base + tl)] = (uint32_t)(a + (b ? total : 0));
                ranges[2 * (base + tl) + 1] = (uint32_t)(b ? b + total : 0);
            }
        }
        total += vb.n;
        free_bins(&vb);
    }
    free(g32);
    return total;
}

/* ------------------------------------------------------------------------- */
/* forward                                                                   */
/* ------------------------------------------------------------------------- */

/* What the pixel loop needs per Gaussian of one view: the geometry the walk decides and blends
 * with (double projection, or the single-precision values in image-parity mode), and in double
 * mode also the single-precision mean and conic, used only to size the flag margin. */
typedef struct {
    double mx, my, ca, cb, cc, o, rgb[3];
    double z; /* camera-space depth */
    double cut, hi; /* keep a pixel iff power >= cut; alpha clamped to 0.99 iff power > hi */
    double cut_err; /* the kernel's error in cut: 0 when cut is the exact -4.5, else POW_LN */
    double mx32, my32, ca32, cb32, cc32;
    int clamp_bits;
} pix_g;

/* Decision margins. The kernel decides the cut test from a single-precision power and threshold
 * (both may carry one more rounding from a change of the logarithm's base), the clamp from the
 * single-precision product o exp(power) against 0.99, and the stop test on its single-precision
 * transmittance. The oracle decides in double and flags a pixel where a decision it takes lies
 * within the kernel's possible error of the threshold:
 *   power:      POW_REL * (|a dx^2|/2 + |b dx dy| + |c dy^2|/2), i.e. 16 single-precision
 *               roundings of the power's terms (an evaluation in any order of its ~8 operations
 *               rounds each term at most ~6 times), plus POW_LN where the threshold is a
 *               logarithm (twice the error of the kernel's single-precision logarithm, which is
 *               within 2e-6 of ln; the cut -4.5 itself is exact) and for the clamp (an
 *               exponential and a product in single precision: a few 1e-7 of power);
 *   double mode: plus the power's change between the double and the single-precision projected
 *               geometry at this pixel (the kernel's power is within the first margin of the
 *               power of its single-precision geometry, which is within this change of the
 *               double power);
 *   stop:       `margin` relative to the 1e-4 threshold (plus, in double mode, the change of the
 *               new transmittance between the two geometries). */
#define POW_REL 9.5367431640625e-07 /* 2^-20 */
#define POW_LN 4e-6

static uint64_t mix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

static void prepare_view(const ora_scene* s, const ora_cams* c, int v, int geom32_mode, ora_g32* g32, pix_g* pg)
{
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < s->P; ++g) {
        geom32_one(s, c, v, g, &g32[g]);
        if (!g32[g].participates) continue;
        proj64 p;
        project64_one(s, c, v, g, &p);
        pix_g* q = &pg[g];
        q->mx32 = g32[g].mx; q->my32 = g32[g].my;
        q->ca32 = g32[g].ca; q->cb32 = g32[g].cb; q->cc32 = g32[g].cc;
        if (geom32_mode) {
            q->mx = q->mx32; q->my = q->my32;
            q->ca = q->ca32; q->cb = q->cb32; q->cc = q->cc32;
            q->z = g32[g].depth;
        } else {
            q->mx = p.mean2d[0]; q->my = p.mean2d[1];
            q->ca = p.conic[0]; q->cb = p.conic[1]; q->cc = p.conic[2];
            q->z = p.tc[2];
        }
        q->o = s->opac[g];
        /* alpha >= 1/255 <=> power >= -ln(255 o); inside the 3-sigma ellipse <=> power >= -4.5 */
        const double lc = -log(255.0 * q->o);
        q->cut = lc > -4.5 ? lc : -4.5;
        q->cut_err = lc > -4.5 ? POW_LN : 0.0;
        q->hi = log(ALPHA_CLAMP / q->o);
        q->clamp_bits = 0;
        for (int k = 0; k < 3; ++k) {
            q->rgb[k] = p.rgb[k];
            if (!(p.rgb_raw[k] > 0)) q->clamp_bits |= 1 << k;
        }
    }
}

/* One step of the front-to-back walk. Returns 0 = skipped by the cut test, 1 = blended,
 * 2 = stop (this Gaussian would drop T below the threshold; not blended). */
typedef struct {
    double alpha, G, T; /* alpha, exp(power), transmittance before this Gaussian */
    double alpha_alt;   /* double mode: alpha from the single-precision geometry */
    int clamped;
    double dx, dy;
} step_info;

/* Flag bits of a pixel: 1 = the stop test, 2 = a cut or clamp test lies within its margin. */
static int walk_step(const pix_g* q, int x, int y, double T, double T_alt, int alt, double margin, int* flag,
                     step_info* st)
{
    const double dx = (x + 0.5) - q->mx, dy = (y + 0.5) - q->my;
    const double ta = q->ca * dx * dx, tb = q->cb * dx * dy, tc = q->cc * dy * dy;
    const double power = -0.5 * (ta + tc) - tb;
    double m = POW_REL * (0.5 * fabs(ta) + fabs(tb) + 0.5 * fabs(tc));
    double p_alt = power;
    if (alt) {
        const double ex = (x + 0.5) - q->mx32, ey = (y + 0.5) - q->my32;
        p_alt = -0.5 * (q->ca32 * ex * ex + q->cc32 * ey * ey) - q->cb32 * ex * ey;
        m += fabs(p_alt - power);
    }
    if (fabs(power - q->cut) <= m + q->cut_err) *flag |= 2;
    if (!(power >= q->cut)) return 0;
    if (fabs(power - q->hi) <= m + POW_LN) *flag |= 2;
    const double G = exp(power);
    const int clamped = power > q->hi;
    const double alpha = clamped ? ALPHA_CLAMP : q->o * G;
    const double Tn = T * (1.0 - alpha);
    double mt = margin * T_STOP;
    st->alpha_alt = alpha;
    if (alt) {
        st->alpha_alt = clamped ? ALPHA_CLAMP : q->o * exp(p_alt);
        mt += fabs(T_alt * (1.0 - st->alpha_alt) - Tn);
    }
    if (fabs(Tn - T_STOP) <= mt) *flag |= 1;
    st->alpha = alpha;
    st->G = G;
    st->T = T;
    st->clamped = clamped;
    st->dx = dx;
    st->dy = dy;
    if (Tn < T_STOP) return 2;
    return 1;
}

/* per-view list of participating Gaussians in (depth bits, g) order, for the brute-force path */
static uint32_t* depth_order(const ora_g32* g32, int64_t P, int64_t* n_out)
{
    int64_t n = 0;
    for (int64_t g = 0; g < P; ++g) n += g32[g].participates;
    ora_pair* tmp = (ora_pair*)malloc(sizeof(ora_pair) * (size_t)(n > 0 ? n : 1));
    int64_t k = 0;
    for (int64_t g = 0; g < P; ++g)
        if (g32[g].participates) {
            tmp[k].key = g32[g].depth_bits;
            tmp[k].g = (uint32_t)g;
            ++k;
        }
    qsort(tmp, (size_t)n, sizeof(ora_pair), pair_cmp);
    uint32_t* out = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) out[i] = tmp[i].g;
    free(tmp);
    *n_out = n;
    return out;
}

int ora_forward(const ora_scene* s, const ora_cams* c, int32_t geom32_mode, int32_t brute_force, double margin,
                double* const* images, double* const* t_final, double* const* depth, int32_t* const* n_contrib,
                uint8_t* const* flags, uint64_t* trace_hash)
{
    const int64_t P = s->P;
    ora_g32* g32 = (ora_g32*)malloc(sizeof(ora_g32) * (size_t)(P > 0 ? P : 1));
    pix_g* pg = (pix_g*)malloc(sizeof(pix_g) * (size_t)(P > 0 ? P : 1));
    for (int v = 0; v < c->B; ++v) {
        const int W = cam_w(c, v), H = cam_h(c, v);
        const double* bg = c->bg + 3 * v;
        prepare_view(s, c, v, geom32_mode, g32, pg);
        view_bins vb = {0};
        uint32_t* order = NULL;
        int64_t n_order = 0;
        if (brute_force) order = depth_order(g32, P, &n_order);
        else bin_view(c, v, g32, P, &vb);
        const int txn = tiles_x(c, v);
        uint64_t hsum = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : hsum)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                const int64_t pix = (int64_t)y * W + x;
                double T = 1.0, T_alt = 1.0, C[3] = {0, 0, 0}, Dz = 0.0;
                int flag = 0, n = 0;
                uint64_t h = mix64((uint64_t)pix);
                const uint32_t* list;
                int64_t len;
                if (brute_force) {
                    list = order;
                    len = n_order;
                } else {
                    const int64_t tl = (int64_t)(y / c->tile_h) * txn + x / c->tile_w;
                    list = NULL;
                    len = vb.end[tl] ? (int64_t)vb.end[tl] - vb.start[tl] : 0;
                }
                const ora_pair* plist = NULL;
                if (!brute_force && len > 0)
                    plist = vb.pairs + vb.start[(int64_t)(y / c->tile_h) * txn + x / c->tile_w];
                for (int64_t i = 0; i < len; ++i) {
                    const uint32_t g = brute_force ? list[i] : plist[i].g;
                    step_info st;
                    int r = walk_step(&pg[g], x, y, T, T_alt, !geom32_mode, margin, &flag, &st);
                    if (r == 0) continue;
                    if (r == 2) {
                        h = mix64(h ^ 0xdeadull);
                        break;
                    }
                    for (int k = 0; k < 3; ++k) C[k] += pg[g].rgb[k] * st.alpha * T;
                    Dz += pg[g].z * st.alpha * T;
                    T = T * (1.0 - st.alpha);
                    T_alt = T_alt * (1.0 - st.alpha_alt);
                    ++n;
                    h = mix64(h ^ ((uint64_t)g << 2) ^ (uint64_t)st.clamped);
                }
                for (int k = 0; k < 3; ++k) images[v][(int64_t)k * H * W + pix] = C[k] + T * bg[k];
                if (t_final) t_final[v][pix] = T;
                if (depth) depth[v][pix] = Dz;
                if (n_contrib) n_contrib[v][pix] = n;
                if (flags) flags[v][pix] = (uint8_t)flag;
                hsum += h;
            }
        }
        if (trace_hash) {
            uint64_t h = hsum;
            for (int64_t g = 0; g < P; ++g)
                if (g32[g].participates) h += mix64(((uint64_t)g << 3) ^ (uint64_t)pg[g].clamp_bits ^ 0x5a5aull);
            trace_hash[v] = h;
        }
        if (brute_force) free(order);
        else free_bins(&vb);
    }
    free(g32);
    free(pg);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* backward                                                                  */
/* ------------------------------------------------------------------------- */

enum { A_MX, A_MY, A_CA, A_CB, A_CC, A_O, A_R, A_G, A_B, A_E1, A_N };

/* d rot_ij / d (w,x,y,z) for the rotation of a unit quaternion */
static void drot_dq(const double q[4], double d[9][4])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    double t[9][4] = {
        {0, 0, -4 * y, -4 * z},
        {-2 * z, 2 * y, 2 * x, -2 * w},
        {2 * y, 2 * z, 2 * w, 2 * x},
        {2 * z, 2 * y, 2 * x, 2 * w},
        {0, -4 * x, 0, -4 * z},
        {-2 * x, -2 * w, 2 * z, 2 * y},
        {-2 * y, 2 * z, -2 * w, 2 * x},
        {2 * x, 2 * w, 2 * z, 2 * y},
        {0, -4 * x, -4 * y, 0},
    };
    memcpy(d, t, sizeof(t));
}

int ora_backward(const ora_scene* s, const ora_cams* c, int32_t geom32_mode, const double* const* dl_dimg,
                 double* g_means, double* g_scales, double* g_quats, double* g_opac, double* g_sh, double* e1,
                 double* e2, int32_t* count, double* g_mean2d, double* e_old)
{
    const int64_t P = s->P;
    const int K = ora_sh_count(s->sh_degree);
    memset(g_means, 0, sizeof(double) * 3 * P);
    memset(g_scales, 0, sizeof(double) * 3 * P);
    memset(g_quats, 0, sizeof(double) * 4 * P);
    memset(g_opac, 0, sizeof(double) * P);
    memset(g_sh, 0, sizeof(double) * (size_t)K * 3 * P);
    double* eold_acc = NULL;
    if (e_old) eold_acc = (double*)calloc((size_t)(2 * P > 0 ? 2 * P : 1), sizeof(double));
    ora_g32* g32 = (ora_g32*)malloc(sizeof(ora_g32) * (size_t)(P > 0 ? P : 1));
    pix_g* pg = (pix_g*)malloc(sizeof(pix_g) * (size_t)(P > 0 ? P : 1));
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double* acc = (double*)malloc(sizeof(double) * A_N * (size_t)(P > 0 ? P : 1) * nthr);

    for (int v = 0; v < c->B; ++v) {
        const int W = cam_w(c, v), H = cam_h(c, v);
        const double* bg = c->bg + 3 * v;
        prepare_view(s, c, v, geom32_mode, g32, pg);
        view_bins vb;
        bin_view(c, v, g32, P, &vb);
        memset(acc, 0, sizeof(double) * A_N * (size_t)P * nthr);
        const int txn = tiles_x(c, v);
        const double* dimg = dl_dimg[v];
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            double* my = acc + (size_t)A_N * P * tid;
            int64_t cap = 256;
            uint32_t* gl = (uint32_t*)malloc(sizeof(uint32_t) * cap);
            step_info* sl = (step_info*)malloc(sizeof(step_info) * cap);
#pragma omp for schedule(dynamic, 4)
            for (int y = 0; y < H; ++y) {
                for (int x = 0; x < W; ++x) {
                    const int64_t pix = (int64_t)y * W + x;
                    const int64_t tl = (int64_t)(y / c->tile_h) * txn + x / c->tile_w;
                    const int64_t len = vb.end[tl] ? (int64_t)vb.end[tl] - vb.start[tl] : 0;
                    double T = 1.0;
                    int flag = 0;
                    int64_t n = 0;
                    for (int64_t i = 0; i < len; ++i) {
                        const uint32_t g = vb.pairs[vb.start[tl] + i].g;
                        step_info st;
                        int r = walk_step(&pg[g], x, y, T, T, 0, 0.0, &flag, &st);
                        if (r == 0) continue;
                        if (r == 2) break;
                        if (n == cap) {
                            cap *= 2;
                            gl = (uint32_t*)realloc(gl, sizeof(uint32_t) * cap);
                            sl = (step_info*)realloc(sl, sizeof(step_info) * cap);
                        }
                        gl[n] = g;
                        sl[n] = st;
                        ++n;
                        T = T * (1.0 - st.alpha);
                    }
                    const double dC[3] = {dimg[pix], dimg[(int64_t)H * W + pix], dimg[2 * (int64_t)H * W + pix]};
                    double Rb[3] = {bg[0], bg[1], bg[2]}; /* colour behind, normalised */
                    for (int64_t i = n - 1; i >= 0; --i) {
                        const uint32_t g = gl[i];
                        const step_info* st = &sl[i];
                        const pix_g* q = &pg[g];
                        double* a = my + (size_t)A_N * g;
                        double dalpha = 0.0;
                        for (int k = 0; k < 3; ++k) {
                            a[A_R + k] += dC[k] * st->alpha * st->T;
                            dalpha += dC[k] * st->T * (q->rgb[k] - Rb[k]);
                            Rb[k] = q->rgb[k] * st->alpha + (1.0 - st->alpha) * Rb[k];
                        }
                        if (st->clamped) continue;
                        a[A_O] += dalpha * st->G;
                        const double dpow = dalpha * st->alpha;
                        const double dx = st->dx, dy = st->dy;
                        /* power = -0.5 (ca dx^2 + 2 cb dx dy + cc dy^2), dx = px - mx */
                        const double gmx = dpow * (q->ca * dx + q->cb * dy);
                        const double gmy = dpow * (q->cb * dx + q->cc * dy);
                        a[A_MX] += gmx;
                        a[A_MY] += gmy;
                        a[A_CA] += dpow * (-0.5 * dx * dx);
                        a[A_CB] += dpow * (-dx * dy);
                        a[A_CC] += dpow * (-0.5 * dy * dy);
                        const double nx = gmx * 0.5 * W, ny = gmy * 0.5 * H;
                        a[A_E1] += sqrt(nx * nx + ny * ny);
                    }
                }
            }
            free(gl);
            free(sl);
        }
        /* reduce per-thread accumulators (fixed order) */
        for (int th = 1; th < nthr; ++th) {
            const double* src = acc + (size_t)A_N * P * th;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < (int64_t)A_N * P; ++i) acc[i] += src[i];
        }
        free_bins(&vb);

        /* chain to the Gaussian parameters */
        const double* R = c->R + 9 * v;
        const double fx = c->intr[4 * v], fy = c->intr[4 * v + 1];
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < P; ++g) {
            if (!g32[g].participates) continue;
            const double* a = acc + (size_t)A_N * g;
            proj64 p;
            project64_one(s, c, v, g, &p);
            /* statistics in NDC */
            const double nx = a[A_MX] * 0.5 * W, ny = a[A_MY] * 0.5 * H;
            if (e1) e1[g] += a[A_E1];
            if (e2) e2[g] += sqrt(nx * nx + ny * ny);
            if (count) count[g] += 1;
            if (eold_acc) { eold_acc[2 * g] += nx; eold_acc[2 * g + 1] += ny; }
            if (g_mean2d) {
                g_mean2d[((int64_t)v * P + g) * 2] = a[A_MX];
                g_mean2d[((int64_t)v * P + g) * 2 + 1] = a[A_MY];
            }
            g_opac[g] += a[A_O];

            double dtc[3] = {0, 0, 0};
            double dmu[3] = {0, 0, 0};
            const double x = p.tc[0], y = p.tc[1], z = p.tc[2];
            /* projected mean */
            dtc[0] += a[A_MX] * fx / z;
            dtc[1] += a[A_MY] * fy / z;
            dtc[2] += -a[A_MX] * fx * x / (z * z) - a[A_MY] * fy * y / (z * z);
            /* conic -> Sigma' : dL/dSigma' = -Q G Q, G = [[ga, gb/2],[gb/2, gc]] */
            const double Q[4] = {p.conic[0], p.conic[1], p.conic[1], p.conic[2]};
            const double Gq[4] = {a[A_CA], 0.5 * a[A_CB], 0.5 * a[A_CB], a[A_CC]};
            double QG[4], Gs[4];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) QG[2 * i + j] = Q[2 * i] * Gq[j] + Q[2 * i + 1] * Gq[2 + j];
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) Gs[2 * i + j] = -(QG[2 * i] * Q[j] + QG[2 * i + 1] * Q[2 + j]);
            /* Sigma' = T Sigma T^T + 0.3 I : dL/dT = 2 Gs T Sigma, dL/dSigma = T^T Gs T */
            double TS[6], dT[6], dSig[9];
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k) {
                    double s_ = 0;
                    for (int m = 0; m < 3; ++m) s_ += p.T[3 * i + m] * p.Sig[3 * m + k];
                    TS[3 * i + k] = s_;
                }
            for (int i = 0; i < 2; ++i)
                for (int k = 0; k < 3; ++k) dT[3 * i + k] = 2.0 * (Gs[2 * i] * TS[k] + Gs[2 * i + 1] * TS[3 + k]);
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 3; ++m) {
                    double s_ = 0;
                    for (int i = 0; i < 2; ++i)
                        for (int j = 0; j < 2; ++j) s_ += p.T[3 * i + k] * Gs[2 * i + j] * p.T[3 * j + m];
                    dSig[3 * k + m] = s_;
                }
            /* T = J W : dL/dJ = dL/dT W^T */
            double dJ[6];
            for (int i = 0; i < 2; ++i)
                for (int m = 0; m < 3; ++m) {
                    double s_ = 0;
                    for (int k = 0; k < 3; ++k) s_ += dT[3 * i + k] * R[3 * m + k];
                    dJ[3 * i + m] = s_;
                }
            /* J(tc) */
            dtc[0] += dJ[2] * (-fx / (z * z));
            dtc[1] += dJ[5] * (-fy / (z * z));
            dtc[2] += dJ[0] * (-fx / (z * z)) + dJ[2] * (2.0 * fx * x / (z * z * z)) + dJ[4] * (-fy / (z * z)) +
                      dJ[5] * (2.0 * fy * y / (z * z * z));
            /* tc = R mu + t */
            for (int k = 0; k < 3; ++k) dmu[k] += R[k] * dtc[0] + R[3 + k] * dtc[1] + R[6 + k] * dtc[2];
            /* Sigma = M M^T, M = rot diag(s) */
            double dM[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    double s_ = 0;
                    for (int k = 0; k < 3; ++k) s_ += (dSig[3 * i + k] + dSig[3 * k + i]) * p.M[3 * k + j];
                    dM[3 * i + j] = s_;
                }
            const double* sc = s->scales + 3 * g;
            double drot[9];
            for (int j = 0; j < 3; ++j) {
                double s_ = 0;
                for (int i = 0; i < 3; ++i) s_ += dM[3 * i + j] * p.rot[3 * i + j];
                g_scales[3 * g + j] += s_;
            }
            for (int i = 0; i < 9; ++i) drot[i] = dM[i] * sc[i % 3];
            double dr_dq[9][4];
            drot_dq(p.qn, dr_dq);
            double dqn[4] = {0, 0, 0, 0};
            for (int i = 0; i < 9; ++i)
                for (int k = 0; k < 4; ++k) dqn[k] += drot[i] * dr_dq[i][k];
            double qd = 0;
            for (int k = 0; k < 4; ++k) qd += p.qn[k] * dqn[k];
            for (int k = 0; k < 4; ++k) g_quats[4 * g + k] += (dqn[k] - p.qn[k] * qd) / p.qlen;
            /* colour */
            double Y[64], dY[192];
            ora_sh_basis(s->sh_degree, p.dir, Y, dY);
            double drgb[3];
            for (int k = 0; k < 3; ++k) drgb[k] = (p.rgb_raw[k] > 0) ? a[A_R + k] : 0.0;
            const double* sh = s->sh + (int64_t)K * 3 * g;
            double dd[3] = {0, 0, 0};
            for (int k = 0; k < K; ++k)
                for (int ch = 0; ch < 3; ++ch) {
                    g_sh[((int64_t)K * g + k) * 3 + ch] += drgb[ch] * Y[k];
                    for (int i = 0; i < 3; ++i) dd[i] += drgb[ch] * sh[3 * k + ch] * dY[3 * k + i];
                }
            /* dir = (mu - c)/|mu - c| */
            double ddot = dd[0] * p.dir[0] + dd[1] * p.dir[1] + dd[2] * p.dir[2];
            for (int i = 0; i < 3; ++i) dmu[i] += (dd[i] - p.dir[i] * ddot) / p.dlen;
            for (int i = 0; i < 3; ++i) g_means[3 * g + i] += dmu[i];
        }
    }
    if (e_old) {
        for (int64_t g = 0; g < P; ++g)
            e_old[g] = sqrt(eold_acc[2 * g] * eold_acc[2 * g] + eold_acc[2 * g + 1] * eold_acc[2 * g + 1]);
        free(eold_acc);
    }
    free(acc);
    free(g32);
    free(pg);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* sampled pixels at any size                                                */
/* ------------------------------------------------------------------------- */

/* Colour, final transmittance and flags of n chosen pixels of view v, each by walking every
 * participating Gaussian of the view in (depth bits, g) order (no tiles), as the brute-force
 * path does; used where rendering the whole batch would take too long. */
int ora_render_pixels(const ora_scene* s, const ora_cams* c, int32_t v, int32_t geom32_mode, double margin,
                      int64_t n, const int32_t* xs, const int32_t* ys, double* rgb, double* t_final, double* depth,
                      uint8_t* flags)
{
    if (v < 0 || v >= c->B) return -1;
    const int64_t P = s->P;
    ora_g32* g32 = (ora_g32*)malloc(sizeof(ora_g32) * (size_t)(P > 0 ? P : 1));
    pix_g* pg = (pix_g*)malloc(sizeof(pix_g) * (size_t)(P > 0 ? P : 1));
    prepare_view(s, c, v, geom32_mode, g32, pg);
    int64_t n_order = 0;
    uint32_t* order = depth_order(g32, P, &n_order);
    const double* bg = c->bg + 3 * v;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n; ++k) {
        const int x = xs[k], y = ys[k];
        double T = 1.0, T_alt = 1.0, C[3] = {0, 0, 0}, Dz = 0.0;
        int flag = 0;
        for (int64_t i = 0; i < n_order; ++i) {
            const uint32_t g = order[i];
            step_info st;
            int r = walk_step(&pg[g], x, y, T, T_alt, !geom32_mode, margin, &flag, &st);
            if (r == 0) continue;
            if (r == 2) break;
            for (int q = 0; q < 3; ++q) C[q] += pg[g].rgb[q] * st.alpha * T;
            Dz += pg[g].z * st.alpha * T;
            T = T * (1.0 - st.alpha);
            T_alt = T_alt * (1.0 - st.alpha_alt);
        }
        for (int q = 0; q < 3; ++q) rgb[3 * k + q] = C[q] + T * bg[q];
        t_final[k] = T;
        if (depth) depth[k] = Dz;
        flags[k] = (uint8_t)flag;
    }
    free(order);
    free(g32);
    free(pg);
    return 0;
}

/* Number of (Gaussian, tile) pairs of every view and of participating (view, Gaussian) records,
 * counted from the decision geometry without sorting. */
int ora_count_pairs(const ora_scene* s, const ora_cams* c, int64_t* records, int64_t* pairs)
{
    ora_g32* g32 = (ora_g32*)malloc(sizeof(ora_g32) * (size_t)(s->P > 0 ? s->P : 1));
    int64_t nr = 0, np = 0;
    for (int v = 0; v < c->B; ++v) {
        ora_geom32_view(s, c, v, g32);
        for (int64_t g = 0; g < s->P; ++g) {
            const ora_g32* q = &g32[g];
            if (!q->participates) continue;
            nr += 1;
            np += (int64_t)(q->x1 / c->tile_w - q->x0 / c->tile_w + 1) * (q->y1 / c->tile_h - q->y0 / c->tile_h + 1);
        }
    }
    free(g32);
    *records = nr;
    *pairs = np;
    return 0;
}

/* Threads the oracle's parallel loops use (the CPU baseline times it on one thread too). */
void ora_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int32_t ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
