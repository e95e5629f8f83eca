/*
 * CPU oracle for the multi-view differentiable Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference that the
 * GPU path is checked against. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does. It
 * shares no code, header, table or constant with the GPU library.
 *
 * What it computes (paper: "Efficient multi-view training for 3D Gaussian
 * Splatting"):
 *   - Sec. 3 (Preliminary): covariance Sigma = R S S^T R^T, EWA projection to a
 *     2D mean and covariance, Eq. 1 front-to-back alpha compositing over the
 *     depth-sorted Gaussians responsible for a pixel.
 *   - Appendix "Rasterization in multi-view training": per-view participation,
 *     duplication per covered tile, (view, tile, depth) keys, one list per
 *     (view, tile).
 *   - Sec. 3 / Sec. 5.1.2 (Eqs. 7-10): L1 and D-SSIM losses.
 *   - Sec. 5.2 (Eqs. 13-14): per-view screen-space error metrics E1 and E2.
 * All continuous arithmetic is double precision. The binning decisions (who
 * participates, tile rectangles, sort keys) are taken in single precision by a
 * fixed operation sequence (ora_geom32.c) because the kernel takes them in
 * single precision and binning is compared bit for bit. The per-pixel cut,
 * clamp and stop tests are taken in double precision; a pixel where one of them
 * lies within the kernel's single-precision error of its threshold is flagged
 * (and excluded from the comparison). The readings behind every constant are
 * listed in the project's design notes.
 *
 * Parity status: every function here is pinned by CPU tests (closed forms,
 * brute force, invariants, finite differences, the paper's cross-view example),
 * except the constants 0.2 (near plane), 0.3 (dilation), 1/255, 0.99 and 1e-4,
 * which the paper does not state: parity unpinned for those constants.
 */
#ifndef ORA_H
#define ORA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Camera batch. View v: wh[2v]=W, wh[2v+1]=H; intr[4v..4v+3]=fx,fy,cx,cy (pixels);
 * R[9v..] row-major world->camera rotation, t[3v..] translation (x_c = R x_w + t);
 * bg[3v..] background colour. Tiles are tile_w x tile_h pixels. */
typedef struct {
    int32_t B;
    int32_t tile_w, tile_h;
    const int32_t* wh;
    const double* intr;
    const double* R;
    const double* t;
    const double* bg;
} ora_cams;

/* Gaussians, double precision, activated: means [P,3], scales [P,3] (>0),
 * quats [P,4] (w,x,y,z; normalised inside), opac [P], sh [P,(d+1)^2,3]. */
typedef struct {
    int64_t P;
    int32_t sh_degree;
    const double* means;
    const double* scales;
    const double* quats;
    const double* opac;
    const double* sh;
} ora_scene;

/* Single-precision decision geometry of one (view, Gaussian). */
typedef struct {
    int32_t participates;
    float depth;            /* camera-space z */
    uint32_t depth_bits;    /* IEEE bits of depth (monotone for depth > 0) */
    float mx, my;           /* projected mean, pixels */
    float ca, cb, cc;       /* conic = inverse dilated 2D covariance, [[ca,cb],[cb,cc]] */
    float cut;              /* single-precision cut threshold, max(-4.5, -ln(255 o)): sizes the footprint */
    float hi;               /* ln(0.99 / o) in single precision (reported only) */
    float radius;
    int32_t x0, x1, y0, y1; /* inclusive pixel box, clipped to the image */
} ora_g32;

/* ora_geom32.c */
float ora_ln32(float x);
void ora_geom32_eval(const float mu[3], const float s[3], const float q[4], float o,
                     const float R[9], const float t[3], float fx, float fy, float cx, float cy,
                     int32_t W, int32_t H, ora_g32* out);

/* ora_sh.c */
int ora_sh_count(int degree);
void ora_sh_basis(int degree, const double d[3], double* Y, double* dY /* [K][3] or NULL */);

/* ora_raster.c */
int64_t ora_total_tiles(const ora_cams* c);
int ora_geom32_view(const ora_scene* s, const ora_cams* c, int32_t v, ora_g32* out /* [P] */);
int64_t ora_binning(const ora_scene* s, const ora_cams* c, uint64_t* keys, uint32_t* vals,
                    int64_t cap, uint32_t* ranges /* [2*total_tiles] or NULL */);
/* depth: per view [H,W], the camera-space depth blended with the colour weights,
 * sum_i z_i alpha_i T_i (may be NULL) */
int ora_forward(const ora_scene* s, const ora_cams* c, int32_t geom32_mode, int32_t brute_force,
                double margin, double* const* images, double* const* t_final, double* const* depth,
                int32_t* const* n_contrib, uint8_t* const* flags, uint64_t* trace_hash /* [B] or NULL */);
int ora_backward(const ora_scene* s, const ora_cams* c, int32_t geom32_mode,
                 const double* const* dl_dimg, double* g_means, double* g_scales, double* g_quats,
                 double* g_opac, double* g_sh, double* e1, double* e2, int32_t* count,
                 double* g_mean2d /* [B][P][2] or NULL */, double* e_old /* [P] or NULL */);
int ora_render_pixels(const ora_scene* s, const ora_cams* c, int32_t v, int32_t geom32_mode, double margin,
                      int64_t n, const int32_t* xs, const int32_t* ys, double* rgb, double* t_final, double* depth,
                      uint8_t* flags);
int ora_count_pairs(const ora_scene* s, const ora_cams* c, int64_t* records, int64_t* pairs);
int ora_project64(const ora_scene* s, const ora_cams* c, int32_t v, double* mean2d, double* cov2d,
                  double* rgb, double* depth);
void ora_set_threads(int32_t n);
int32_t ora_max_threads(void);

/* ora_loss.c */
int ora_loss(const ora_cams* c, const double* const* img, const double* const* tgt, double w_l1,
             double w_dssim, double* loss, double* const* dl_dimg);
int ora_ssim_map(int32_t W, int32_t H, const double* a, const double* b, double* out);

#ifdef __cplusplus
}
#endif
#endif
