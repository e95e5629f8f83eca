/*
 * mvgs: multi-view differentiable Gaussian-splatting rasterizer for MI355X (gfx950).
 *
 * C ABI of libmvgs.so. Every call enqueues work on the caller's HIP stream and
 * returns without waiting, except where a call says it synchronizes. All
 * device buffers are owned by the caller unless stated otherwise; the library
 * owns its frames and workspace. Arguments are validated before any HIP call;
 * an invalid call returns MVGS_EINVAL and touches no device state.
 *
 * Paper: "Efficient multi-view training for 3D Gaussian Splatting".
 *   Sec. 3 (Preliminary): a Gaussian has mean mu, scale S, rotation R, colour c
 *     and opacity o; Sigma = R S S^T R^T is projected to a 2D mean mu' and
 *     covariance Sigma'; Eq. 1 alpha-composites the depth-sorted Gaussians
 *     responsible for each pixel; the rasterizer preprocesses (cull, project,
 *     organise) and renders tile by tile.
 *   Appendix "Rasterization in multi-view training": per-view participation is
 *     decided before memory is sized; projected Gaussians are duplicated per
 *     covered tile and sorted by a 64-bit key holding tile, view and depth; one
 *     block renders each (tile, view).
 *   Sec. 5.2, Eqs. 13-14: densification statistics accumulated per Gaussian
 *     from positional gradients taken in each view's own screen space.
 *
 * Conventions (the paper leaves them open): x_c = R x_w + t with camera axes
 * x right, y down, z forward; pixel (x, y) has its centre at (x+0.5, y+0.5);
 * parameters arrive activated (scales > 0, opacities in (0,1), quaternions
 * (w,x,y,z) of any non-zero length); colour is real spherical harmonics of
 * degree <= 3 on the direction camera centre -> mean, plus 0.5, clamped at 0;
 * near plane z > 0.2; +0.3 px^2 on the 2D covariance diagonal; a Gaussian
 * covers a pixel iff power >= max(-4.5, -ln(255 o)) (3-sigma ellipse and
 * alpha >= 1/255); alpha = min(0.99, o exp(power)); compositing stops before
 * the transmittance would fall below 1e-4; background added as T_final * bg.
 */
#ifndef MVGS_H
#define MVGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. 0 is success; failures are negative. */
#define MVGS_OK 0
#define MVGS_EINVAL (-1)    /* invalid argument; nothing was enqueued */
#define MVGS_ENOMEM (-2)    /* device or host allocation failed */
#define MVGS_ECAPACITY (-3) /* a size limit of the format was exceeded (see mvgs_forward) */
#define MVGS_EHIP (-4)      /* a HIP runtime call failed; mvgs_last_error has the text */
#define MVGS_ERETRY (-5)    /* capacity mode: the depth keys left the sort window; make the call again */

#define MVGS_MAX_VIEWS 65535
#define MVGS_MAX_TILES_PER_VIEW 65536

typedef struct mvgs_context mvgs_context;
typedef struct mvgs_frame mvgs_frame;

/* One pinhole camera (host memory). R row-major world->camera rotation, t its
 * translation, fx/fy/cx/cy in pixels, bg the background colour. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float bg[3];
} mvgs_camera;

/* Gaussian parameters, all float32 device pointers, row-major and contiguous:
 * means [P,3], scales [P,3], quats [P,4] (w,x,y,z), opacities [P],
 * sh [P,(sh_degree+1)^2,3] (coefficient-major, RGB innermost). */
typedef struct {
    int64_t P;
    int32_t sh_degree;
    const float* means;
    const float* scales;
    const float* quats;
    const float* opacities;
    const float* sh;
} mvgs_gaussians;

/* Parameter gradients (device, same shapes as mvgs_gaussians), overwritten. */
typedef struct {
    float* means;
    float* scales;
    float* quats;
    float* opacities;
    float* sh;
} mvgs_grads;

/* Densification statistics (device, [P] each), accumulated with +=:
 * e1 += sum_v sum_{p in v} ||dL_p/dmu'_ndc||, e2 += sum_v ||sum_{p in v} dL_p/dmu'_ndc||,
 * count += number of views the Gaussian took part in (Sec. 5.2, Eqs. 13-14; the
 * positional gradient is taken in normalised device coordinates, i.e. the pixel
 * gradient times (W/2, H/2)). */
typedef struct {
    float* e1;
    float* e2;
    int32_t* count;
} mvgs_densify;

/* Context options. tile_w, tile_h in {8, 16, 32} (0 selects 16). pixels_per_lane in {1, 2, 4}:
 * each lane of a blend wavefront owns that many pixels of its 8x8, 8x16 or 16x16 sub-tile; 2
 * needs tile_h >= 16, 4 needs tile_w and tile_h >= 16; 0 lets each forward choose: the largest
 * the tile allows that still launches 4096 blend wavefronts (small frames take fewer pixels per
 * lane and more wavefronts), the backward on its frame following it.
 * Results do not depend on these choices.
 * workspace_limit: 0 for none, else the most device bytes the context may hold (workspace,
 * upload staging and all its frames, as mvgs_memory_held counts them). A call that would grow
 * past it allocates nothing and returns MVGS_ECAPACITY; a serving loop admits work against an
 * HBM budget this way. Must be >= 0. reserved0 must be zero.
 * capacity_records, capacity_pairs: both 0 (sizes found per call: the forward synchronizes once),
 * or both in [1, 2^32): capacity mode. The forward then makes no host synchronization: buffers are
 * sized once by the capacities, every kernel reads the actual counts from device memory, and a
 * call whose participating (view, Gaussian) records or (Gaussian, tile) pairs exceed them does no
 * work (images get the background) and is reported by mvgs_frame_check. Such a forward, with the
 * loss and backward on its frame, can be captured into a HIP graph (the stream in capture mode),
 * after one call of each with the same shapes outside the capture. Partial rendering works in
 * capacity mode too: its selection kernels are then launched for the bound n_tiles + n_sel / 64 + 1
 * on tasks and read the count from device memory, and a rejected selection voids the call like an
 * overflow (mvgs_frame_check reports it); sub-sampling, merge and the 3D loss capture as well. */
typedef struct {
    int32_t tile_w;
    int32_t tile_h;
    int32_t pixels_per_lane;
    int32_t reserved0;
    int64_t workspace_limit;
    int64_t capacity_records;
    int64_t capacity_pairs;
    /* Device memory of the context's workspace and frames: both NULL for hipMalloc / hipFree, or
     * both set. alloc(bytes, alloc_ctx) returns at least `bytes` of device memory on the context's
     * device, aligned to 256 bytes, or NULL (the call then fails with MVGS_ENOMEM); free(ptr,
     * alloc_ctx) takes back a block alloc gave. The library calls them only from inside its own
     * calls, on the thread and during the call that grows, replaces or (mvgs_destroy, after it has
     * waited for the device) frees a buffer. free may be called while kernels that use the block
     * are still queued on that call's stream: the allocator must not hand the block to other work
     * before that work in stream order (a stream-ordered caching allocator, such as PyTorch's
     * with the call's stream current, does this). The dedicated upload staging of calls recorded
     * into a graph capture is allocated with hipMalloc / hipHostMalloc whatever these say. */
    void* (*alloc)(size_t bytes, void* alloc_ctx);
    void (*free)(void* ptr, void* alloc_ctx);
    void* alloc_ctx;
} mvgs_options;

/* Create a context on the current HIP device. `opt` may be NULL (defaults).
 * A context's workspace serves one stream at a time: calls on one context must
 * not overlap on different streams. Returns MVGS_EINVAL for a bad tile shape. */
int mvgs_create(mvgs_context** out, const mvgs_options* opt);

/* Destroy a context and every frame it still owns (waits for the device). */
void mvgs_destroy(mvgs_context* ctx);

/* Forward pass over a batch of B views (paper Sec. 3 and the multi-view
 * appendix): per-view participation and projection, duplication per covered
 * tile, sort by (view, tile, depth) with ties by Gaussian index, per-(view,
 * tile) ranges, and front-to-back blending of every pixel of every view in one
 * launch per stage.
 *   cams    host array of B cameras, 1 <= B <= 65535; each view at most
 *           65536 tiles; width, height >= 1; fx, fy > 0.
 *   images  host array of B device pointers; view v receives float32
 *           [3, height_v, width_v] (planar RGB).
 *   frame   receives a new frame that keeps what the backward needs (records,
 *           sorted lists, ranges, final transmittance, last contributor per
 *           pixel); release it with mvgs_frame_release.
 * Synchronizes the stream once to read the number of (Gaussian, tile) pairs,
 * which sizes the sort (not in capacity mode: see mvgs_options). Returns
 * MVGS_ECAPACITY if that number reaches 2^32 or the workspace would exceed the
 * context's limit (no frame is made then). */
int mvgs_forward(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams, int32_t B,
                 float* const* images, mvgs_frame** frame);

/* Participation pre-pass per view (the multi-view appendix decides which Gaussians take part in
 * each view before any per-record memory is sized): for each of the B views, the number of
 * participating Gaussians (its records) and of the (Gaussian, tile) pairs they cover with this
 * context's tile shape, exactly as a forward of these cameras would count them. records, pairs:
 * host arrays of B. Runs one kernel over the Gaussians on `stream` and synchronizes it (not
 * capturable). Counts of a batch are the sums of its views' counts. */
int mvgs_count_views(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams, int32_t B,
                     int64_t* records, int64_t* pairs);

/* Admission bound: the device bytes this context would hold (as mvgs_memory_held counts them)
 * after a forward of B views over P Gaussians whose participation pre-pass counted `records` and
 * `pairs` (summed over the views; mvgs_count_views), followed by the work in `work`:
 * MVGS_WORK_LOSS (mvgs_loss with w_dssim 0) or MVGS_WORK_LOSS_DSSIM (with D-SSIM), and
 * MVGS_WORK_BACKWARD (mvgs_backward on the frame). It replays the growth of every buffer those
 * calls would size, from the context's present buffers and frame pool, with the allocator's
 * growth rule; host only, no device work. So with a workspace limit of at least *bytes, these
 * calls, made next on this context with these cameras and Gaussians, are not refused. In capacity
 * mode records and pairs are the context's capacities. MVGS_EINVAL for counts no batch can have;
 * MVGS_ECAPACITY if records or pairs reach 2^32 (the forward would refuse them). */
#define MVGS_WORK_FORWARD 0
#define MVGS_WORK_LOSS 1
#define MVGS_WORK_LOSS_DSSIM 2
#define MVGS_WORK_BACKWARD 4
int mvgs_workspace_bound(mvgs_context* ctx, const mvgs_camera* cams, int32_t B, int64_t P, int64_t records,
                         int64_t pairs, int32_t work, int64_t* bytes);

/* Partial rendering (paper Sec. 5.1.1, "Thread-efficient partial rendering", and Alg. 3): each view
 * renders only a selection of its pixels, the paper's index array. The selection is given per
 * (view, tile) of the batch, in the order of the ranges (view-major; tiles of tile_w x tile_h of
 * this context, row-major):
 *   sel_offsets  device uint32 [n_tiles + 1], rising from 0 to n_sel; segment s of the selection is
 *                [sel_offsets[s], sel_offsets[s+1]), s = tile_base(v) + ty * tiles_x(v) + tx
 *   sel_pixels   device uint32 [n_sel], pixel indices y * width_v + x inside the segment's tile,
 *                each pixel at most once, in any order
 * Modes: MVGS_PARTIAL_COMPACT is the paper's thread-efficient scheme, one wavefront per 64 selected
 * pixels of a segment so that no lane idles; MVGS_PARTIAL_MASKED is its binary-mask baseline, the
 * full-tile launch with the lanes of unselected pixels idle. Both give bit-identical values, equal to
 * the full forward's at the selected pixels. Only selected pixels of images[v] are written (the
 * others keep their contents), so passing one buffer for all views of a sub-sampled batch yields
 * the merged image. The selection is copied into the frame and checked on the device before any
 * blending: a bad selection returns MVGS_EINVAL (after the stream synchronization the forward does
 * anyway). In capacity mode the forward does not synchronize: a bad selection (or more tasks than
 * their bound) makes the call do no work, and mvgs_frame_check returns MVGS_EINVAL for it; a
 * selection of exactly width * height pixels over views of one size is then taken as a partition
 * of the plane for mvgs_loss_3d, and mvgs_frame_check also returns MVGS_EINVAL if it selects a
 * plane position in two views. mvgs_backward on such a frame reads dL/dimage at the selected pixels only;
 * mvgs_export_transmittance writes the selected pixels only (masked mode: every pixel, 1 where
 * unselected). Otherwise as mvgs_forward. */
#define MVGS_PARTIAL_COMPACT 0
#define MVGS_PARTIAL_MASKED 1
int mvgs_forward_partial(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams,
                         int32_t B, const uint32_t* sel_offsets, const uint32_t* sel_pixels, int64_t n_sel,
                         int32_t mode, float* const* images, mvgs_frame** frame);

/* Pixel sub-sampling for partial rendering of B views of one size (paper Sec. 5.1.1: pixels of every
 * tile are sub-sampled per view): the positions of each tile (of this context's tile shape) are
 * ranked by keys[y * width + x] (device uint32 [height * width], random numbers drawn by the
 * caller), ties by position, and the position of rank r goes to view r mod B. The views thus share
 * every tile out evenly (ceil or floor of N/B pixels each) and together cover the image plane once.
 * Writes the selection in mvgs_forward_partial's format: sel_offsets [B * tiles + 1], sel_pixels
 * [height * width] (caller-owned device buffers), each segment in ascending pixel index (compact
 * bands per wavefront). MVGS_EINVAL if the views differ in size. */
int mvgs_subsample(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B, const uint32_t* keys,
                   uint32_t* sel_offsets, uint32_t* sel_pixels);

/* Photometric loss (paper Sec. 3; D-SSIM of Sec. 5.1.2, Eqs. 7-10):
 *   L = w_l1 * mean|I - T| + w_dssim * (1 - mean SSIM(I, T))
 * means over every (view, channel, row, column); SSIM with an 11x11 Gaussian
 * window (sigma 1.5, normalised to sum 1, zero outside the image), C1 = 0.01^2,
 * C2 = 0.03^2. Writes the scalar loss to loss_dev (device float) and dL/dI to
 * dl_dimages (B device pointers, [3,H,W] each; overwritten). images and
 * targets are B device pointers of the same shapes. */
int mvgs_loss(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B, const float* const* images,
              const float* const* targets, float w_l1, float w_dssim, float* loss_dev, float* const* dl_dimages);

/* Bytes of device scratch memory mvgs_loss_noalloc may use (per GPU). */
#define MVGS_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)

/* mvgs_loss for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and results (the
 * loss and dL/dI bit for bit mvgs_loss's), but every intermediate lives in a fixed
 * MVGS_NOALLOC_SCRATCH_BYTES array that the library holds on each GPU it runs on until the process
 * ends; the call allocates nothing, neither in the context nor on the host (no staging: the view
 * table is written by a kernel from its arguments). Limits: B <= 64 views, and the scratch must
 * hold the partial sums (1/256 byte per pixel with L1 only; 24 bytes per 32x32 tile with
 * D-SSIM, so about 1.4G pixels); beyond them the call returns MVGS_ECAPACITY and enqueues nothing. Every call on one GPU shares that GPU's array: calls that may
 * overlap on the device (other streams, other threads, other contexts) race and must be ordered by
 * the caller. The first call on a device looks the array up (no allocation). */
int mvgs_loss_noalloc(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B,
                      const float* const* images, const float* const* targets, float w_l1, float w_dssim,
                      float* loss_dev, float* const* dl_dimages);

/* L1 + 3D distance-aware D-SSIM (paper Sec. 5.1.2, Eqs. 7-11) on the merged image plane of a
 * thread-efficient partial frame whose selection covers the views' common image plane once (as
 * mvgs_subsample makes). Pixel (x, y) of the plane was rendered from one view; its surface point is
 * the blended depth over the blended opacity, zbar = D / (1 - T_final), along that view's camera
 * ray, in world space (no point where nothing was blended). The SSIM window (11 x 11) around each
 * centre weighs a neighbour by exp(-|P(q) - P(c)|^2 / (2 s_c^2)), s_c = 1.5 zbar_c / fx (1.5
 * pixels at the centre's depth), normalised over the in-plane window; a centre without a point
 * keeps only itself; the weights are constants of the loss (no gradient reaches the depth).
 *   L = w_l1 * mean|I - T| + w_dssim * (1 - mean SSIM*)   over (channel, row, column)
 * image, target: device [3, H, W] merged planes; writes the loss to loss_dev and dL/dI to
 * dl_dimage ([3, H, W], overwritten). Pass dl_dimage for every view to mvgs_backward. */
int mvgs_loss_3d(mvgs_context* ctx, void* stream, const mvgs_frame* frame, const float* image, const float* target,
                 float w_l1, float w_dssim, float* loss_dev, float* dl_dimage);

/* Test hook: the blended depth (sum of z alpha T over the blended Gaussians, z the camera-space
 * depth) of a thread-efficient partial frame's selected pixels into B device [H, W] planes (other
 * pixels untouched). */
int mvgs_export_depth(mvgs_context* ctx, void* stream, const mvgs_frame* frame, float* const* depth);

/* Multi-view adaptive density control (paper Sec. 5.2.2): per Gaussian, with the per-view mean
 * statistics m1 = e1 / count and m2 = e2 / count (0 where count is 0), compared in single precision:
 *   opacity < min_opacity                                 -> pruned (no output)
 *   largest scale > dense_scale and m1 > split_threshold  -> split into two children,
 *       means mu + R (s * z_k) (R the normalised quaternion's rotation, z_k = normals[6g + 3k ..]),
 *       scales s / 1.6, other parameters copied
 *   largest scale <= dense_scale and m2 > clone_threshold -> cloned (itself and an identical copy)
 *   otherwise                                             -> kept.
 * The paper splits on E1 and clones on E2 and scales the pruning threshold by the number of views
 * per batch (pass min_opacity already scaled). Outputs keep the originals' order, each original's
 * outputs in a row; src (device int32 [n_out], may be NULL) receives the original of each output,
 * to carry other per-Gaussian state along. normals: device float [P, 2, 3] standard normal draws
 * (the caller's random numbers). out: device buffers for `capacity` Gaussians (the input's SH
 * degree). Synchronizes the stream once to read n_out; MVGS_ECAPACITY (nothing written) if the
 * result exceeds capacity (2 P always suffices). */
typedef struct {
    float split_threshold;
    float clone_threshold;
    float dense_scale;
    float min_opacity;
} mvgs_adc_params;

typedef struct {
    float* means;
    float* scales;
    float* quats;
    float* opacities;
    float* sh;
} mvgs_gaussians_out;

int mvgs_adapt_density(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const float* e1, const float* e2,
                       const int32_t* count, const float* normals, const mvgs_adc_params* prm,
                       const mvgs_gaussians_out* out, int32_t* src, int64_t capacity, int64_t* n_out);

/* One Adam step (the optimiser 3DGS trains with) of the activated parameters, in place. Scales
 * and opacities move in their unconstrained coordinates, log-scale and opacity logit: their
 * gradients are taken through exp and the sigmoid and the step is applied as s * exp(-step) and
 * sigmoid(logit(o) - step) (opacities of exactly 0 or 1 stay). Per element, with the gradient g
 * in those coordinates: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * step = lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = prm->step >= 1.
 * params: device float, the layout of mvgs_gaussians. grads: the gradients mvgs_backward wrote
 * (statistics pointers unused). moments: device float [P, 11 + 3K, 2] (m, v interleaved; per
 * Gaussian the elements of means, scales, quats, opacity, SH in that order), zero before the
 * first step. The SH learning rate is lr_sh_dc for the first coefficient, lr_sh_rest for the
 * others. Launches one kernel, no synchronization (may be captured).
 * step_dev: NULL, or a device int32 step counter. Then t is read on the device: the call adds 1 to
 * *step_dev and takes the new value as t (prm->step is not used), so that a step captured into a
 * graph counts its own replays; one more small kernel runs first. skip_dev: NULL, or a device word
 * (with step_dev only): when it is non-zero at run time the call changes nothing, counter
 * included; pass the frame's void word (mvgs_frame_void_word) so that a captured training step
 * whose forward overflowed its capacities leaves the parameters alone. */
typedef struct {
    float lr_means, lr_scales, lr_quats, lr_opacities, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    int32_t step;
    int32_t* step_dev;
    const uint32_t* skip_dev;
} mvgs_adam_params;

int mvgs_adam_step(mvgs_context* ctx, void* stream, int64_t P, int32_t sh_degree, const mvgs_gaussians_out* params,
                   const mvgs_grads* grads, float* moments, const mvgs_adam_params* prm);

/* out[r, :] = in[src[r], :] for r < n over float rows of `width` (device): carries per-Gaussian
 * state such as the optimiser moments through mvgs_adapt_density's src map. in and out must not
 * overlap; src entries must index rows of in (not checked on the device). */
int mvgs_gather_rows(mvgs_context* ctx, void* stream, const int32_t* src, int64_t n, int64_t width, const float* in,
                     float* out);

/* Running moments of mini-batch gradients for the Monte Carlo variance estimate of Sec. 3.2 (the
 * mean squared norm minus the squared norm of the mean). The gradient vector is the
 * concatenation means | scales | quats | opacities | SH of one backward's grads (n = P (11 + 3K)
 * elements). Adds it to sum (device double [n]); adds its squared norm to acc[0] and sets acc[1]
 * (device double [2]) to the squared norm of the updated sum. After k calls:
 * variance = acc[0] / k - acc[1] / k^2. The sums are reduced in a fixed order (reproducible). No
 * synchronization; the first call on a context allocates 16 KiB of partial sums, so capture a
 * call only after one uncaptured call. */
int mvgs_grad_moments(mvgs_context* ctx, void* stream, int64_t P, int32_t sh_degree, const mvgs_grads* grads,
                      double* sum, double* acc);

/* Merges per-view planes into the image plane of a partial frame (Alg. 3: each pixel of the plane
 * belongs to the view that selected it), e.g. the views' targets into the target of the merged
 * render. planes: B device pointers to [channels, H, W] float (the views must share one size);
 * out: device [channels, H, W]; each selected pixel of view v takes planes[v]'s value there, other
 * pixels of out are left alone. MVGS_EINVAL for a full (unselected) frame. */
int mvgs_frame_merge(mvgs_context* ctx, void* stream, const mvgs_frame* frame, const float* const* planes,
                     int32_t channels, float* out);

/* Backward pass: from dL/dimage (B device pointers [3,H,W]) to parameter
 * gradients (overwritten) and, when `densify` is not NULL, the densification
 * statistics (accumulated). `g` must hold the same parameters the frame was
 * rendered from. Blend state is recomputed from the frame's final
 * transmittance and last contributor, not stored per pixel and Gaussian. */
int mvgs_backward(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_frame* frame,
                  const float* const* dl_dimages, mvgs_grads* grads, mvgs_densify* densify);

/* Return a frame's memory to its context. The frame must not be in use by
 * work still pending on a stream other than the one it was created on. The
 * handle is stale afterwards: every call given it returns MVGS_EINVAL, also
 * after a later forward reuses the pooled frame object (a handle carries the
 * object's 16-bit generation, which each release advances). Frames die with
 * their context. */
int mvgs_frame_release(mvgs_context* ctx, mvgs_frame* frame);

/* Capacity mode: wait for the frame's forward and report whether it fitted the capacities
 * (MVGS_ECAPACITY if not: its images and any backward on it are void; make a context with larger
 * capacities). The depth sort of a capacity-mode forward orders the window of depth keys (whole
 * 8-bit passes around them) that the last frame checked on this context had, or all 32 bits before
 * any check; a forward whose keys leave that window is void too: MVGS_ERETRY, and the check
 * moves the window to its keys, so the same call (or the same capture, with the same capacities)
 * made again succeeds. A partial frame is also void, with MVGS_EINVAL, if its selection was rejected; if
 * its width * height pixels select a plane position in two views, MVGS_EINVAL says that its 3D
 * loss and merge are void. Sets the sizes mvgs_frame_info and mvgs_export_binning use.
 * Synchronizes the stream; not capturable. Returns MVGS_OK at once for frames not made in
 * capacity mode. */
int mvgs_frame_check(mvgs_context* ctx, void* stream, mvgs_frame* frame);

/* Capacity mode: the device word (owned by the frame, valid while it is held) that is non-zero
 * once the frame's forward has run if the frame is void, for device-side decisions such as
 * mvgs_adam_params.skip_dev. *word = NULL for frames not made in capacity mode (their errors are
 * returned by the forward itself). */
int mvgs_frame_void_word(const mvgs_frame* frame, const uint32_t** word);

/* For a frame made by a forward captured into a graph: replace its cameras (same count and image
 * sizes; poses, intrinsics and background may change). Host-only: it rewrites the staging memory
 * the graph's upload node reads, so the next replay renders the new cameras. No replay that
 * reads this frame may be in flight. */
int mvgs_frame_set_cameras(mvgs_context* ctx, mvgs_frame* frame, const mvgs_camera* cams, int32_t B);

/* Change a context's workspace limit (bytes, 0 for none; see mvgs_options). Memory already held
 * is kept: the limit applies to later growth. No device work. */
int mvgs_set_workspace_limit(mvgs_context* ctx, int64_t bytes);

/* Device bytes the context holds now (workspace, staging, frames live or pooled). Host only. */
int mvgs_memory_held(mvgs_context* ctx, int64_t* bytes);

/* Device bytes the forward that made this frame asked for at exact sizes (its own buffers plus
 * the context workspace it used), without the growth slack of the context's allocator. */
int mvgs_frame_workspace(const mvgs_frame* frame, int64_t* bytes);

/* Sizes of a frame: participating (view, Gaussian) records, (Gaussian, tile)
 * pairs and tiles over all views. Any pointer may be NULL. */
int mvgs_frame_info(const mvgs_frame* frame, int64_t* n_records, int64_t* n_pairs, int64_t* n_tiles);

/* Radix passes the frame's forward ran (for rooflines): the depth sort of the records orders
 * only the bits in which their depth keys differ (ceil(bits / 8) passes of even width); the tile
 * sort of the pairs orders the bits of the batch's global tile ids, its first pass fused with pair
 * emission (counted here). 0 for an empty sort. Either pointer may be NULL. */
int mvgs_frame_sort_info(const mvgs_frame* frame, int32_t* depth_passes, int32_t* tile_passes);

/* Test hook: copy a frame's binning to caller device buffers: keys [n_pairs]
 * (view<<48 | tile<<32 | depth bits), values [n_pairs] (Gaussian index), and
 * ranges [n_tiles][2] ([start,end) per (view, tile), view-major, row-major
 * tiles; empty tiles give [0,0)). Any output may be NULL. */
int mvgs_export_binning(mvgs_context* ctx, void* stream, const mvgs_frame* frame, uint64_t* keys,
                        uint32_t* values, uint32_t* ranges);

/* Test hook: copy each view's final transmittance to B device pointers
 * ([H,W] float32 each). */
int mvgs_export_transmittance(mvgs_context* ctx, void* stream, const mvgs_frame* frame, float* const* t_final);

/* Stage timing (opt-in). When enabled, every call records a pair of HIP events on its stream
 * around each stage below; mvgs_profile_read waits for them and adds their elapsed times.
 * Stages: 0 count (participation, record/pair totals), 1 records (projection + SH),
 * 2 depth_sort, 3 emit (pair emission in depth order), 4 tile_sort, 5 ranges,
 * 6 blend_fwd, 7 loss, 8 blend_bwd, 9 preprocess_bwd. */
#define MVGS_STAGE_COUNT 10
int mvgs_profile_enable(mvgs_context* ctx, int enable);
/* Accumulated milliseconds and launch counts per stage since the last reset (host arrays of
 * MVGS_STAGE_COUNT; either may be NULL). Waits for the recorded events. */
int mvgs_profile_read(mvgs_context* ctx, double* ms, int64_t* calls);
int mvgs_profile_reset(mvgs_context* ctx);
const char* mvgs_stage_name(int stage);

/* Work of a frame's walks (for rooflines; it walks every pixel's list again, so it costs about a
 * forward). Writes two device uint64 to work_dev: [0] the sum over pixels of the list entries from
 * the start of the pixel's (view, tile) list up to its last blended Gaussian (what Alg. 2's
 * per-thread loop visits), [1] the number of (pixel, Gaussian) pairs blended by Eq. 1, which
 * does not depend on the tile shape. */
int mvgs_frame_work(mvgs_context* ctx, void* stream, const mvgs_frame* frame, uint64_t* work_dev);

/* Human-readable text of a status code (static storage). */
const char* mvgs_status_string(int status);

/* Text of the last error recorded on a context (empty if none). */
const char* mvgs_last_error(const mvgs_context* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MVGS_H */
