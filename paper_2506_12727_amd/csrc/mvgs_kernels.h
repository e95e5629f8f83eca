// Launch interfaces of the mvgs kernels (host side, internal to libmvgs).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mvgs_device.h"

namespace mvgs {

struct GaussianArgs {
    const float* means;
    const float* scales;
    const float* quats;
    const float* opac;
    const float* sh;
    int64_t P;
    int sh_degree;
};

struct GradArgs {
    float* means;
    float* scales;
    float* quats;
    float* opac;
    float* sh;
    float* e1;       // may be null (then e2, count are ignored)
    float* e2;
    int32_t* count;
};

// k_preprocess.hip
// key_range: null, or 2 device words (min, ~max) that the depth keys of the participating records
// are folded into with atomicMin (the caller sets both to ~0 first)
void launch_count(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th, uint32_t* nrec,
                  uint32_t* ntiles, hipStream_t s, uint32_t* key_range = nullptr);
// overflow: null, or a device word that, when non-zero, makes the kernel write nothing
// per-view participating records and covered tiles (counts [B][2], written), through per-workgroup
// partials in scratch (count_views_scratch_bytes)
size_t count_views_scratch_bytes(int64_t P, int B);
void launch_count_views(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th,
                        unsigned long long* counts, unsigned long long* scratch, hipStream_t s);
void launch_records(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th, const uint32_t* rec_off,
                    BlendRec* recs, uint32_t* depth_key, uint2* tile_rect, uint16_t* rec_view, hipStream_t s,
                    const uint32_t* overflow = nullptr);
// overflow: as above; when set, every Gaussian is treated as taking part in no view
void launch_preprocess_bwd(const GaussianArgs& ga, const DevCam* cams, const uint32_t* rec_off,
                           const uint16_t* rec_view, const float* acc, const GradArgs& gr, hipStream_t s,
                           const uint32_t* overflow = nullptr);

// k_sort.hip
// Counts in capacity mode: a launch is sized by a host bound n and, when n_dev is not null, works
// on the first min(*n_dev, n) items only (n_dev is written by earlier kernels on the stream).
__device__ __forceinline__ size_t count_of(size_t bound, const uint32_t* n_dev) {
    if (!n_dev) return bound;
    const size_t d = *n_dev;
    return d < bound ? d : bound;
}

// Exclusive scan of n u32 values (in may equal out). The total is written to *total64 (device).
// `scratch` must hold scan_scratch_bytes(n) bytes.
size_t scan_scratch_bytes(size_t n);
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t n, uint64_t* total64, void* scratch,
                        hipStream_t s, const uint32_t* n_dev = nullptr);
// Sum of n u32 values as u64 into *total64 (device).
void reduce_sum_u32(const uint32_t* in, size_t n, uint64_t* total64, void* scratch, hipStream_t s);

// Stable LSD radix sort of (key, value) u32 pairs by key - key_base on bits [0, bits) (every key
// must lie in [key_base, key_base + 2^bits)), at most 8 bits per pass; a pass reads the keys twice
// (count, scatter) and writes keys and values once. The input is in keys[0] and vals[0] (or, with
// identity_values, the values are 0..n-1 and vals[0] is only ping-pong space); passes alternate
// between buffers 0 and 1. With pay, an 8-byte payload per item (input in pay[0]) travels with
// its key the same way. Returns the index of the buffer holding the result; with sorted_keys
// false the last pass writes no keys (only the order of the values and payloads is wanted).
size_t radix_scratch_bytes(size_t n);
int radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], bool identity_values, size_t n, int bits, void* scratch,
                   hipStream_t s, const uint32_t* n_dev = nullptr, uint32_t key_base = 0, uint2* pay[2] = nullptr,
                   bool sorted_keys = true);

void fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
// per * min(*n_dev, n) values (all per * n when n_dev is null)
void fill_u32_count(uint32_t* p, size_t n, const uint32_t* n_dev, uint32_t per, uint32_t v, hipStream_t s);
// eff = the counts, or 0 and 0 with *overflow = 1 when they exceed the capacities; with key_range
// (min, ~max of the depth keys) also 8 when the keys leave [key_base, key_base + 2^key_bits), and
// the range copied to range_out
void launch_capacity_clamp(const uint64_t* totals, uint64_t cap_v, uint64_t cap_k, uint32_t* eff, uint32_t* overflow,
                           hipStream_t s, const uint32_t* key_range = nullptr, uint32_t key_base = 0,
                           int key_bits = 32, uint32_t* range_out = nullptr);

// Pairs of the depth-ordered records and their stable sort by global tile id (of `bits` bits):
// from the records and their tile rectangles in depth order (sorted_rec, sorted_rect: [n_rec],
// the rectangles carried through the depth sort), every (global tile, record) pair is emitted
// straight into its place after the first radix pass (keys, vals: [K]); sort_pairs_rest runs the
// remaining passes from buffers 0 and returns the index of the buffer holding the sorted pairs.
// n_rec and K are bounds when n_rec_dev / K_dev (device) give the counts. key16: the tile ids fit
// in 16 bits (at most 65,536 tiles) and the key buffers hold uint16_t, else uint32_t.
size_t emit_sort_scratch_bytes(size_t n_rec, size_t K);
void emit_pairs_first_pass(const uint32_t* sorted_rec, const uint2* sorted_rect, const DevCam* cams, int B,
                           size_t n_rec, const uint32_t* n_rec_dev, void* keys, bool key16, uint32_t* vals, size_t K,
                           const uint32_t* K_dev, int bits, void* scratch, hipStream_t s);
int sort_pairs_rest(void* keys[2], bool key16, uint32_t* vals[2], size_t K, const uint32_t* K_dev, int bits,
                    void* scratch, hipStream_t s);
void launch_ranges(const void* keys, bool key16, uint32_t K, uint32_t n_tiles, uint2* ranges, hipStream_t s,
                   const uint32_t* K_dev = nullptr);
void launch_export_keys(const void* tile_keys, bool key16, const uint32_t* vals, const BlendRec* recs,
                        const DevCam* cams, int B, uint32_t K, uint64_t* keys_out, uint32_t* vals_out,
                        hipStream_t s);

// k_blend.hip
struct BlendFwdArgs {
    const DevCam* cams;
    int B;
    uint32_t n_tiles;
    const uint2* ranges;
    const uint32_t* vals;
    const BlendRec* recs;
    float* const* images;   // device array of B device pointers
    float* t_final;         // [total pixels]
    uint32_t* n_last;       // [total pixels]
    const uint32_t* mask;   // null, or one bit per pixel of the batch: render only the set ones
};
struct BlendBwdArgs {
    const DevCam* cams;
    int B;
    uint32_t n_tiles;
    const uint2* ranges;
    const uint32_t* vals;
    const BlendRec* recs;
    const float* const* dl_dimg;  // device array of B device pointers
    const float* t_final;
    const uint32_t* n_last;
    float* acc;             // [V][kAccStride]
    int want_e1;
    const uint32_t* mask;   // as in BlendFwdArgs
};
bool blend_supported(int tw, int th, int ppl);
int blend_default_ppl(int tw, int th);
void launch_frame_work(const DevCam* cams, int B, const uint2* ranges, const uint32_t* vals, const BlendRec* recs,
                       const uint32_t* n_last, uint32_t n_pixels, int tw, int th, uint64_t* out, hipStream_t s);
void launch_blend_fwd(const BlendFwdArgs& a, int tw, int th, int ppl, hipStream_t s);
void launch_blend_bwd(const BlendBwdArgs& a, int tw, int th, int ppl, hipStream_t s);

// k_partial.hip: partial rendering over a pixel selection (see the file comment)
constexpr uint32_t kSelBadOffsets = 1, kSelOutside = 2, kSelDuplicate = 4, kSelTooLong = 8;
constexpr uint32_t kSelErrors = 15;
constexpr uint32_t kSelPlaneOverlap = 16;   // not an error: two views share a plane position
struct SelBlendArgs {
    const DevCam* cams;
    int B;
    const uint2* ranges;
    const uint32_t* vals;
    const BlendRec* recs;
    const uint32_t* sel_off;    // [n_tiles + 1]
    const uint32_t* sel_pix;    // [n_sel]
    const uint2* tasks;         // (segment, chunk of 64) per wavefront
    uint32_t n_tasks;
    float* const* images;       // forward: device array of B device pointers
    float* t_sel;               // [n_sel]
    uint32_t* last_sel;         // [n_sel]
    float* depth_sel;           // [n_sel] blended depth (forward)
    const float* const* dl_dimg;  // backward
    float* acc;
    int want_e1;
    const uint32_t* n_dev;      // capacity mode: the task count (device; n_tasks is then the bound)
    const uint32_t* void_word;  // capacity mode: non-zero voids the frame (nothing is rendered)
};
void launch_sel_void(const uint32_t* sel_err, const uint64_t* task_total, uint32_t task_cap, uint32_t* eff,
                     uint32_t* void_word, hipStream_t s);
void launch_sel_check(const DevCam* cams, int B, uint32_t n_tiles, int tw, int th, const uint32_t* sel_off,
                      const uint32_t* sel_pix, uint32_t n_sel, uint32_t* mask, uint32_t* plane_mask, uint32_t* n_tasks,
                      uint32_t* err, hipStream_t s);
void launch_sel_tasks(uint32_t n_tiles, const uint32_t* n_tasks, const uint32_t* task_off, uint32_t cap,
                      uint2* tasks, hipStream_t s);
void launch_blend_fwd_sel(const SelBlendArgs& a, hipStream_t s);
void launch_blend_bwd_sel(const SelBlendArgs& a, hipStream_t s);
void launch_subsample(const uint32_t* keys, int W, int H, int B, int tw, int th, uint32_t* sel_off,
                      uint32_t* sel_pix, void* scan_scratch, hipStream_t s);
void launch_sel_merge(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                      const float* const* planes, int C, uint32_t plane_px, float* out, hipStream_t s,
                      const uint32_t* void_word = nullptr);
void launch_sel_scatter(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                        const float* v_sel, float* const* out, hipStream_t s, const uint32_t* void_word = nullptr);
void launch_frame_work_sel(const DevCam* cams, int B, uint32_t n_tiles, const uint2* ranges, const uint32_t* vals,
                           const BlendRec* recs, const uint32_t* sel_off, const uint32_t* sel_pix,
                           const uint32_t* last_sel, uint64_t* out, hipStream_t s);

// k_densify.hip: multi-view adaptive density control
struct AdcParams {
    float split_threshold, clone_threshold, dense_scale, min_opacity;
};
void launch_adc_classify(const GaussianArgs& ga, const float* e1, const float* e2, const int32_t* count,
                         const AdcParams& prm, uint32_t* n_out, uint8_t* action, hipStream_t s);
void launch_adc_write(const GaussianArgs& ga, const float* normals, const uint8_t* action, const uint32_t* off,
                      float* means, float* scales, float* quats, float* opac, float* sh, int32_t* src, hipStream_t s);

// k_train.hip: optimiser step, state gather and gradient moments of the training loop
struct AdamArgs {
    float lr_means, lr_scales, lr_quats, lr_opacities, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float bc1, bc2;   // bias corrections 1 - beta^step
};
// state (device, 3 words) null: the bias corrections of `a`; else the step reads them from the
// state launch_adam_count wrote, and does nothing when its first word is set
void launch_adam(float* means, float* scales, float* quats, float* opac, float* sh, const GradArgs& gr, float* mom,
                 int64_t P, int sh_degree, const AdamArgs& a, hipStream_t s, const float* state = nullptr);
// device step counter: unless *skip, ++*step and the bias corrections for it into state[1..2];
// state[0] = skip
void launch_adam_count(int32_t* step, const uint32_t* skip, float beta1, float beta2, float* state, hipStream_t s);
void launch_gather_rows(const int32_t* src, int64_t n, int64_t width, const float* in, float* out, hipStream_t s);
// the five gradient tensors (means, scales, quats, opacities, SH) as one vector: x[k] holds
// elements [end[k-1], end[k]) of it
struct GradSegments {
    const float* x[5];
    int64_t end[5];
};
constexpr int kMomentBlocks = 1024;   // workgroups of the moment pass (2 double partials each)
size_t moment_blocks(int64_t n);       // workgroups the moment pass uses for n elements
void launch_grad_moments(const GradSegments& g, double* sum, double* acc, double* partials, hipStream_t s);

// k_loss3d.hip: L1 + 3D distance-aware D-SSIM on the merged plane of a thread-efficient partial
// frame whose selection covers the plane once
size_t loss3d_scratch_bytes(int W, int H);
void launch_loss3d(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                   const float* t_sel, const float* depth_sel, int W, int H, const float* img, const float* tgt,
                   float w_l1, float w_dssim, float* loss_out, float* grad, void* scratch, hipStream_t s,
                   const uint32_t* void_word = nullptr);

// k_loss.hip
struct LossView {
    const float* img;
    const float* tgt;
    float* grad;
    int32_t W, H;
    uint32_t pix_base;
    uint32_t pad;
};
// D-SSIM output tiles (per channel) of a W x H view
uint32_t ssim_tiles(int W, int H);
// partial sums of the loss kernels over total_pixels pixels whose views hold ssim_tiles_total tiles
size_t loss_scratch_bytes(uint32_t total_pixels, uint64_t ssim_tiles_total);
// at most this many views per launch_put_loss_views (kernel-argument table; one wavefront)
constexpr int kLossArgViews = 64;
void launch_put_loss_views(const LossView* views, int B, LossView* dst, hipStream_t s);
void launch_loss(const LossView* views_dev, const LossView* views_host, int B, uint32_t total_pixels, float w_l1,
                 float w_dssim, float* loss_out, void* scratch, hipStream_t s);

}  // namespace mvgs
