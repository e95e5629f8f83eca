// Partial rendering (Sec. 5.1.1, Alg. 3): each view of the batch renders only a selection of its
// pixels, so that a batch of views costs about one view's worth of blending.
//
// The selection is the paper's index array. For every (view, tile) of the batch, in the global
// tile order of the ranges (view-major, row-major tiles), a segment of pixel indices y * W + x of
// that view lying in that tile. Thread-efficient mode gives every 64 selected pixels of a segment
// one wavefront (a "task"): its lanes take their pixels from the index array and walk the
// segment's sorted list exactly as the full-tile kernels walk theirs, so no lane waits on an
// unselected pixel. The binary-mask baseline of the paper instead runs the full-tile kernels with
// one bit per pixel (k_blend.hip).
//
// Sub-sampling: for B views of one size, each tile's pixel positions are ranked by a random key
// drawn by the caller (ties by position) and the position of rank r goes to view r mod B, so the
// views share every tile out evenly and together cover the image plane once.
#include "blend_device.h"

namespace mvgs {

// One wavefront per segment (plus one for the closing offset): offsets must rise from 0 to n_sel,
// a segment holds at most one tile of pixels, every pixel lies in its (view, tile) and appears
// once. Marks the pixels in `mask` (zeroed by the caller) and counts the segment's tasks. With
// plane_mask (views of one size, zeroed), also notes whether two views take the same position.
__global__ void __launch_bounds__(256) k_sel_check(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                   int tw, int th, const uint32_t* __restrict__ sel_off,
                                                   const uint32_t* __restrict__ sel_pix, uint32_t n_sel,
                                                   uint32_t* __restrict__ mask, uint32_t* __restrict__ plane_mask,
                                                   uint32_t* __restrict__ n_tasks, uint32_t* __restrict__ err) {
    // one wavefront per segment, its lanes over the segment's entries
    const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    if (t > n_tiles) return;
    if (t == n_tiles) {
        if (lane == 0 && sel_off[n_tiles] != n_sel) atomicOr(err, kSelBadOffsets);
        return;
    }
    const uint32_t a = sel_off[t], b = sel_off[t + 1];
    if ((t == 0 && a != 0) || a > b || b > n_sel) {
        if (lane == 0) {
            n_tasks[t] = 0;
            atomicOr(err, kSelBadOffsets);
        }
        return;
    }
    const uint32_t cnt = b - a;
    if (cnt > (uint32_t)(tw * th)) {
        if (lane == 0) {
            n_tasks[t] = 0;
            atomicOr(err, kSelTooLong);
        }
        return;
    }
    const DevCam& c = cams[find_view(cams, B, t)];
    const uint32_t local = t - c.tile_base;
    const int ty = (int)(local / (uint32_t)c.tiles_x), tx = (int)local - ty * c.tiles_x;
    const int x0 = tx * tw, y0 = ty * th;
    const int x1 = min(x0 + tw, c.W), y1 = min(y0 + th, c.H);
    const uint32_t hw = (uint32_t)c.W * (uint32_t)c.H;
    uint32_t bad = 0;
    for (uint32_t i0 = a; i0 < b; i0 += 64u) {   // whole wavefront in every round
        const uint32_t i = i0 + lane;
        bool in = false;
        uint32_t p = 0;
        if (i < b) {
            p = sel_pix[i];
            if (p >= hw) {
                bad |= kSelOutside;
            } else {
                const int y = (int)(p / (uint32_t)c.W), x = (int)(p - (uint32_t)y * (uint32_t)c.W);
                if (x < x0 || x >= x1 || y < y0 || y >= y1) bad |= kSelOutside;
                else in = true;
            }
        }
        const uint32_t gp = c.pix_base + p;
        // strictly ascending pixels (as sub-sampling writes them): no duplicate inside this round,
        // and pixels sharing a mask word sit in runs of neighbouring lanes, so each run sets its
        // bits with one atomic from its last lane
        // (a rejected pixel would leave a gap inside a run: then every lane takes the plain path)
        const uint32_t gp_prev = (uint32_t)__shfl_up((int)gp, 1, 64);
        const bool asc = ballot64((i < b && !in) || (in && lane > 0 && gp <= gp_prev)) == 0;
        if (asc) {
            uint32_t wd = in ? gp >> 5 : 0xffffffffu, bits = in ? 1u << (gp & 31u) : 0u;
            uint32_t pw = in ? p >> 5 : 0xffffffffu, pbits = in ? 1u << (p & 31u) : 0u;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t ob = (uint32_t)__shfl_up((int)bits, off, 64);
                const uint32_t ow = (uint32_t)__shfl_up((int)wd, off, 64);
                const uint32_t opb = (uint32_t)__shfl_up((int)pbits, off, 64);
                const uint32_t opw = (uint32_t)__shfl_up((int)pw, off, 64);
                if ((int)lane >= off && ow == wd) bits |= ob;
                if ((int)lane >= off && opw == pw) pbits |= opb;
            }
            const uint32_t wd_next = (uint32_t)__shfl_down((int)wd, 1, 64);
            const uint32_t pw_next = (uint32_t)__shfl_down((int)pw, 1, 64);
            if (in && (lane == 63 || wd_next != wd)) {
                if (atomicOr(mask + wd, bits) & bits) bad |= kSelDuplicate;
            }
            // views of one size: is each position of the shared image plane taken by one view only?
            if (plane_mask && in && (lane == 63 || pw_next != pw)) {
                if (atomicOr(plane_mask + pw, pbits) & pbits) bad |= kSelPlaneOverlap;
            }
        } else if (in) {
            const uint32_t bit = 1u << (gp & 31u);
            if (atomicOr(mask + (gp >> 5), bit) & bit) bad |= kSelDuplicate;
            if (plane_mask) {
                const uint32_t pb = 1u << (p & 31u);
                if (atomicOr(plane_mask + (p >> 5), pb) & pb) bad |= kSelPlaneOverlap;
            }
        }
    }
    if (bad) atomicOr(err, bad);
    if (lane == 0) n_tasks[t] = (cnt + 63u) / 64u;
}

// Task table: task task_off[t] + j is chunk j of segment t. Writes past `cap` (possible only for
// offsets k_sel_check rejects) are dropped.
__global__ void __launch_bounds__(256) k_sel_tasks(uint32_t n_tiles, const uint32_t* __restrict__ n_tasks,
                                                   const uint32_t* __restrict__ task_off, uint32_t cap,
                                                   uint2* __restrict__ tasks) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t n = n_tasks[t], o = task_off[t];
    for (uint32_t j = 0; j < n; ++j)
        if (o + j < cap) tasks[o + j] = make_uint2(t, j);
}

// The lanes of one task: pixel, position in the selection, and the view and list of its segment.
struct SelWave {
    int v;
    uint2 rg;
    uint32_t i;       // selection entry of this lane
    bool valid;
    int x, y;
    int bx0, bx1, by0, by1;   // bounding rectangle of the task's pixels
};

// The task of this wavefront: tasks are taken in XCD runs; in capacity mode the grid is a bound
// and n_dev (device) the count, and a set void word (a rejected selection, or records or pairs over
// their capacities) leaves every task undone.
__device__ __forceinline__ bool sel_task(uint32_t n_tasks, const uint32_t* __restrict__ n_dev,
                                         const uint32_t* __restrict__ void_word, uint32_t* pos) {
    if (void_word && *void_word) return false;
    *pos = xcd_tile(blockIdx.x, n_tasks);
    return !n_dev || *pos < *n_dev;
}

__device__ __forceinline__ SelWave sel_wave(const DevCam* __restrict__ cams, int B, const uint2* __restrict__ ranges,
                                            const uint32_t* __restrict__ sel_off,
                                            const uint32_t* __restrict__ sel_pix, const uint2* __restrict__ tasks,
                                            uint32_t pos, int lane) {
    SelWave w;
    const uint2 tk = tasks[pos];
    const uint32_t t = tk.x;
    w.v = find_view(cams, B, t);
    const DevCam& c = cams[w.v];
    w.rg = ranges[t];
    w.i = sel_off[t] + tk.y * 64u + (uint32_t)lane;
    w.valid = w.i < sel_off[t + 1];
    const uint32_t p = w.valid ? sel_pix[w.i] : 0u;
    w.y = (int)(p / (uint32_t)c.W);
    w.x = (int)(p - (uint32_t)w.y * (uint32_t)c.W);
    w.bx0 = wave_min_i32(w.valid ? w.x : 0x7fffffff);
    w.bx1 = wave_max_i32(w.valid ? w.x : -1);
    w.by0 = wave_min_i32(w.valid ? w.y : 0x7fffffff);
    w.by1 = wave_max_i32(w.valid ? w.y : -1);
    return w;
}

__global__ void __launch_bounds__(64) k_blend_fwd_sel(const DevCam* __restrict__ cams, int B,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals,
                                                      const BlendRec* __restrict__ recs,
                                                      const uint32_t* __restrict__ sel_off,
                                                      const uint32_t* __restrict__ sel_pix,
                                                      const uint2* __restrict__ tasks, uint32_t n_tasks,
                                                      float* const* __restrict__ images, float* __restrict__ t_sel,
                                                      uint32_t* __restrict__ last_sel, float* __restrict__ depth_sel,
                                                      const uint32_t* __restrict__ n_dev,
                                                      const uint32_t* __restrict__ void_word) {
    const int lane = (int)threadIdx.x;
    uint32_t pos;
    if (!sel_task(n_tasks, n_dev, void_word, &pos)) return;
    const SelWave w = sel_wave(cams, B, ranges, sel_off, sel_pix, tasks, pos, lane);
    const DevCam& c = cams[w.v];
    const float px = (float)w.x + 0.5f;
    const float py[1] = {(float)w.y + 0.5f};
    FwdPix st[1] = {FwdPix{w.valid ? 1.0f : -1.0f, 0.0f, 0.0f, 0.0f, 0u, 0.0f}};
    walk_forward<1, true>(st, px, py, w.rg, vals, recs, lane, w.bx0, w.bx1, w.by0, w.by1);
    if (w.valid) {
        const size_t hw = (size_t)c.W * c.H, pix = (size_t)w.y * c.W + w.x;
        float* img = images[w.v];
        const float T = fabsf(st[0].T);
        img[pix] = __builtin_fmaf(T, c.bg[0], st[0].C0);
        img[hw + pix] = __builtin_fmaf(T, c.bg[1], st[0].C1);
        img[2 * hw + pix] = __builtin_fmaf(T, c.bg[2], st[0].C2);
        t_sel[w.i] = T;
        last_sel[w.i] = st[0].last;
        depth_sel[w.i] = st[0].D;
    }
}

template <bool E1>
__global__ void __launch_bounds__(64) k_blend_bwd_sel(const DevCam* __restrict__ cams, int B,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ vals,
                                                      const BlendRec* __restrict__ recs,
                                                      const uint32_t* __restrict__ sel_off,
                                                      const uint32_t* __restrict__ sel_pix,
                                                      const uint2* __restrict__ tasks, uint32_t n_tasks,
                                                      const float* const* __restrict__ dl_dimg,
                                                      const float* __restrict__ t_sel,
                                                      const uint32_t* __restrict__ last_sel,
                                                      float* __restrict__ acc, const uint32_t* __restrict__ n_dev,
                                                      const uint32_t* __restrict__ void_word) {
    const int lane = (int)threadIdx.x;
    uint32_t pos;
    if (!sel_task(n_tasks, n_dev, void_word, &pos)) return;
    const SelWave w = sel_wave(cams, B, ranges, sel_off, sel_pix, tasks, pos, lane);
    const DevCam& c = cams[w.v];
    const float px = (float)w.x + 0.5f;
    BwdPix st[1] = {BwdPix{1.0f, 0.0f, 0.0f, 0.0f, c.bg[0], c.bg[1], c.bg[2], (float)w.y + 0.5f, 0u}};
    if (w.valid) {
        const size_t hw = (size_t)c.W * c.H, pix = (size_t)w.y * c.W + w.x;
        const float* g = dl_dimg[w.v];
        st[0].dC0 = g[pix];
        st[0].dC1 = g[hw + pix];
        st[0].dC2 = g[2 * hw + pix];
        st[0].T = t_sel[w.i];
        st[0].last = last_sel[w.i];
    }
    const uint32_t hi_end = __builtin_amdgcn_readfirstlane(wave_max_u32(st[0].last));
    walk_backward<E1, 1>(st, px, hi_end, 0u, w.rg, vals, recs, lane, w.bx0, w.bx1, w.by0, w.by1, 0.5f * (float)c.W,
                         0.5f * (float)c.H, acc);
}

// Sub-sampling, step 1: the size of every segment. Tile t of view v holds n_t pixels and view v
// gets ranks v, v + B, ..., i.e. ceil((n_t - v) / B) of them.
__global__ void __launch_bounds__(256) k_subsample_counts(int W, int H, int B, int tw, int th, int tiles_x,
                                                          uint32_t tiles_per_view, uint32_t* __restrict__ counts) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= (uint32_t)B * tiles_per_view) return;
    const uint32_t v = s / tiles_per_view, t = s - v * tiles_per_view;
    const int ty = (int)(t / (uint32_t)tiles_x), tx = (int)t - ty * tiles_x;
    const uint32_t n = (uint32_t)((min(W, tx * tw + tw) - tx * tw) * (min(H, ty * th + th) - ty * th));
    counts[s] = n > v ? (n - v + (uint32_t)B - 1u) / (uint32_t)B : 0u;
}

// Ascending bitonic sort of m (a power of two, at most 1024) 64-bit values in LDS by 256 threads.
__device__ __forceinline__ void lds_bitonic_sort(uint64_t* s, int m) {
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = (int)threadIdx.x; i < m; i += 256) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = s[i], b = s[ixj];
                    if ((a > b) == ((i & k) == 0)) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Sub-sampling, step 2: one workgroup per tile. The tile's positions (row-major index j) are
// sorted in LDS by (key, j); the position of rank r goes to view r mod B. A second sort by
// (view, j) lists each view's positions in ascending order (so the wavefronts of a segment cover
// compact bands of the tile); view v's run starts at v floor(n / B) + min(v, n mod B).
__global__ void __launch_bounds__(256) k_subsample_scatter(const uint32_t* __restrict__ keys, int W, int H, int B,
                                                           int tw, int th, int tiles_x, uint32_t tiles_per_view,
                                                           const uint32_t* __restrict__ sel_off,
                                                           uint32_t* __restrict__ sel_pix) {
    __shared__ uint64_t s[1024];
    const uint32_t t = blockIdx.x;
    const int ty = (int)(t / (uint32_t)tiles_x), tx = (int)t - ty * tiles_x;
    const int x0 = tx * tw, y0 = ty * th;
    const int w = min(W, x0 + tw) - x0, h = min(H, y0 + th) - y0;
    const int n = w * h;
    int m = 1;
    while (m < n) m <<= 1;
    for (int j = (int)threadIdx.x; j < m; j += 256) {
        uint64_t v = ~0ull;
        if (j < n) {
            const uint32_t p = (uint32_t)(y0 + j / w) * (uint32_t)W + (uint32_t)(x0 + j % w);
            v = ((uint64_t)keys[p] << 32) | (uint32_t)j;
        }
        s[j] = v;
    }
    __syncthreads();
    lds_bitonic_sort(s, m);
    for (int r = (int)threadIdx.x; r < n; r += 256)
        s[r] = ((uint64_t)(uint32_t)(r % B) << 32) | (uint32_t)(s[r] & 0xffffffffu);
    __syncthreads();
    lds_bitonic_sort(s, m);
    const int q = n / B, rem = n - q * B;
    for (int i = (int)threadIdx.x; i < n; i += 256) {
        const int v = (int)(s[i] >> 32), j = (int)(s[i] & 0xffffffffu);
        const int e = i - (v * q + min(v, rem));
        const uint32_t p = (uint32_t)(y0 + j / w) * (uint32_t)W + (uint32_t)(x0 + j % w);
        sel_pix[sel_off[(uint32_t)v * tiles_per_view + t] + (uint32_t)e] = p;
    }
}

// Walk work of a thread-efficient frame (as k_frame_work), one thread per segment.
__global__ void __launch_bounds__(256) k_frame_work_sel(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                        const uint2* __restrict__ ranges,
                                                        const uint32_t* __restrict__ vals,
                                                        const BlendRec* __restrict__ recs,
                                                        const uint32_t* __restrict__ sel_off,
                                                        const uint32_t* __restrict__ sel_pix,
                                                        const uint32_t* __restrict__ last_sel,
                                                        unsigned long long* __restrict__ out) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    unsigned long long steps = 0, blended = 0;
    if (t < n_tiles) {
        const DevCam& c = cams[find_view(cams, B, t)];
        const uint32_t start = ranges[t].x;
        for (uint32_t i = sel_off[t]; i < sel_off[t + 1]; ++i) {
            const uint32_t p = sel_pix[i], nl = last_sel[i];
            if (nl <= start) continue;
            steps += nl - start;
            const int y = (int)(p / (uint32_t)c.W), x = (int)(p - (uint32_t)y * (uint32_t)c.W);
            const float px = (float)x + 0.5f, py = (float)y + 0.5f;
            for (uint32_t j = start; j < nl; ++j) {
                const BlendRec& R = recs[vals[j]];
                if (pixel_power(px, py, R.mx, R.my, R.hca, R.nb, R.hcc) >= R.cut) ++blended;
            }
        }
    }
    if (steps) atomicAdd(out, steps);
    if (blended) atomicAdd(out + 1, blended);
}

__global__ void k_zero_pair(unsigned long long* p) {
    p[0] = 0ull;
    p[1] = 0ull;
}

void launch_sel_check(const DevCam* cams, int B, uint32_t n_tiles, int tw, int th, const uint32_t* sel_off,
                      const uint32_t* sel_pix, uint32_t n_sel, uint32_t* mask, uint32_t* plane_mask, uint32_t* n_tasks,
                      uint32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_sel_check, dim3((n_tiles + 1 + 3) / 4), dim3(256), 0, s, cams, B, n_tiles, tw, th,
                       sel_off, sel_pix, n_sel, mask, plane_mask, n_tasks, err);
}

// Per-selected-pixel values (final transmittance, depth) into per-view [H, W] planes; other pixels
// are left untouched.
__global__ void __launch_bounds__(256) k_sel_scatter_f(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                       const uint32_t* __restrict__ sel_off,
                                                       const uint32_t* __restrict__ sel_pix,
                                                       const float* __restrict__ v_sel, float* const* __restrict__ out,
                                                       const uint32_t* __restrict__ void_word) {
    const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);   // one wavefront per segment
    if (t >= n_tiles || (void_word && *void_word)) return;
    float* o = out[find_view(cams, B, t)];
    for (uint32_t i = sel_off[t] + (threadIdx.x & 63u); i < sel_off[t + 1]; i += 64u) o[sel_pix[i]] = v_sel[i];
}

// Per-view [C, H, W] planes of one size merged into one plane: each selected pixel takes the value
// of the view that selected it; other pixels are left untouched.
__global__ void __launch_bounds__(256) k_sel_merge(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                   const uint32_t* __restrict__ sel_off,
                                                   const uint32_t* __restrict__ sel_pix,
                                                   const float* const* __restrict__ planes, int C, uint32_t plane_px,
                                                   float* __restrict__ out, const uint32_t* __restrict__ void_word) {
    const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);   // one wavefront per segment
    if (t >= n_tiles || (void_word && *void_word)) return;
    const float* in = planes[find_view(cams, B, t)];
    for (uint32_t i = sel_off[t] + (threadIdx.x & 63u); i < sel_off[t + 1]; i += 64u) {
        const uint32_t p = sel_pix[i];
        for (int c = 0; c < C; ++c) out[(size_t)c * plane_px + p] = in[(size_t)c * plane_px + p];
    }
}

void launch_sel_merge(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                      const float* const* planes, int C, uint32_t plane_px, float* out, hipStream_t s,
                      const uint32_t* void_word) {
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_sel_merge, dim3((n_tiles + 3) / 4), dim3(256), 0, s, cams, B, n_tiles, sel_off, sel_pix,
                       planes, C, plane_px, out, void_word);
}

// Capacity mode: a rejected selection (bit 1 of the void word) or more tasks than their bound
// (bit 2) voids the frame like a capacity overflow: the record and pair counts become 0 and no
// kernel reads the pixel indices.
__global__ void k_sel_void(const uint32_t* __restrict__ sel_err, const unsigned long long* __restrict__ task_total,
                           uint32_t task_cap, uint32_t* __restrict__ eff, uint32_t* __restrict__ void_word) {
    uint32_t bits = (*sel_err & kSelErrors) ? 2u : 0u;
    if (*task_total > task_cap) bits |= 4u;
    if (bits) {
        eff[0] = 0u;
        eff[1] = 0u;
        *void_word |= bits;
    }
}

void launch_sel_void(const uint32_t* sel_err, const uint64_t* task_total, uint32_t task_cap, uint32_t* eff,
                     uint32_t* void_word, hipStream_t s) {
    hipLaunchKernelGGL(k_sel_void, dim3(1), dim3(1), 0, s, sel_err, (const unsigned long long*)task_total, task_cap,
                       eff, void_word);
}

void launch_sel_tasks(uint32_t n_tiles, const uint32_t* n_tasks, const uint32_t* task_off, uint32_t cap,
                      uint2* tasks, hipStream_t s) {
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_sel_tasks, dim3((n_tiles + 255) / 256), dim3(256), 0, s, n_tiles, n_tasks, task_off, cap,
                       tasks);
}

void launch_blend_fwd_sel(const SelBlendArgs& a, hipStream_t s) {
    if (!a.n_tasks) return;
    hipLaunchKernelGGL(k_blend_fwd_sel, dim3(a.n_tasks), dim3(64), 0, s, a.cams, a.B, a.ranges, a.vals, a.recs,
                       a.sel_off, a.sel_pix, a.tasks, a.n_tasks, a.images, a.t_sel, a.last_sel, a.depth_sel, a.n_dev,
                       a.void_word);
}

void launch_blend_bwd_sel(const SelBlendArgs& a, hipStream_t s) {
    if (!a.n_tasks) return;
    if (a.want_e1)
        hipLaunchKernelGGL(k_blend_bwd_sel<true>, dim3(a.n_tasks), dim3(64), 0, s, a.cams, a.B, a.ranges, a.vals,
                           a.recs, a.sel_off, a.sel_pix, a.tasks, a.n_tasks, a.dl_dimg, a.t_sel, a.last_sel, a.acc,
                           a.n_dev, a.void_word);
    else
        hipLaunchKernelGGL(k_blend_bwd_sel<false>, dim3(a.n_tasks), dim3(64), 0, s, a.cams, a.B, a.ranges, a.vals,
                           a.recs, a.sel_off, a.sel_pix, a.tasks, a.n_tasks, a.dl_dimg, a.t_sel, a.last_sel, a.acc,
                           a.n_dev, a.void_word);
}

void launch_subsample(const uint32_t* keys, int W, int H, int B, int tw, int th, uint32_t* sel_off,
                      uint32_t* sel_pix, void* scan_scratch, hipStream_t s) {
    const int tiles_x = (W + tw - 1) / tw, tiles_y = (H + th - 1) / th;
    const uint32_t tpv = (uint32_t)(tiles_x * tiles_y);
    const uint32_t nseg = (uint32_t)B * tpv;
    hipLaunchKernelGGL(k_subsample_counts, dim3((nseg + 255) / 256), dim3(256), 0, s, W, H, B, tw, th, tiles_x, tpv,
                       sel_off);
    // offsets in place; the closing offset (the total) is W * H
    scan_exclusive_u32(sel_off, sel_off, nseg, nullptr, scan_scratch, s);
    fill_u32(sel_off + nseg, 1, (uint32_t)W * (uint32_t)H, s);
    hipLaunchKernelGGL(k_subsample_scatter, dim3(tpv), dim3(256), 0, s, keys, W, H, B, tw, th, tiles_x, tpv, sel_off,
                       sel_pix);
}

void launch_sel_scatter(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                        const float* v_sel, float* const* out, hipStream_t s, const uint32_t* void_word) {
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_sel_scatter_f, dim3((n_tiles + 3) / 4), dim3(256), 0, s, cams, B, n_tiles, sel_off,
                       sel_pix, v_sel, out, void_word);
}

void launch_frame_work_sel(const DevCam* cams, int B, uint32_t n_tiles, const uint2* ranges, const uint32_t* vals,
                           const BlendRec* recs, const uint32_t* sel_off, const uint32_t* sel_pix,
                           const uint32_t* last_sel, uint64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_pair, dim3(1), dim3(1), 0, s, (unsigned long long*)out);
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_frame_work_sel, dim3((n_tiles + 255) / 256), dim3(256), 0, s, cams, B, n_tiles, ranges, vals,
                       recs, sel_off, sel_pix, last_sel, (unsigned long long*)out);
}

}  // namespace mvgs
