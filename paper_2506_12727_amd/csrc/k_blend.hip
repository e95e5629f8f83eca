// Tile blending, forward and backward (paper Sec. 3, Eq. 1; Alg. 2 tiled rendering; multi-view
// appendix: one block per (tile, view)).
//
// Launch: one workgroup per (view, tile) over all views of the batch in a single grid; a tile of
// TW x TH pixels is covered by (TW/8) x (TH/8) wavefronts, each owning an 8 x 8 sub-tile, one
// pixel per lane. Every lane of a wavefront blends the same Gaussian at the same time, so the
// Gaussian's record is wavefront-uniform: it is read through the scalar unit into SGPRs and
// feeds the vector ALU directly. Unlike the paper's Alg. 2 there is no shared-memory batch and
// no block barrier: each wavefront walks its tile's sorted list on its own, skips Gaussians whose
// pixel box misses its sub-tile (a scalar test), and leaves as soon as all of its pixels have
// stopped. Workgroups are mapped so that each XCD receives a contiguous run of tiles.
#include "blend_device.h"

namespace mvgs {

// Geometry of one wavefront: an SW x SH sub-tile of the (view, tile) of this workgroup with
// SW * SH = 64 PPL (8x8, 8x16 or 16x16); lane l owns the PPL pixels
// (sx0 + l % SW, sy0 + l / SW + (64 / SW) k), k < PPL.
template <int PPL>
struct SubTile {
    static constexpr int SW = PPL == 4 ? 16 : 8;
    static constexpr int ROWS = 64 / SW;     // pixel rows one lane-step covers
    static constexpr int SH = ROWS * PPL;
};

struct WaveTile {
    int v;
    int sx0, sx1, sy0, sy1;
    uint2 rg;
    bool empty;
};

template <int TW, int TH, int PPL>
__device__ __forceinline__ WaveTile wave_tile(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                              const uint2* __restrict__ ranges) {
    using ST = SubTile<PPL>;
    constexpr int WX = TW / ST::SW;
    WaveTile w;
    const uint32_t tile = xcd_tile(blockIdx.x, n_tiles);
    w.v = find_view(cams, B, tile);
    const DevCam& c = cams[w.v];
    const uint32_t local = tile - c.tile_base;
    const int ty = (int)(local / (uint32_t)c.tiles_x);
    const int tx = (int)local - ty * c.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    w.sx0 = tx * TW + (wave % WX) * ST::SW;
    w.sy0 = ty * TH + (wave / WX) * ST::SH;
    w.empty = w.sx0 >= c.W || w.sy0 >= c.H;
    w.sx1 = min(w.sx0 + ST::SW - 1, c.W - 1);
    w.sy1 = min(w.sy0 + ST::SH - 1, c.H - 1);
    w.rg = ranges[tile];
    return w;
}

constexpr uint32_t kUnselected = 0xffffffffu;

// Whether pixel (x, y) of view c is rendered: inside the image and, when a selection mask (one bit
// per pixel of the batch, at pix_base + y W + x) is given, selected.
__device__ __forceinline__ bool pixel_selected(const DevCam& c, int x, int y, const uint32_t* __restrict__ mask) {
    if (!(x < c.W && y < c.H)) return false;
    if (!mask) return true;
    const uint32_t gp = c.pix_base + (uint32_t)y * (uint32_t)c.W + (uint32_t)x;
    return (mask[gp >> 5] >> (gp & 31u)) & 1u;
}

template <int TW, int TH, int PPL>
__global__ void __launch_bounds__(TW * TH / PPL) k_blend_fwd(const DevCam* __restrict__ cams, int B,
                                                             uint32_t n_tiles, const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ vals,
                                                             const BlendRec* __restrict__ recs,
                                                             float* const* __restrict__ images,
                                                             float* __restrict__ t_final,
                                                             uint32_t* __restrict__ n_last,
                                                             const uint32_t* __restrict__ mask) {
    const WaveTile wt = wave_tile<TW, TH, PPL>(cams, B, n_tiles, ranges);
    if (wt.empty) return;
    using ST = SubTile<PPL>;
    const DevCam& c = cams[wt.v];
    const int lane = (int)(threadIdx.x & 63);
    const int x = wt.sx0 + (lane % ST::SW);
    const float px = (float)x + 0.5f;
    float py[PPL];
    FwdPix st[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int y = wt.sy0 + (lane / ST::SW) + ST::ROWS * k;
        py[k] = (float)y + 0.5f;
        // an unselected pixel starts stopped, marked by an impossible last contributor, so the
        // mask is not needed again after the walk (it would hold scalar registers the walk uses)
        const bool sel = pixel_selected(c, x, y, mask);
        st[k] = FwdPix{sel ? 1.0f : -1.0f, 0.0f, 0.0f, 0.0f, sel ? 0u : kUnselected, 0.0f};
    }
    // The walk of walk_forward, written out here: with the call, the compiler optimises the loop
    // apart from this kernel and the kernel runs out of scalar registers. The next window's loads
    // are issued before the current window's candidates are blended.
    WindowPre nxt = window_load(vals, recs, wt.rg.x, wt.rg.y, lane);
    for (uint32_t base = wt.rg.x; base < wt.rg.y; base += 64) {
        uint64_t lm[PPL];
        uint64_t any = 0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            lm[k] = ballot64(pix_live(st[k]));
            any |= lm[k];
        }
        if (any == 0) break;
        // candidates are culled against the pixels still live
        int ax0, ax1, ay0, ay1;
        active_rect<PPL, ST::SW>(lm, wt.sx0, wt.sy0, ax0, ax1, ay0, ay1);
        const WindowPre cur = nxt;
        const uint32_t rl = cur.rl;
        uint64_t m = window_test(cur, recs, ax0, ax1, ay0, ay1);
        if (base + 64u < wt.rg.y) nxt = window_load(vals, recs, base + 64u, wt.rg.y, lane);
        while (m) {
            // up to four records per round trip through the scalar cache
            const int j0 = __builtin_ctzll(m);
            m &= m - 1;
            const int j1 = m ? __builtin_ctzll(m) : j0;
            if (m) m &= m - 1;
            const bool h1 = j1 != j0;
            const int j2 = m ? __builtin_ctzll(m) : j0;
            if (m) m &= m - 1;
            const bool h2 = j2 != j0;
            const int j3 = m ? __builtin_ctzll(m) : j0;
            if (m) m &= m - 1;
            const bool h3 = j3 != j0;
            const RecS q0 = load_rec(recs, readlane_u32(rl, j0));
            const RecS q1 = load_rec(recs, readlane_u32(rl, j1));
            const RecS q2 = load_rec(recs, readlane_u32(rl, j2));
            const RecS q3 = load_rec(recs, readlane_u32(rl, j3));
            // the column terms of the power once per lane, shared by its PPL pixels
            const PowerX t0 = power_x(px, q0.mx, q0.hca, q0.nb);
#pragma unroll
            for (int k = 0; k < PPL; ++k) blend_step<false>(st[k], q0, t0, py[k], base + (uint32_t)j0);
            if (h1) {
                const PowerX t1 = power_x(px, q1.mx, q1.hca, q1.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<false>(st[k], q1, t1, py[k], base + (uint32_t)j1);
            }
            if (h2) {
                const PowerX t2 = power_x(px, q2.mx, q2.hca, q2.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<false>(st[k], q2, t2, py[k], base + (uint32_t)j2);
            }
            if (h3) {
                const PowerX t3 = power_x(px, q3.mx, q3.hca, q3.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<false>(st[k], q3, t3, py[k], base + (uint32_t)j3);
            }
        }
    }
    const size_t hw = (size_t)c.W * c.H;
    float* img = images[wt.v];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int y = wt.sy0 + (lane / ST::SW) + ST::ROWS * k;
        if (x < c.W && y < c.H) {
            const size_t pix = (size_t)y * c.W + x;
            const bool sel = st[k].last != kUnselected;
            const float T = fabsf(st[k].T);
            if (sel) {
                img[pix] = __builtin_fmaf(T, c.bg[0], st[k].C0);
                img[hw + pix] = __builtin_fmaf(T, c.bg[1], st[k].C1);
                img[2 * hw + pix] = __builtin_fmaf(T, c.bg[2], st[k].C2);
            }
            t_final[c.pix_base + pix] = T;
            n_last[c.pix_base + pix] = sel ? st[k].last : 0u;
        }
    }
}

template <int TW, int TH, int PPL, bool E1>
__global__ void __launch_bounds__(TW * TH / PPL) k_blend_bwd(const DevCam* __restrict__ cams, int B,
                                                             uint32_t n_tiles, const uint2* __restrict__ ranges,
                                                             const uint32_t* __restrict__ vals,
                                                             const BlendRec* __restrict__ recs,
                                                             const float* const* __restrict__ dl_dimg,
                                                             const float* __restrict__ t_final,
                                                             const uint32_t* __restrict__ n_last,
                                                             float* __restrict__ acc,
                                                             const uint32_t* __restrict__ mask) {
    const WaveTile wt = wave_tile<TW, TH, PPL>(cams, B, n_tiles, ranges);
    if (wt.empty) return;
    using ST = SubTile<PPL>;
    const DevCam& c = cams[wt.v];
    const int lane = (int)(threadIdx.x & 63);
    const int x = wt.sx0 + (lane % ST::SW);
    const float px = (float)x + 0.5f;
    const float half_w = 0.5f * (float)c.W, half_h = 0.5f * (float)c.H;
    const size_t hw = (size_t)c.W * c.H;
    const float* g = dl_dimg[wt.v];
    BwdPix st[PPL];
    uint32_t lane_last = 0, lane_first = ~0u;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
        const int y = wt.sy0 + (lane / ST::SW) + ST::ROWS * k;
        st[k] = BwdPix{1.0f, 0.0f, 0.0f, 0.0f, c.bg[0], c.bg[1], c.bg[2], (float)y + 0.5f, 0u};
        if (pixel_selected(c, x, y, mask)) {
            const size_t pix = (size_t)y * c.W + x;
            st[k].dC0 = g[pix];
            st[k].dC1 = g[hw + pix];
            st[k].dC2 = g[2 * hw + pix];
            st[k].T = t_final[c.pix_base + pix];
            st[k].last = n_last[c.pix_base + pix];
            lane_last = max(lane_last, st[k].last);
        }
        // a pixel without contributors is made inert, so the walk may skip its position test
        if (st[k].last == 0u) st[k].T = st[k].dC0 = st[k].dC1 = st[k].dC2 = 0.0f;
        lane_first = min(lane_first, st[k].last == 0u ? ~0u : st[k].last);
    }
    const uint32_t hi_end = __builtin_amdgcn_readfirstlane(wave_max_u32(lane_last));
    const uint32_t lo_end = __builtin_amdgcn_readfirstlane(~wave_max_u32(~lane_first));
    walk_backward<E1, PPL, ST::SW>(st, px, hi_end, lo_end, wt.rg, vals, recs, lane, wt.sx0, wt.sx1, wt.sy0, wt.sy1,
                                   half_w, half_h, acc);
}

// Work of a frame's walks, one thread per pixel: out[0] += list entries from the start of the pixel's
// (view, tile) list to its last blended Gaussian; out[1] += Gaussians blended into the pixel (entries
// before the last blended one that pass the cut test at the pixel, walked again here).
__global__ void __launch_bounds__(256) k_frame_work(const DevCam* __restrict__ cams, int B,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ vals,
                                                    const BlendRec* __restrict__ recs,
                                                    const uint32_t* __restrict__ n_last, uint32_t n_pixels, int tw,
                                                    int th, unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[2][256];
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    unsigned long long steps = 0, blended = 0;
    if (p < n_pixels) {
        int lo = 0, hi = B;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cams[mid].pix_base <= p) lo = mid;
            else hi = mid;
        }
        const DevCam& c = cams[lo];
        const uint32_t i = p - c.pix_base;
        const int y = (int)(i / (uint32_t)c.W), x = (int)(i - (uint32_t)y * c.W);
        const uint32_t tile = c.tile_base + (uint32_t)((y / th) * c.tiles_x + x / tw);
        const uint32_t start = ranges[tile].x, nl = n_last[p];
        if (nl > start) {
            steps = nl - start;
            const float px = (float)x + 0.5f, py = (float)y + 0.5f;
            for (uint32_t j = start; j < nl; ++j) {
                const BlendRec& R = recs[vals[j]];
                if (pixel_power(px, py, R.mx, R.my, R.hca, R.nb, R.hcc) >= R.cut) ++blended;
            }
        }
    }
    red[0][threadIdx.x] = steps;
    red[1][threadIdx.x] = blended;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(out, red[0][0]);
        atomicAdd(out + 1, red[1][0]);
    }
}

__global__ void k_zero_u64x2(unsigned long long* p) {
    p[0] = 0ull;
    p[1] = 0ull;
}

void launch_frame_work(const DevCam* cams, int B, const uint2* ranges, const uint32_t* vals, const BlendRec* recs,
                       const uint32_t* n_last, uint32_t n_pixels, int tw, int th, uint64_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64x2, dim3(1), dim3(1), 0, s, (unsigned long long*)out);
    if (!n_pixels) return;
    hipLaunchKernelGGL(k_frame_work, dim3((n_pixels + 255) / 256), dim3(256), 0, s, cams, B, ranges, vals, recs,
                       n_last, n_pixels, tw, th, (unsigned long long*)out);
}

bool blend_supported(int tw, int th, int ppl) {
    const bool okw = tw == 8 || tw == 16 || tw == 32;
    const bool okh = th == 8 || th == 16 || th == 32;
    if (!okw || !okh) return false;
    if (ppl == 1) return true;
    if (ppl == 2) return th >= 16;
    if (ppl == 4) return tw >= 16 && th >= 16;
    return false;
}

int blend_default_ppl(int tw, int th) {
    if (tw >= 16 && th >= 16) return 4;
    return th >= 16 ? 2 : 1;
}

template <int W_, int H_, int P_>
static void launch_fwd_t(const BlendFwdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_fwd<W_, H_, P_>), dim3(a.n_tiles), dim3(W_ * H_ / P_), 0, s, a.cams, a.B, a.n_tiles,
                       a.ranges, a.vals, a.recs, a.images, a.t_final, a.n_last, a.mask);
}

template <int W_, int H_, int P_>
static void launch_bwd_t(const BlendBwdArgs& a, hipStream_t s) {
    if (a.want_e1)
        hipLaunchKernelGGL((k_blend_bwd<W_, H_, P_, true>), dim3(a.n_tiles), dim3(W_ * H_ / P_), 0, s, a.cams, a.B,
                           a.n_tiles, a.ranges, a.vals, a.recs, a.dl_dimg, a.t_final, a.n_last, a.acc, a.mask);
    else
        hipLaunchKernelGGL((k_blend_bwd<W_, H_, P_, false>), dim3(a.n_tiles), dim3(W_ * H_ / P_), 0, s, a.cams, a.B,
                           a.n_tiles, a.ranges, a.vals, a.recs, a.dl_dimg, a.t_final, a.n_last, a.acc, a.mask);
}

// every supported (tile_w, tile_h, pixels per lane)
#define MVGS_BLEND_CONFIGS(X) \
    X(8, 8, 1) X(16, 8, 1) X(32, 8, 1) \
    X(8, 16, 1) X(16, 16, 1) X(32, 16, 1) X(8, 16, 2) X(16, 16, 2) X(32, 16, 2) \
    X(8, 32, 1) X(16, 32, 1) X(32, 32, 1) X(8, 32, 2) X(16, 32, 2) X(32, 32, 2) \
    X(16, 16, 4) X(32, 16, 4) X(16, 32, 4) X(32, 32, 4)

void launch_blend_fwd(const BlendFwdArgs& a, int tw, int th, int ppl, hipStream_t s) {
    if (!a.n_tiles) return;
#define MVGS_F(W_, H_, P_) \
    if (tw == W_ && th == H_ && ppl == P_) { launch_fwd_t<W_, H_, P_>(a, s); return; }
    MVGS_BLEND_CONFIGS(MVGS_F)
#undef MVGS_F
}

void launch_blend_bwd(const BlendBwdArgs& a, int tw, int th, int ppl, hipStream_t s) {
    if (!a.n_tiles) return;
#define MVGS_B(W_, H_, P_) \
    if (tw == W_ && th == H_ && ppl == P_) { launch_bwd_t<W_, H_, P_>(a, s); return; }
    MVGS_BLEND_CONFIGS(MVGS_B)
#undef MVGS_B
}

}  // namespace mvgs
