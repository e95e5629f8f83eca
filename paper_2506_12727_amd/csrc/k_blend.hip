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
#include "mvgs_kernels.h"

namespace mvgs {

constexpr float kLog2e = 1.4426950408889634f;

// Contiguous tile runs per XCD: block b is dispatched to XCD b % 8.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t q = n >> 3, rem = n & 7u;
    return x * q + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ int find_view(const DevCam* __restrict__ cams, int B, uint32_t tile) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cams[mid].tile_base <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool box_misses(uint32_t bx, uint32_t by, int sx0, int sx1, int sy0, int sy1) {
    return (int)(bx & 0xffffu) > sx1 || (int)(bx >> 16) < sx0 || (int)(by & 0xffffu) > sy1 || (int)(by >> 16) < sy0;
}

__device__ __forceinline__ float fast_exp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }

// Wavefront-uniform copy of the fields the walks use.
struct RecS {
    float mx, my, hca, nb, hcc, o, cut, hi, r, g, b;
};

__device__ __forceinline__ RecS load_rec(const BlendRec* __restrict__ recs, uint32_t r) {
    const BlendRec* R = recs + r;
    RecS s;
    s.mx = R->mx; s.my = R->my; s.hca = R->hca; s.nb = R->nb; s.hcc = R->hcc; s.o = R->o;
    s.cut = R->cut; s.hi = R->hi; s.r = R->r; s.g = R->g; s.b = R->b;
    return s;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Candidate window: lane k looks at list entry base + k, loads its record index and pixel box with
// one vector load each, and the ballot keeps the entries whose box meets the wavefront's sub-tile.
__device__ __forceinline__ uint64_t window_mask(const uint32_t* __restrict__ vals, const BlendRec* __restrict__ recs,
                                                uint32_t base, uint32_t end, int lane, int sx0, int sx1, int sy0,
                                                int sy1, uint32_t& rl) {
    const uint32_t idx = base + (uint32_t)lane;
    bool keep = false;
    rl = 0;
    if (idx < end) {
        rl = vals[idx];
        const uint2 bx = *reinterpret_cast<const uint2*>(recs + rl);
        keep = !box_misses(bx.x, bx.y, sx0, sx1, sy0, sy1);
    }
    return ballot64(keep);
}

struct FwdState {
    float T, C0, C1, C2;
    uint32_t last;
    bool done;
};

__device__ __forceinline__ void blend_step(FwdState& st, const RecS& q, float px, float py, uint32_t pos) {
    if (st.done) return;
    const float power = pixel_power(px, py, q.mx, q.my, q.hca, q.nb, q.hcc);
    if (power >= q.cut) {
        const float alpha = (power > q.hi) ? kAlphaMax : q.o * fast_exp(power);
        const float Tn = __builtin_fmaf(-st.T, alpha, st.T);
        if (Tn < kTStop) {
            st.done = true;
        } else {
            const float w = alpha * st.T;
            st.C0 = __builtin_fmaf(q.r, w, st.C0);
            st.C1 = __builtin_fmaf(q.g, w, st.C1);
            st.C2 = __builtin_fmaf(q.b, w, st.C2);
            st.T = Tn;
            st.last = pos + 1;
        }
    }
}

template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH) k_blend_fwd(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                       const uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ vals,
                                                       const BlendRec* __restrict__ recs,
                                                       float* const* __restrict__ images,
                                                       float* __restrict__ t_final, uint32_t* __restrict__ n_last) {
    constexpr int WX = TW / 8;
    const uint32_t tile = xcd_tile(blockIdx.x, n_tiles);
    const int v = find_view(cams, B, tile);
    const DevCam& c = cams[v];
    const uint32_t local = tile - c.tile_base;
    const int ty = (int)(local / (uint32_t)c.tiles_x);
    const int tx = (int)local - ty * c.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int sx0 = tx * TW + (wave % WX) * 8, sy0 = ty * TH + (wave / WX) * 8;
    if (sx0 >= c.W || sy0 >= c.H) return;
    const int sx1 = min(sx0 + 7, c.W - 1), sy1 = min(sy0 + 7, c.H - 1);
    const int x = sx0 + (lane & 7), y = sy0 + (lane >> 3);
    const bool valid = x < c.W && y < c.H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint2 rg = ranges[tile];

    FwdState st{1.0f, 0.0f, 0.0f, 0.0f, 0u, !valid};
    for (uint32_t base = rg.x; base < rg.y; base += 64) {
        if (ballot64(!st.done) == 0) break;
        uint32_t rl;
        uint64_t m = window_mask(vals, recs, base, rg.y, lane, sx0, sx1, sy0, sy1, rl);
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
            blend_step(st, q0, px, py, base + (uint32_t)j0);
            if (h1) blend_step(st, q1, px, py, base + (uint32_t)j1);
            if (h2) blend_step(st, q2, px, py, base + (uint32_t)j2);
            if (h3) blend_step(st, q3, px, py, base + (uint32_t)j3);
        }
    }
    if (valid) {
        const size_t hw = (size_t)c.W * c.H;
        const size_t pix = (size_t)y * c.W + x;
        float* img = images[v];
        img[pix] = __builtin_fmaf(st.T, c.bg[0], st.C0);
        img[hw + pix] = __builtin_fmaf(st.T, c.bg[1], st.C1);
        img[2 * hw + pix] = __builtin_fmaf(st.T, c.bg[2], st.C2);
        t_final[c.pix_base + pix] = st.T;
        n_last[c.pix_base + pix] = st.last;
    }
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}

struct BwdState {
    float T, dC0, dC1, dC2, Rb0, Rb1, Rb2;
    uint32_t last;
};

// One Gaussian of the reverse walk: this lane's contributions, summed over the wavefront and
// added to the record's accumulators.
template <bool E1>
__device__ __forceinline__ void unblend_step(BwdState& st, const RecS& q, uint32_t r, uint32_t pos, float px,
                                             float py, float half_w, float half_h, int lane,
                                             float* __restrict__ acc) {
    float g_mx = 0.f, g_my = 0.f, g_ca = 0.f, g_cb = 0.f, g_cc = 0.f, g_o = 0.f;
    float g_r = 0.f, g_g = 0.f, g_b = 0.f, g_e1 = 0.f;
    bool contrib = false;
    if (pos < st.last) {
        const float dx = px - q.mx, dy = py - q.my;
        const float power = pixel_power(px, py, q.mx, q.my, q.hca, q.nb, q.hcc);
        if (power >= q.cut) {
            contrib = true;
            const bool clamped = power > q.hi;
            const float G = fast_exp(power);
            const float alpha = clamped ? kAlphaMax : q.o * G;
            st.T = st.T * __builtin_amdgcn_rcpf(1.0f - alpha);   // transmittance in front of this Gaussian
            const float w = alpha * st.T;
            g_r = st.dC0 * w;
            g_g = st.dC1 * w;
            g_b = st.dC2 * w;
            const float dalpha = st.T * (st.dC0 * (q.r - st.Rb0) + st.dC1 * (q.g - st.Rb1) + st.dC2 * (q.b - st.Rb2));
            st.Rb0 = __builtin_fmaf(q.r - st.Rb0, alpha, st.Rb0);
            st.Rb1 = __builtin_fmaf(q.g - st.Rb1, alpha, st.Rb1);
            st.Rb2 = __builtin_fmaf(q.b - st.Rb2, alpha, st.Rb2);
            if (!clamped) {
                g_o = dalpha * G;
                const float dpow = dalpha * alpha;
                const float ca = -2.0f * q.hca, cbq = -q.nb, cc = -2.0f * q.hcc;
                g_mx = dpow * (ca * dx + cbq * dy);
                g_my = dpow * (cbq * dx + cc * dy);
                g_ca = -0.5f * dpow * dx * dx;
                g_cb = -dpow * dx * dy;
                g_cc = -0.5f * dpow * dy * dy;
                if (E1) {
                    const float nx = g_mx * half_w, ny = g_my * half_h;
                    g_e1 = sqrtf(nx * nx + ny * ny);
                }
            }
        }
    }
    if (ballot64(contrib) == 0) return;
    const float s0 = wave_sum(g_mx), s1 = wave_sum(g_my), s2 = wave_sum(g_ca), s3 = wave_sum(g_cb);
    const float s4 = wave_sum(g_cc), s5 = wave_sum(g_o), s6 = wave_sum(g_r), s7 = wave_sum(g_g);
    const float s8 = wave_sum(g_b);
    const float s9 = E1 ? wave_sum(g_e1) : 0.0f;
    float val = s0;
    val = lane == 1 ? s1 : val;
    val = lane == 2 ? s2 : val;
    val = lane == 3 ? s3 : val;
    val = lane == 4 ? s4 : val;
    val = lane == 5 ? s5 : val;
    val = lane == 6 ? s6 : val;
    val = lane == 7 ? s7 : val;
    val = lane == 8 ? s8 : val;
    val = lane == 9 ? s9 : val;
    if (lane < (E1 ? 10 : 9)) unsafeAtomicAdd(acc + (size_t)r * kAccStride + lane, val);
}

template <int TW, int TH, bool E1>
__global__ void __launch_bounds__(TW * TH) k_blend_bwd(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                       const uint2* __restrict__ ranges,
                                                       const uint32_t* __restrict__ vals,
                                                       const BlendRec* __restrict__ recs,
                                                       const float* const* __restrict__ dl_dimg,
                                                       const float* __restrict__ t_final,
                                                       const uint32_t* __restrict__ n_last,
                                                       float* __restrict__ acc) {
    constexpr int WX = TW / 8;
    const uint32_t tile = xcd_tile(blockIdx.x, n_tiles);
    const int v = find_view(cams, B, tile);
    const DevCam& c = cams[v];
    const uint32_t local = tile - c.tile_base;
    const int ty = (int)(local / (uint32_t)c.tiles_x);
    const int tx = (int)local - ty * c.tiles_x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int sx0 = tx * TW + (wave % WX) * 8, sy0 = ty * TH + (wave / WX) * 8;
    if (sx0 >= c.W || sy0 >= c.H) return;
    const int sx1 = min(sx0 + 7, c.W - 1), sy1 = min(sy0 + 7, c.H - 1);
    const int x = sx0 + (lane & 7), y = sy0 + (lane >> 3);
    const bool valid = x < c.W && y < c.H;
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const uint2 rg = ranges[tile];
    const float half_w = 0.5f * (float)c.W, half_h = 0.5f * (float)c.H;

    BwdState st{1.0f, 0.0f, 0.0f, 0.0f, c.bg[0], c.bg[1], c.bg[2], 0u};
    if (valid) {
        const size_t hw = (size_t)c.W * c.H;
        const size_t pix = (size_t)y * c.W + x;
        const float* g = dl_dimg[v];
        st.dC0 = g[pix];
        st.dC1 = g[hw + pix];
        st.dC2 = g[2 * hw + pix];
        st.T = t_final[c.pix_base + pix];
        st.last = n_last[c.pix_base + pix];
    }
    const uint32_t hi_end = __builtin_amdgcn_readfirstlane(wave_max_u32(st.last));

    for (uint32_t top = hi_end; top > rg.x;) {
        const uint32_t base = top - rg.x > 64u ? top - 64u : rg.x;
        uint32_t rl;
        uint64_t m = window_mask(vals, recs, base, top, lane, sx0, sx1, sy0, sy1, rl);
        top = base;
        while (m) {
            // highest list position first; up to four records per round trip
            const int j0 = 63 - __builtin_clzll(m);
            m &= ~(1ull << j0);
            const int j1 = m ? 63 - __builtin_clzll(m) : j0;
            if (m) m &= ~(1ull << j1);
            const bool h1 = j1 != j0;
            const int j2 = m ? 63 - __builtin_clzll(m) : j0;
            if (m) m &= ~(1ull << j2);
            const bool h2 = j2 != j0;
            const int j3 = m ? 63 - __builtin_clzll(m) : j0;
            if (m) m &= ~(1ull << j3);
            const bool h3 = j3 != j0;
            const uint32_t r0 = readlane_u32(rl, j0), r1 = readlane_u32(rl, j1);
            const uint32_t r2 = readlane_u32(rl, j2), r3 = readlane_u32(rl, j3);
            const RecS q0 = load_rec(recs, r0);
            const RecS q1 = load_rec(recs, r1);
            const RecS q2 = load_rec(recs, r2);
            const RecS q3 = load_rec(recs, r3);
            unblend_step<E1>(st, q0, r0, base + (uint32_t)j0, px, py, half_w, half_h, lane, acc);
            if (h1) unblend_step<E1>(st, q1, r1, base + (uint32_t)j1, px, py, half_w, half_h, lane, acc);
            if (h2) unblend_step<E1>(st, q2, r2, base + (uint32_t)j2, px, py, half_w, half_h, lane, acc);
            if (h3) unblend_step<E1>(st, q3, r3, base + (uint32_t)j3, px, py, half_w, half_h, lane, acc);
        }
    }
}

// sum over pixels of (last blended list position + 1 - list start): the reverse walk's steps
__global__ void __launch_bounds__(256) k_frame_work(const DevCam* __restrict__ cams, int B,
                                                    const uint2* __restrict__ ranges,
                                                    const uint32_t* __restrict__ n_last, uint32_t n_pixels, int tw,
                                                    int th, unsigned long long* __restrict__ steps) {
    __shared__ unsigned long long red[256];
    const uint32_t p = blockIdx.x * 256 + threadIdx.x;
    unsigned long long w = 0;
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
        w = nl > start ? (unsigned long long)(nl - start) : 0ull;
    }
    red[threadIdx.x] = w;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(steps, red[0]);
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

void launch_frame_work(const DevCam* cams, int B, const uint2* ranges, const uint32_t* n_last, uint32_t n_pixels,
                       int tw, int th, uint64_t* steps, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, (unsigned long long*)steps);
    if (!n_pixels) return;
    hipLaunchKernelGGL(k_frame_work, dim3((n_pixels + 255) / 256), dim3(256), 0, s, cams, B, ranges, n_last,
                       n_pixels, tw, th, (unsigned long long*)steps);
}

bool blend_supported(int tw, int th) {
    const bool okw = tw == 8 || tw == 16 || tw == 32;
    const bool okh = th == 8 || th == 16 || th == 32;
    return okw && okh;
}

#define MVGS_TILE_SWITCH(TWv, THv, CALL)               \
    do {                                                \
        if (TWv == 8 && THv == 8) { CALL(8, 8); }       \
        else if (TWv == 16 && THv == 8) { CALL(16, 8); }   \
        else if (TWv == 8 && THv == 16) { CALL(8, 16); }   \
        else if (TWv == 16 && THv == 16) { CALL(16, 16); } \
        else if (TWv == 32 && THv == 8) { CALL(32, 8); }   \
        else if (TWv == 8 && THv == 32) { CALL(8, 32); }   \
        else if (TWv == 32 && THv == 16) { CALL(32, 16); } \
        else if (TWv == 16 && THv == 32) { CALL(16, 32); } \
        else { CALL(32, 32); }                          \
    } while (0)

void launch_blend_fwd(const BlendFwdArgs& a, int tw, int th, hipStream_t s) {
    if (!a.n_tiles) return;
#define MVGS_BF(W_, H_)                                                                                        \
    hipLaunchKernelGGL((k_blend_fwd<W_, H_>), dim3(a.n_tiles), dim3(W_ * H_), 0, s, a.cams, a.B, a.n_tiles,    \
                       a.ranges, a.vals, a.recs, a.images, a.t_final, a.n_last)
    MVGS_TILE_SWITCH(tw, th, MVGS_BF);
#undef MVGS_BF
}

void launch_blend_bwd(const BlendBwdArgs& a, int tw, int th, hipStream_t s) {
    if (!a.n_tiles) return;
#define MVGS_BB(W_, H_)                                                                                        \
    do {                                                                                                       \
        if (a.want_e1)                                                                                         \
            hipLaunchKernelGGL((k_blend_bwd<W_, H_, true>), dim3(a.n_tiles), dim3(W_ * H_), 0, s, a.cams, a.B, \
                               a.n_tiles, a.ranges, a.vals, a.recs, a.dl_dimg, a.t_final, a.n_last, a.acc);    \
        else                                                                                                   \
            hipLaunchKernelGGL((k_blend_bwd<W_, H_, false>), dim3(a.n_tiles), dim3(W_ * H_), 0, s, a.cams,     \
                               a.B, a.n_tiles, a.ranges, a.vals, a.recs, a.dl_dimg, a.t_final, a.n_last,      \
                               a.acc);                                                                         \
    } while (0)
    MVGS_TILE_SWITCH(tw, th, MVGS_BB);
#undef MVGS_BB
}

}  // namespace mvgs
