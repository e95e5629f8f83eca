// Photometric loss and its image gradient (paper Sec. 3: L1 plus D-SSIM; Sec. 5.1.2, Eqs. 7-10).
//
//   L = w_l1 * mean |I - T| + w_dssim * (1 - mean SSIM(I, T)),  means over (view, channel, row, col)
// SSIM uses the 11x11 Gaussian window (sigma 1.5, normalised to sum 1, zero padding), which is the
// outer product of a normalised 11-tap 1D window, so every windowed moment is a separable
// convolution. The gradient of SSIM at pixel q gathers, over the windows containing q,
//   w(q - p) [dS/dmu1(p) + 2 I(q) dS/dE[I^2](p) + T(q) dS/dE[IT](p)],
// which is the same separable convolution applied to three per-pixel derivative maps.
// Partial sums are reduced in a fixed order, so the loss is deterministic.
#include <algorithm>
#include <cmath>

#include "mvgs_kernels.h"

namespace mvgs {

constexpr int kLossThreads = 256;
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Win11 {
    float w[11];
};

__device__ __forceinline__ int find_loss_view(const LossView* __restrict__ v, int B, uint32_t pix) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (v[mid].pix_base <= pix) lo = mid;
        else hi = mid;
    }
    return lo;
}

// L1 term: writes grad = w_l1 * sign(I - T) / N and one partial sum of |I - T| per block. Four
// consecutive pixels per thread, loaded and stored as float4 where they lie in one view at an
// aligned offset (one scalar pixel at a time elsewhere).
__device__ __forceinline__ float l1_sign(float d, float scale) { return d > 0.0f ? scale : (d < 0.0f ? -scale : 0.0f); }

__global__ void __launch_bounds__(kLossThreads) k_l1(const LossView* __restrict__ views, int B, uint32_t total,
                                                     float scale, float* __restrict__ partial) {
    __shared__ float red[kLossThreads / 64];
    const uint32_t p0 = (blockIdx.x * kLossThreads + threadIdx.x) * 4u;
    float s = 0.0f;
    if (p0 < total) {
        const int v = find_loss_view(views, B, p0);
        const LossView lv = views[v];
        const size_t hw = (size_t)lv.W * lv.H;
        const size_t i = p0 - lv.pix_base;
        const bool aligned = (((uintptr_t)lv.img | (uintptr_t)lv.tgt | (uintptr_t)lv.grad) & 15u) == 0;
        if (aligned && (hw & 3u) == 0 && (i & 3u) == 0 && i + 3 < hw) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float4 a = *reinterpret_cast<const float4*>(lv.img + ch * hw + i);
                const float4 t = *reinterpret_cast<const float4*>(lv.tgt + ch * hw + i);
                const float4 d = make_float4(a.x - t.x, a.y - t.y, a.z - t.z, a.w - t.w);
                s += fabsf(d.x) + fabsf(d.y) + fabsf(d.z) + fabsf(d.w);
                *reinterpret_cast<float4*>(lv.grad + ch * hw + i) =
                    make_float4(l1_sign(d.x, scale), l1_sign(d.y, scale), l1_sign(d.z, scale), l1_sign(d.w, scale));
            }
        } else {
            for (uint32_t p = p0; p < p0 + 4u && p < total; ++p) {
                const LossView lw = views[find_loss_view(views, B, p)];
                const size_t hw2 = (size_t)lw.W * lw.H, j = p - lw.pix_base;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float d = lw.img[ch * hw2 + j] - lw.tgt[ch * hw2 + j];
                    s += fabsf(d);
                    lw.grad[ch * hw2 + j] = l1_sign(d, scale);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// D-SSIM with L1, fused: one workgroup per 32x32 output tile of one channel of one view. The
// gradient at q needs the derivative maps over q's 11x11 window, and those need the moments over
// their own windows, so the workgroup stages the 52x52 input neighbourhood of I and T in LDS and
// keeps every intermediate there: the five moments along x (52 rows x 42 columns), then along y
// with SSIM and its three derivative maps on the 42x42 neighbourhood of the tile (zero outside the
// image: the sums run over image pixels only), then the derivative maps convolved along x and y.
// Each thread slides the 11-tap window (fused multiply-adds) over a run of consecutive outputs held
// in registers. HBM sees I and T read once (plus the halo, mostly from L2) and the gradient
// written once.
constexpr int kSsimTile = 32;
constexpr int kSsimA = kSsimTile + 10;   // derivative-map neighbourhood
constexpr int kSsimI = kSsimTile + 20;   // input neighbourhood
constexpr int kSsimThreads = 256;

struct SsimLds {
    union {
        float in[2][kSsimI][kSsimI];   // I and T
        float abc[3][kSsimA][kSsimA];  // derivative maps (after the moments along x)
    } u;
    union {
        float hs[2][kSsimI][kSsimA];   // moments along x (two at a time)
        float hb[3][kSsimA][kSsimTile];  // derivative maps along x
    } v;
    float red[2][kSsimThreads / 64];
};

__global__ void __launch_bounds__(kSsimThreads) k_ssim_fused(const float* __restrict__ img,
                                                             const float* __restrict__ tgt,
                                                             float* __restrict__ grad, int W, int H, int tiles_x,
                                                             Win11 win, float l1scale, float dscale,
                                                             float* __restrict__ partial, uint32_t part_base,
                                                             uint32_t n_parts) {
    __shared__ SsimLds L;
    const int ch = blockIdx.y;
    const int t = threadIdx.x;
    const int ty = (int)blockIdx.x / tiles_x, tx = (int)blockIdx.x - ty * tiles_x;
    const int x0 = tx * kSsimTile, y0 = ty * kSsimTile;
    const size_t hw = (size_t)W * H;
    const float* a = img + ch * hw;
    const float* b = tgt + ch * hw;
    float* gout = grad + ch * hw;
    // 1. I and T over rows y0 - 10 .. y0 + 41 and columns x0 - 10 .. x0 + 41 (zero outside)
    for (int e = t; e < kSsimI * kSsimI; e += kSsimThreads) {
        const int r = e / kSsimI, c = e - r * kSsimI;
        const int y = y0 - 10 + r, x = x0 - 10 + c;
        const bool in = x >= 0 && x < W && y >= 0 && y < H;
        const size_t q = (size_t)y * W + x;
        L.u.in[0][r][c] = in ? a[q] : 0.0f;
        L.u.in[1][r][c] = in ? b[q] : 0.0f;
    }
    __syncthreads();
    // 2.-3. the five moments along x (row r, columns j .. j + 6 of the 42 per task) and then along
    // y (column j, rows i .. i + 6 per task) at the 42x42 positions p = (x0 - 5 + j, y0 - 5 + i),
    // in three rounds (I and T; I^2 and T^2; I T) so that the moments along x take two maps of LDS
    // instead of five: the workgroup then fits four times per CU instead of twice
    float mom[5][7];
    int j = 0, i0 = 0;
    const bool task3 = t < kSsimA * 6;
    if (task3) {
        j = t / 6;
        i0 = (t - j * 6) * 7;
    }
#pragma unroll
    for (int round = 0; round < 3; ++round) {
        // one task per thread: row r, output columns j0 .. j0 + n - 1 (groups of 11, 11, 10, 10 of
        // the 42), the products I^2, T^2 or I T formed once per input
        if (t < kSsimI * 4) {
            const int r = t >> 2, g = t & 3;
            const int j0 = g < 2 ? 11 * g : 22 + 10 * (g - 2);
            const int n = g < 2 ? 11 : 10;
            float u[21], v[21];
#pragma unroll
            for (int k = 0; k < 21; ++k) {
                const bool ok = k < n + 10;
                u[k] = ok ? L.u.in[0][r][j0 + k] : 0.0f;
                v[k] = ok ? L.u.in[1][r][j0 + k] : 0.0f;
                if (round == 1) {
                    u[k] = u[k] * u[k];
                    v[k] = v[k] * v[k];
                } else if (round == 2) {
                    u[k] = u[k] * v[k];
                }
            }
#pragma unroll
            for (int jj = 0; jj < 11; ++jj) {
                float m0 = 0, m1 = 0;
#pragma unroll
                for (int k = 0; k < 11; ++k) {
                    m0 = __builtin_fmaf(win.w[k], u[jj + k], m0);
                    if (round < 2) m1 = __builtin_fmaf(win.w[k], v[jj + k], m1);
                }
                if (jj < n) {
                    L.v.hs[0][r][j0 + jj] = m0;
                    if (round < 2) L.v.hs[1][r][j0 + jj] = m1;
                }
            }
        }
        __syncthreads();
        if (task3) {
#pragma unroll
            for (int m = 0; m < (round < 2 ? 2 : 1); ++m) {
                float h[17];
#pragma unroll
                for (int k = 0; k < 17; ++k) h[k] = L.v.hs[m][i0 + k][j];
#pragma unroll
                for (int ii = 0; ii < 7; ++ii) {
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < 11; ++k) acc = __builtin_fmaf(win.w[k], h[ii + k], acc);
                    mom[2 * round + m][ii] = acc;
                }
            }
        }
        __syncthreads();   // (the maps are overwritten by the next round; after the last, the inputs are free)
    }
    // SSIM and its derivative maps; SSIM summed over the tile's own pixels
    float ssim_sum = 0.0f;
    if (task3) {
        // (the inputs are no longer read: the derivative maps take their place)
        const int px = x0 - 5 + j;
        const bool own_col = j >= 5 && j < 5 + kSsimTile && px < W;
#pragma unroll
        for (int ii = 0; ii < 7; ++ii) {
            const int i = i0 + ii, py = y0 - 5 + i;
            float dm0 = 0.0f, dm1 = 0.0f, dm2 = 0.0f;
            if (px >= 0 && px < W && py >= 0 && py < H) {
                const float mu1 = mom[0][ii], mu2 = mom[1][ii];
                const float s11 = mom[2][ii] - mu1 * mu1, s22 = mom[3][ii] - mu2 * mu2, s12 = mom[4][ii] - mu1 * mu2;
                const float A1 = 2.0f * mu1 * mu2 + kC1, A2 = 2.0f * s12 + kC2;
                const float B1 = mu1 * mu1 + mu2 * mu2 + kC1, B2 = s11 + s22 + kC2;
                const float iB = 1.0f / (B1 * B2);
                const float S = A1 * A2 * iB;
                dm0 = dscale * (2.0f * mu2 * (A2 - A1) * iB - 2.0f * mu1 * S * (1.0f / B1 - 1.0f / B2));
                dm1 = dscale * (-S / B2);
                dm2 = dscale * (2.0f * A1 * iB);
                if (own_col && i >= 5 && i < 5 + kSsimTile) ssim_sum += S;
            }
            L.u.abc[0][i][j] = dm0;
            L.u.abc[1][i][j] = dm1;
            L.u.abc[2][i][j] = dm2;
        }
    }
    __syncthreads();
    // 4. derivative maps along x: row i, output columns jq0 .. jq0 + n - 1 of the 32 (groups of
    // 6, 6, 5, 5, 5, 5: 252 tasks, one per thread)
    if (t < kSsimA * 6) {
        const int i = t / 6, g = t - i * 6;
        const int jq0 = g < 2 ? 6 * g : 12 + 5 * (g - 2);
        const int n = g < 2 ? 6 : 5;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float h[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) h[k] = k < n + 10 ? L.u.abc[c][i][jq0 + k] : 0.0f;
#pragma unroll
            for (int jj = 0; jj < 6; ++jj) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < 11; ++k) acc = __builtin_fmaf(win.w[k], h[jj + k], acc);
                if (jj < n) L.v.hb[c][i][jq0 + jj] = acc;
            }
        }
    }
    __syncthreads();
    // 5. along y, and the gradient dL/dI(q) = L1 term + s0 + 2 I s1 + T s2: column jq, rows
    // iq .. iq + 3 of the 32
    float l1_sum = 0.0f;
    {
        const int jq = t & 31, iq0 = (t >> 5) * 4;
        float s[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float h[14];
#pragma unroll
            for (int k = 0; k < 14; ++k) h[k] = L.v.hb[c][iq0 + k][jq];
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                float acc = 0.0f;
#pragma unroll
                for (int k = 0; k < 11; ++k) acc = __builtin_fmaf(win.w[k], h[ii + k], acc);
                s[c][ii] = acc;
            }
        }
        const int x = x0 + jq;
        if (x < W) {
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
                const int y = y0 + iq0 + ii;
                if (y < H) {
                    const size_t q = (size_t)y * W + x;
                    const float I = a[q], T = b[q], d = I - T;
                    l1_sum += fabsf(d);
                    gout[q] = l1_sign(d, l1scale) + (s[0][ii] + 2.0f * I * s[1][ii] + T * s[2][ii]);
                }
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        l1_sum += __shfl_down(l1_sum, o, 64);
        ssim_sum += __shfl_down(ssim_sum, o, 64);
    }
    if ((t & 63) == 0) {
        L.red[0][t >> 6] = l1_sum;
        L.red[1][t >> 6] = ssim_sum;
    }
    __syncthreads();
    if (t == 0) {
        const uint32_t k = part_base + blockIdx.y * gridDim.x + blockIdx.x;
        partial[k] = L.red[0][0] + L.red[0][1] + L.red[0][2] + L.red[0][3];
        partial[n_parts + k] = L.red[1][0] + L.red[1][1] + L.red[1][2] + L.red[1][3];
    }
}

// Deterministic reduction in two stages. First, each workgroup adds kReduceChunk consecutive
// partials of the concatenation [l1 partials | ssim partials] into two doubles (one per kind).
constexpr uint32_t kReduceChunk = 4096;

__global__ void __launch_bounds__(256) k_loss_reduce(const float* __restrict__ partials, uint32_t n_l1,
                                                     uint32_t n, double* __restrict__ out) {
    __shared__ double red[2][4];
    double a = 0.0, b = 0.0;
    const uint32_t c0 = blockIdx.x * kReduceChunk, c1 = min(n, c0 + kReduceChunk);
    for (uint32_t i = c0 + threadIdx.x; i < c1; i += 256) {
        const double v = (double)partials[i];
        if (i < n_l1) a += v;
        else b += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_down(a, o, 64);
        b += __shfl_down(b, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = a;
        red[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        out[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Then loss = w_l1 * sum(l1 partials) / N + w_dssim * (1 - sum(ssim partials) / N).
__global__ void __launch_bounds__(256) k_loss_final(const double* __restrict__ chunks, uint32_t n_chunks,
                                                    double inv_n, float w_l1, float w_dssim, float* __restrict__ out) {
    __shared__ double red[2][256];
    double a = 0.0, b = 0.0;
    for (uint32_t i = threadIdx.x; i < n_chunks; i += 256) {
        a += chunks[2 * i];
        b += chunks[2 * i + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double l = (double)w_l1 * red[0][0] * inv_n;
        if (w_dssim != 0.0f) l += (double)w_dssim * (1.0 - red[1][0] * inv_n);
        *out = (float)l;
    }
}

static Win11 gaussian_window() {
    Win11 w;
    double e[11], s = 0.0;
    for (int k = 0; k < 11; ++k) {
        const double u = k - 5;
        e[k] = std::exp(-u * u / (2.0 * 1.5 * 1.5));
        s += e[k];
    }
    for (int k = 0; k < 11; ++k) w.w[k] = (float)(e[k] / s);
    return w;
}

uint32_t ssim_tiles(int W, int H) {
    return (uint32_t)((W + kSsimTile - 1) / kSsimTile) * (uint32_t)((H + kSsimTile - 1) / kSsimTile);
}

size_t loss_scratch_bytes(uint32_t total_pixels, uint64_t ssim_tiles_total) {
    // float partials (L1 blocks, or an L1 and an SSIM sum per channel tile), then (8-byte aligned)
    // two doubles per reduction chunk
    const size_t n_l1 = (total_pixels + 4 * kLossThreads - 1) / (4 * kLossThreads);
    const size_t n_part = std::max<size_t>(n_l1, 6 * (size_t)ssim_tiles_total);
    return (n_part + 64) * sizeof(float) + 2 * sizeof(double) * (n_part / kReduceChunk + 2);
}

// The view table written by a kernel from its arguments (no host staging buffer, so the launch also
// works where the caller may not allocate).
struct LossViewArgs {
    LossView v[kLossArgViews];
};

__global__ void k_put_loss_views(LossViewArgs a, int B, LossView* __restrict__ dst) {
    if ((int)threadIdx.x < B) dst[threadIdx.x] = a.v[threadIdx.x];
}

void launch_put_loss_views(const LossView* views, int B, LossView* dst, hipStream_t s) {
    LossViewArgs a{};
    for (int v = 0; v < B && v < kLossArgViews; ++v) a.v[v] = views[v];
    hipLaunchKernelGGL(k_put_loss_views, dim3(1), dim3(64), 0, s, a, B, dst);
}

void launch_loss(const LossView* views_dev, const LossView* views_host, int B, uint32_t total_pixels, float w_l1,
                 float w_dssim, float* loss_out, void* scratch, hipStream_t s) {
    const double N = 3.0 * (double)total_pixels;
    float* partial = (float*)scratch;
    uint32_t n_l1, n_part;
    if (w_dssim == 0.0f) {
        n_l1 = n_part = (total_pixels + 4 * kLossThreads - 1) / (4 * kLossThreads);
        hipLaunchKernelGGL(k_l1, dim3(n_l1), dim3(kLossThreads), 0, s, views_dev, B, total_pixels,
                           (float)(w_l1 / N), partial);
    } else {
        // one L1 and one SSIM partial per (view, channel, tile), L1 ones first
        uint32_t n_s = 0;
        for (int v = 0; v < B; ++v) n_s += 3 * ssim_tiles(views_host[v].W, views_host[v].H);
        const Win11 win = gaussian_window();
        uint32_t base = 0;
        for (int v = 0; v < B; ++v) {
            const LossView& lv = views_host[v];
            const uint32_t nt = ssim_tiles(lv.W, lv.H);
            const int tiles_x = (lv.W + kSsimTile - 1) / kSsimTile;
            hipLaunchKernelGGL(k_ssim_fused, dim3(nt, 3), dim3(kSsimThreads), 0, s, lv.img, lv.tgt, lv.grad, lv.W,
                               lv.H, tiles_x, win, (float)(w_l1 / N), (float)(-(double)w_dssim / N), partial, base,
                               n_s);
            base += 3 * nt;
        }
        n_l1 = n_s;
        n_part = 2 * n_s;
    }
    const uint32_t n_chunks = (n_part + kReduceChunk - 1) / kReduceChunk;
    double* chunks = reinterpret_cast<double*>(((uintptr_t)(partial + n_part) + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_loss_reduce, dim3(n_chunks), dim3(256), 0, s, (const float*)partial, n_l1, n_part, chunks);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (const double*)chunks, n_chunks, 1.0 / N, w_l1,
                       w_dssim, loss_out);
}

}  // namespace mvgs
