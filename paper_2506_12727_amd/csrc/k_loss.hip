// Photometric loss and its image gradient (paper Sec. 3: L1 plus D-SSIM; Sec. 5.1.2, Eqs. 7-10).
//
//   L = w_l1 * mean |I - T| + w_dssim * (1 - mean SSIM(I, T)),  means over (view, channel, row, col)
// SSIM uses the 11x11 Gaussian window (sigma 1.5, normalised to sum 1, zero padding), which is the
// outer product of a normalised 11-tap 1D window, so every windowed moment is a separable
// convolution. The gradient of SSIM at pixel q gathers, over the windows containing q,
//   w(q - p) [dS/dmu1(p) + 2 I(q) dS/dE[I^2](p) + T(q) dS/dE[IT](p)],
// which is the same separable convolution applied to three per-pixel derivative maps.
// Partial sums are reduced in a fixed order, so the loss is deterministic.
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

// Horizontal pass: 5 windowed sums (I, T, I^2, T^2, IT) along x. Grid (blocks, 3 channels).
__global__ void __launch_bounds__(kLossThreads) k_ssim_h(const float* __restrict__ img, const float* __restrict__ tgt,
                                                         int W, int H, Win11 win, float* __restrict__ out) {
    const int ch = blockIdx.y;
    const size_t hw = (size_t)W * H;
    const uint32_t p = blockIdx.x * kLossThreads + threadIdx.x;
    if (p >= hw) return;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * W);
    const float* a = img + ch * hw + (size_t)y * W;
    const float* b = tgt + ch * hw + (size_t)y * W;
    float m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int xx = x + k - 5;
        if (xx < 0 || xx >= W) continue;
        const float u = a[xx], v = b[xx], w = win.w[k];
        m0 += w * u;
        m1 += w * v;
        m2 += w * u * u;
        m3 += w * v * v;
        m4 += w * u * v;
    }
    float* o = out + (size_t)ch * 5 * hw;
    o[p] = m0;
    o[hw + p] = m1;
    o[2 * hw + p] = m2;
    o[3 * hw + p] = m3;
    o[4 * hw + p] = m4;
}

// Vertical pass: moments -> SSIM (one partial sum per block) and the three derivative maps,
// pre-multiplied by dL/dSSIM = -w_dssim / N.
__global__ void __launch_bounds__(kLossThreads) k_ssim_v(const float* __restrict__ hsum, int W, int H, Win11 win,
                                                         float dscale, float* __restrict__ dmaps,
                                                         float* __restrict__ partial) {
    __shared__ float red[kLossThreads];
    const int ch = blockIdx.y;
    const size_t hw = (size_t)W * H;
    const uint32_t p = blockIdx.x * kLossThreads + threadIdx.x;
    float S = 0.0f;
    if (p < hw) {
        const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * W);
        const float* h = hsum + (size_t)ch * 5 * hw;
        float m[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int yy = y + k - 5;
            if (yy < 0 || yy >= H) continue;
            const size_t q = (size_t)yy * W + x;
            const float w = win.w[k];
#pragma unroll
            for (int j = 0; j < 5; ++j) m[j] += w * h[j * hw + q];
        }
        const float mu1 = m[0], mu2 = m[1];
        const float s11 = m[2] - mu1 * mu1, s22 = m[3] - mu2 * mu2, s12 = m[4] - mu1 * mu2;
        const float A1 = 2.0f * mu1 * mu2 + kC1, A2 = 2.0f * s12 + kC2;
        const float B1 = mu1 * mu1 + mu2 * mu2 + kC1, B2 = s11 + s22 + kC2;
        const float iB = 1.0f / (B1 * B2);
        S = A1 * A2 * iB;
        const float d_mu1 = 2.0f * mu2 * (A2 - A1) * iB - 2.0f * mu1 * S * (1.0f / B1 - 1.0f / B2);
        const float d_m11 = -S / B2;
        const float d_m12 = 2.0f * A1 * iB;
        float* d = dmaps + (size_t)ch * 3 * hw;
        d[p] = dscale * d_mu1;
        d[hw + p] = dscale * d_m11;
        d[2 * hw + p] = dscale * d_m12;
    }
    red[threadIdx.x] = S;
    __syncthreads();
    for (int off = kLossThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Backward horizontal pass over the three derivative maps.
__global__ void __launch_bounds__(kLossThreads) k_ssim_bh(const float* __restrict__ dmaps, int W, int H, Win11 win,
                                                          float* __restrict__ out) {
    const int ch = blockIdx.y;
    const size_t hw = (size_t)W * H;
    const uint32_t p = blockIdx.x * kLossThreads + threadIdx.x;
    if (p >= hw) return;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * W);
    const float* d = dmaps + (size_t)ch * 3 * hw + (size_t)y * W;
    float s[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int xx = x + k - 5;
        if (xx < 0 || xx >= W) continue;
        const float w = win.w[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) s[j] += w * d[j * hw + xx];
    }
    float* o = out + (size_t)ch * 3 * hw;
#pragma unroll
    for (int j = 0; j < 3; ++j) o[j * hw + p] = s[j];
}

// Backward vertical pass and combination into the image gradient (added to the L1 part).
__global__ void __launch_bounds__(kLossThreads) k_ssim_bv(const float* __restrict__ hmaps,
                                                          const float* __restrict__ img,
                                                          const float* __restrict__ tgt, int W, int H, Win11 win,
                                                          float* __restrict__ grad) {
    const int ch = blockIdx.y;
    const size_t hw = (size_t)W * H;
    const uint32_t p = blockIdx.x * kLossThreads + threadIdx.x;
    if (p >= hw) return;
    const int y = (int)(p / (uint32_t)W), x = (int)(p - (uint32_t)y * W);
    const float* h = hmaps + (size_t)ch * 3 * hw;
    float s[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const int yy = y + k - 5;
        if (yy < 0 || yy >= H) continue;
        const size_t q = (size_t)yy * W + x;
        const float w = win.w[k];
#pragma unroll
        for (int j = 0; j < 3; ++j) s[j] += w * h[j * hw + q];
    }
    const size_t i = ch * hw + p;
    grad[i] += s[0] + 2.0f * img[i] * s[1] + tgt[i] * s[2];
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

size_t loss_scratch_bytes(uint32_t total_pixels, int B) {
    // partials (l1 + ssim) then, per view in turn, 8 maps per channel of the largest view
    (void)B;
    const size_t n_l1 = (total_pixels + kLossThreads - 1) / kLossThreads;
    const size_t n_part = n_l1 + 3 * (size_t)total_pixels / kLossThreads + 3 * (size_t)B;
    // float partials, then (8-byte aligned) two doubles per reduction chunk
    return (n_part + 64) * sizeof(float) + 2 * sizeof(double) * (n_part / kReduceChunk + 2);
}

size_t ssim_map_bytes(uint32_t max_view_pixels) { return (size_t)max_view_pixels * 3 * 8 * sizeof(float); }

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
                 float w_dssim, float* loss_out, void* scratch, void* maps, hipStream_t s) {
    const double N = 3.0 * (double)total_pixels;
    float* partial = (float*)scratch;
    const uint32_t n_l1 = (total_pixels + 4 * kLossThreads - 1) / (4 * kLossThreads);
    hipLaunchKernelGGL(k_l1, dim3(n_l1), dim3(kLossThreads), 0, s, views_dev, B, total_pixels, (float)(w_l1 / N),
                       partial);
    float* sp = partial + n_l1;
    uint32_t n_s = 0;
    if (w_dssim != 0.0f) {
        const Win11 win = gaussian_window();
        for (int v = 0; v < B; ++v) {
            const LossView& lv = views_host[v];
            const uint32_t hw = (uint32_t)lv.W * (uint32_t)lv.H;
            const uint32_t nb = (hw + kLossThreads - 1) / kLossThreads;
            float* hsum = (float*)maps;                       // 5 maps x 3 channels
            float* dm = hsum + (size_t)15 * hw;                // 3 maps x 3 channels
            hipLaunchKernelGGL(k_ssim_h, dim3(nb, 3), dim3(kLossThreads), 0, s, lv.img, lv.tgt, lv.W, lv.H, win,
                               hsum);
            hipLaunchKernelGGL(k_ssim_v, dim3(nb, 3), dim3(kLossThreads), 0, s, (const float*)hsum, lv.W, lv.H, win,
                               (float)(-(double)w_dssim / N), dm, sp + n_s);
            n_s += 3 * nb;
            float* hb = hsum;  // the moment maps are no longer needed
            hipLaunchKernelGGL(k_ssim_bh, dim3(nb, 3), dim3(kLossThreads), 0, s, (const float*)dm, lv.W, lv.H, win,
                               hb);
            hipLaunchKernelGGL(k_ssim_bv, dim3(nb, 3), dim3(kLossThreads), 0, s, (const float*)hb, lv.img, lv.tgt,
                               lv.W, lv.H, win, lv.grad);
        }
    }
    const uint32_t n_part = n_l1 + n_s;
    const uint32_t n_chunks = (n_part + kReduceChunk - 1) / kReduceChunk;
    double* chunks = reinterpret_cast<double*>(((uintptr_t)(partial + n_part) + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_loss_reduce, dim3(n_chunks), dim3(256), 0, s, (const float*)partial, n_l1, n_part, chunks);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (const double*)chunks, n_chunks, 1.0 / N, w_l1,
                       w_dssim, loss_out);
}

}  // namespace mvgs
