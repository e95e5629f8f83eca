// 3D distance-aware D-SSIM (paper Sec. 5.1.2, Eqs. 7-11) on the merged image plane of a
// thread-efficient partial render, with L1, and the image gradient.
//
// Every pixel of the plane was rendered from one view of the batch. Its surface point is the
// blended depth over the blended opacity along that view's camera ray, mapped to world space; the
// SSIM window around a centre weighs each neighbour by a Gaussian of the 3D distance between their
// points, with sigma 1.5 pixels taken at the centre's depth, normalised over the in-plane window.
// Neighbours from other views, or far away in depth, thus get little weight. The weights are
// constants of the loss (no gradient reaches the depth).
//
// Three passes over the plane: points (double precision, so that differences of neighbouring
// points do not cancel), then per centre the weighted moments, SSIM, the loss partial sums and
// three coefficients per channel with dSSIM(c)/dI(q) = w_cq (a_c + b_c I(q) + d_c T(q)); then per
// pixel the sum of those terms over the centres whose window holds it.
#include "mvgs_kernels.h"

namespace mvgs {

constexpr int kWin = 5;                 // window radius: 11 x 11
constexpr float kSigmaPx = 1.5f;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

// One wavefront per selection segment: the surface point of each of its pixels, stored at the
// pixel's plane position as (x, y, z, scale); scale 0 marks a pixel where nothing was blended.
__global__ void __launch_bounds__(256) k_points3d(const DevCam* __restrict__ cams, int B, uint32_t n_tiles,
                                                  const uint32_t* __restrict__ sel_off,
                                                  const uint32_t* __restrict__ sel_pix,
                                                  const float* __restrict__ t_sel, const float* __restrict__ depth_sel,
                                                  double4* __restrict__ pts, const uint32_t* __restrict__ void_word) {
    const uint32_t t = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (t >= n_tiles || (void_word && *void_word)) return;
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cams[mid].tile_base <= t) lo = mid;
        else hi = mid;
    }
    const DevCam& c = cams[lo];
    for (uint32_t i = sel_off[t] + (threadIdx.x & 63u); i < sel_off[t + 1]; i += 64u) {
        const uint32_t p = sel_pix[i];
        const double a = 1.0 - (double)t_sel[i];
        double4 out = make_double4(0.0, 0.0, 0.0, 0.0);
        if (a > 0.0) {
            const int y = (int)(p / (uint32_t)c.W), x = (int)(p - (uint32_t)y * (uint32_t)c.W);
            const double z = (double)depth_sel[i] / a;
            const double cx = z * (((double)x + 0.5 - (double)c.cx) / (double)c.fx) - (double)c.t[0];
            const double cy = z * (((double)y + 0.5 - (double)c.cy) / (double)c.fy) - (double)c.t[1];
            const double cz = z - (double)c.t[2];
            // world = R^T (camera - t)
            out.x = (double)c.R[0] * cx + (double)c.R[3] * cy + (double)c.R[6] * cz;
            out.y = (double)c.R[1] * cx + (double)c.R[4] * cy + (double)c.R[7] * cz;
            out.z = (double)c.R[2] * cx + (double)c.R[5] * cy + (double)c.R[8] * cz;
            out.w = (double)kSigmaPx * z / (double)c.fx;
        }
        pts[p] = out;
    }
}

// The two window passes work on 16 x 16 pixels per workgroup with the 26 x 26 neighbourhood
// (5-pixel halo) staged in LDS: points as double (their differences are taken in double, then
// rounded), the exponent factor k = log2(e) / (2 s^2) of each pixel's own sigma (kNoPoint where
// nothing was blended, kOutside beyond the image), and the colours or the coefficients.
// The weight of neighbour q in the window of centre c is exp2(-|P(q) - P(c)|^2 k_c); a centre
// without a point keeps only itself, a neighbour without a point has no weight.
constexpr int kT = 16, kHalo = kT + 2 * kWin, kHN = kHalo * kHalo;
constexpr float kNoPoint = -1.0f, kOutside = -2.0f;
constexpr double kLog2eD = 1.4426950408889634;

struct HaloPoints {
    double px[kHN], py[kHN], pz[kHN];
    float k[kHN];
};

__device__ __forceinline__ void stage_points(const double4* __restrict__ pts, int W, int H, int x0, int y0,
                                             HaloPoints& h) {
    for (int i = threadIdx.x; i < kHN; i += 256) {
        const int gx = x0 - kWin + i % kHalo, gy = y0 - kWin + i / kHalo;
        double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
        float k = kOutside;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) {
            p = pts[(size_t)gy * W + gx];
            k = p.w > 0.0 ? (float)(kLog2eD / (2.0 * p.w * p.w)) : kNoPoint;
        }
        h.px[i] = p.x;
        h.py[i] = p.y;
        h.pz[i] = p.z;
        h.k[i] = k;
    }
}

__device__ __forceinline__ float pair_weight(const HaloPoints& h, int c, int q, float kc) {
    const float dx = (float)(h.px[q] - h.px[c]), dy = (float)(h.py[q] - h.py[c]), dz = (float)(h.pz[q] - h.pz[c]);
    return __builtin_amdgcn_exp2f(-(dx * dx + dy * dy + dz * dz) * kc);
}

// Per centre: weighted moments over the window, SSIM per channel, loss partial sums (per
// workgroup, double) and the three gradient coefficients per channel (already divided by the
// window's weight sum).
__global__ void __launch_bounds__(256) k_ssim3d_fwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                    const double4* __restrict__ pts, int W, int H,
                                                    float* __restrict__ coef, double* __restrict__ partial) {
    __shared__ HaloPoints h;
    __shared__ float col[6][kHN];
    __shared__ double red[2][4];
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    const size_t hw = (size_t)W * H;
    stage_points(pts, W, H, x0, y0, h);
    for (int i = threadIdx.x; i < kHN; i += 256) {
        const int gx = x0 - kWin + i % kHalo, gy = y0 - kWin + i / kHalo;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const size_t g = in ? (size_t)gy * W + gx : 0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            col[ch][i] = in ? img[ch * hw + g] : 0.0f;
            col[3 + ch][i] = in ? tgt[ch * hw + g] : 0.0f;
        }
    }
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = x0 + lx, y = y0 + ly;
    double s_ssim = 0.0, s_l1 = 0.0;
    if (x < W && y < H) {
        const int ci = (ly + kWin) * kHalo + lx + kWin;
        const float kc = h.k[ci];
        float sw = 0.0f, m1[3] = {0, 0, 0}, m2[3] = {0, 0, 0}, e11[3] = {0, 0, 0}, e22[3] = {0, 0, 0},
              e12[3] = {0, 0, 0};
        for (int dy = -kWin; dy <= kWin; ++dy) {
            const int row = ci + dy * kHalo;
            for (int dx = -kWin; dx <= kWin; ++dx) {
                const int q = row + dx;
                float w;
                if (kc < 0.0f) {
                    w = q == ci ? 1.0f : 0.0f;
                } else {
                    if (h.k[q] < 0.0f) continue;
                    w = pair_weight(h, ci, q, kc);
                }
                if (w == 0.0f) continue;
                sw += w;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float a = col[ch][q], b = col[3 + ch][q];
                    const float wa = w * a, wb = w * b;
                    m1[ch] += wa;
                    m2[ch] += wb;
                    e11[ch] = __builtin_fmaf(wa, a, e11[ch]);
                    e22[ch] = __builtin_fmaf(wb, b, e22[ch]);
                    e12[ch] = __builtin_fmaf(wa, b, e12[ch]);
                }
            }
        }
        const size_t c = (size_t)y * W + x;
        const float inv = 1.0f / sw;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float mu1 = m1[ch] * inv, mu2 = m2[ch] * inv;
            const float s11 = e11[ch] * inv - mu1 * mu1, s22 = e22[ch] * inv - mu2 * mu2;
            const float s12 = e12[ch] * inv - mu1 * mu2;
            const float A = 2.0f * mu1 * mu2 + kC1, Bn = 2.0f * s12 + kC2;
            const float Cn = mu1 * mu1 + mu2 * mu2 + kC1, Dn = s11 + s22 + kC2;
            const float CD = Cn * Dn;
            const float S = A * Bn / CD;
            const float dmu = 2.0f * mu2 * Bn / CD - S * 2.0f * mu1 / Cn;
            const float ds11 = -S / Dn, ds12 = 2.0f * A / CD;
            coef[(size_t)(3 * ch + 0) * hw + c] = (dmu - 2.0f * mu1 * ds11 - mu2 * ds12) * inv;
            coef[(size_t)(3 * ch + 1) * hw + c] = 2.0f * ds11 * inv;
            coef[(size_t)(3 * ch + 2) * hw + c] = ds12 * inv;
            s_ssim += (double)S;
            s_l1 += (double)fabsf(col[ch][ci] - col[3 + ch][ci]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        s_ssim += __shfl_down(s_ssim, o, 64);
        s_l1 += __shfl_down(s_l1, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s_ssim;
        red[1][threadIdx.x >> 6] = s_l1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partial[2 * b + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Per pixel q: dL/dI(q) = w_l1 sign(I - T) / N - w_dssim / N * sum over centres c whose window holds q
// of w_cq (a_c + b_c I(q) + d_c T(q)).
__global__ void __launch_bounds__(256) k_ssim3d_bwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                    const double4* __restrict__ pts, const float* __restrict__ coef,
                                                    int W, int H, float w_l1, float w_dssim,
                                                    float* __restrict__ grad) {
    __shared__ HaloPoints h;
    __shared__ float cf[9][kHN];
    const int x0 = blockIdx.x * kT, y0 = blockIdx.y * kT;
    const size_t hw = (size_t)W * H;
    stage_points(pts, W, H, x0, y0, h);
    for (int i = threadIdx.x; i < kHN; i += 256) {
        const int gx = x0 - kWin + i % kHalo, gy = y0 - kWin + i / kHalo;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const size_t g = in ? (size_t)gy * W + gx : 0;
#pragma unroll
        for (int j = 0; j < 9; ++j) cf[j][i] = in ? coef[(size_t)j * hw + g] : 0.0f;
    }
    __syncthreads();
    const int lx = threadIdx.x & 15, ly = threadIdx.x >> 4;
    const int x = x0 + lx, y = y0 + ly;
    if (x >= W || y >= H) return;
    const size_t q = (size_t)y * W + x;
    const int qi = (ly + kWin) * kHalo + lx + kWin;
    float a[3], b[3], acc[3] = {0, 0, 0};
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        a[ch] = img[ch * hw + q];
        b[ch] = tgt[ch * hw + q];
    }
    if (h.k[qi] < 0.0f) {
        // no point here: only its own window holds it (with weight 1)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] = cf[3 * ch][qi] + cf[3 * ch + 1][qi] * a[ch] + cf[3 * ch + 2][qi] * b[ch];
    } else {
        for (int dy = -kWin; dy <= kWin; ++dy) {
            const int row = qi + dy * kHalo;
            for (int dx = -kWin; dx <= kWin; ++dx) {
                const int c = row + dx;
                const float kc = h.k[c];
                if (kc < 0.0f) continue;
                const float w = pair_weight(h, c, qi, kc);
                if (w == 0.0f) continue;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    const float t = cf[3 * ch][c] + cf[3 * ch + 1][c] * a[ch] + cf[3 * ch + 2][c] * b[ch];
                    acc[ch] = __builtin_fmaf(w, t, acc[ch]);
                }
            }
        }
    }
    const float invN = 1.0f / (3.0f * (float)hw);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float d = a[ch] - b[ch];
        const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        grad[ch * hw + q] = w_l1 * sg * invN - w_dssim * acc[ch] * invN;
    }
}

// L1 alone (w_dssim = 0): the gradient w_l1 sign(I - T) / N and per-workgroup L1 sums, with the
// same grid and partial layout as the window passes.
__global__ void __launch_bounds__(256) k_l1_plane(const float* __restrict__ img, const float* __restrict__ tgt,
                                                  int W, int H, float w_l1, float* __restrict__ grad,
                                                  double* __restrict__ partial) {
    __shared__ double red[4];
    const int x = blockIdx.x * kT + (threadIdx.x & 15), y = blockIdx.y * kT + (threadIdx.x >> 4);
    const size_t hw = (size_t)W * H;
    double s_l1 = 0.0;
    if (x < W && y < H) {
        const size_t q = (size_t)y * W + x;
        const float invN = 1.0f / (3.0f * (float)hw);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = img[ch * hw + q] - tgt[ch * hw + q];
            const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
            grad[ch * hw + q] = w_l1 * sg * invN;
            s_l1 += (double)fabsf(d);
        }
    }
    for (int o = 32; o > 0; o >>= 1) s_l1 += __shfl_down(s_l1, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s_l1;
    __syncthreads();
    if (threadIdx.x == 0) {
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        partial[2 * b] = 0.0;
        partial[2 * b + 1] = red[0] + red[1] + red[2] + red[3];
    }
}

__global__ void k_loss3d_final(const double* __restrict__ partial, int n, double N, float w_l1, float w_dssim,
                               float* __restrict__ out) {
    __shared__ double red[2][256];
    double s = 0.0, l = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s += partial[2 * i];
        l += partial[2 * i + 1];
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[0] = (float)((double)w_l1 * red[1][0] / N + (double)w_dssim * (1.0 - red[0][0] / N));
}

size_t loss3d_scratch_bytes(int W, int H) {
    const size_t hw = (size_t)W * H;
    const size_t blocks = (size_t)((W + 15) / 16) * ((H + 15) / 16);
    return hw * sizeof(double4) + 9 * hw * sizeof(float) + 2 * blocks * sizeof(double) + 256;
}

void launch_loss3d(const DevCam* cams, int B, uint32_t n_tiles, const uint32_t* sel_off, const uint32_t* sel_pix,
                   const float* t_sel, const float* depth_sel, int W, int H, const float* img, const float* tgt,
                   float w_l1, float w_dssim, float* loss_out, float* grad, void* scratch, hipStream_t s,
                   const uint32_t* void_word) {
    const size_t hw = (size_t)W * H;
    uint8_t* p = (uint8_t*)scratch;
    double4* pts = (double4*)p;
    p += hw * sizeof(double4);
    float* coef = (float*)p;
    p += 9 * hw * sizeof(float);
    p = (uint8_t*)(((uintptr_t)p + 7) & ~(uintptr_t)7);
    double* partial = (double*)p;
    const dim3 grid((W + 15) / 16, (H + 15) / 16);
    const int blocks = (int)(grid.x * grid.y);
    if (w_dssim == 0.0f) {
        hipLaunchKernelGGL(k_l1_plane, grid, dim3(256), 0, s, img, tgt, W, H, w_l1, grad, partial);
    } else {
        hipLaunchKernelGGL(k_points3d, dim3((n_tiles + 3) / 4), dim3(256), 0, s, cams, B, n_tiles, sel_off,
                           sel_pix, t_sel, depth_sel, pts, void_word);
        hipLaunchKernelGGL(k_ssim3d_fwd, grid, dim3(256), 0, s, img, tgt, pts, W, H, coef, partial);
        hipLaunchKernelGGL(k_ssim3d_bwd, grid, dim3(256), 0, s, img, tgt, pts, coef, W, H, w_l1, w_dssim, grad);
    }
    hipLaunchKernelGGL(k_loss3d_final, dim3(1), dim3(256), 0, s, partial, blocks, 3.0 * (double)hw, w_l1, w_dssim,
                       loss_out);
}

}  // namespace mvgs
