// Kernels of the synthetic training loop around the rasterizer: one Adam update of the activated
// parameters, the row gather that carries per-Gaussian optimiser state through densification, and
// the running moments of mini-batch gradients used to estimate their variance (Sec. 3.2).
//
// The parameters are kept activated (the rasterizer's inputs). Scales and opacities are optimised
// in their unconstrained coordinates, log-scale and opacity logit, as 3DGS does; those coordinates
// are implied by the activated values: the gradient is taken through the activation and the step
// is applied as s * exp(-step) and sigmoid(logit(o) - step) = 1 / (1 + (1 - o) / o * exp(step)).
#include "mvgs_kernels.h"

namespace mvgs {

// One element per thread over [P][D] with D = 11 + 3K: means 3, scales 3, quats 4, opacity 1, SH 3K.
// Idx is uint32_t when P D fits (a 32-bit division by D instead of a 64-bit one).
template <typename Idx>
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ means, float* __restrict__ scales,
                                              float* __restrict__ quats, float* __restrict__ opac,
                                              float* __restrict__ sh, const float* __restrict__ g_means,
                                              const float* __restrict__ g_scales, const float* __restrict__ g_quats,
                                              const float* __restrict__ g_opac, const float* __restrict__ g_sh,
                                              float2* __restrict__ mom, int64_t P, int K, AdamArgs a,
                                              const float* __restrict__ state) {
    if (state) {   // counted on the device
        if (state[0] != 0.0f) return;
        a.bc1 = state[1];
        a.bc2 = state[2];
    }
    const Idx D = (Idx)(11 + 3 * K);
    const Idx i = (Idx)blockIdx.x * 256u + (Idx)threadIdx.x;
    if ((int64_t)i >= P * (int64_t)D) return;
    const int64_t g = (int64_t)(i / D);
    const int d = (int)(i - (Idx)g * D);
    float* p;
    float grad, lr;
    float x = 0.0f;   // scale or opacity before the step
    if (d < 3) {
        p = means + 3 * g + d;
        grad = g_means[3 * g + d];
        lr = a.lr_means;
    } else if (d < 6) {
        p = scales + 3 * g + (d - 3);
        x = *p;
        grad = g_scales[3 * g + (d - 3)] * x;   // d/d log s
        lr = a.lr_scales;
    } else if (d < 10) {
        p = quats + 4 * g + (d - 6);
        grad = g_quats[4 * g + (d - 6)];
        lr = a.lr_quats;
    } else if (d == 10) {
        p = opac + g;
        x = *p;
        grad = g_opac[g] * (x * (1.0f - x));     // d/d logit o
        lr = a.lr_opacities;
    } else {
        const int e = d - 11;
        p = sh + (int64_t)3 * K * g + e;
        grad = g_sh[(int64_t)3 * K * g + e];
        lr = e < 3 ? a.lr_sh_dc : a.lr_sh_rest;
    }
    float2 mv = mom[i];
    mv.x = a.beta1 * mv.x + (1.0f - a.beta1) * grad;
    mv.y = a.beta2 * mv.y + (1.0f - a.beta2) * (grad * grad);
    mom[i] = mv;
    const float step = lr * (mv.x / a.bc1) / (sqrtf(mv.y / a.bc2) + a.eps);
    if (d >= 3 && d < 6) {
        *p = x * expf(-step);
    } else if (d == 10) {
        // 0 and 1 are fixed points of the logit step (and would give 0 * inf here)
        if (x > 0.0f && x < 1.0f) *p = 1.0f / (1.0f + (1.0f - x) / x * expf(step));
    } else {
        *p = *p - step;
    }
}

template <typename Idx>
__global__ void __launch_bounds__(256) k_gather_rows(const int32_t* __restrict__ src, int64_t n, int64_t width,
                                                     const float* __restrict__ in, float* __restrict__ out) {
    const Idx i = (Idx)blockIdx.x * 256u + (Idx)threadIdx.x;
    if ((int64_t)i >= n * width) return;
    const Idx r = i / (Idx)width;
    out[i] = in[(int64_t)src[r] * width + (int64_t)(i - r * (Idx)width)];
}

// sum += x over the concatenation of the five gradient tensors; per workgroup, the partial sums
// of ||x||^2 and of ||sum after the update||^2 (fixed grid and order: the result is reproducible).
__global__ void __launch_bounds__(256) k_grad_moments(GradSegments g, double* __restrict__ sum,
                                                      double* __restrict__ partials) {
    __shared__ double red[2][4];
    double a0 = 0.0, a1 = 0.0;
    const int64_t n = g.end[4];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int k = 0;
        while (i >= g.end[k]) ++k;
        const double v = (double)g.x[k][i - (k ? g.end[k - 1] : 0)];
        const double s = sum[i] + v;
        sum[i] = s;
        a0 += v * v;
        a1 += s * s;
    }
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_down(a0, o, 64);
        a1 += __shfl_down(a1, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a0;
        red[1][w] = a1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partials[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// acc[0] += sum of the squared-norm partials; acc[1] = sum of the partials of ||sum||^2.
__global__ void __launch_bounds__(256) k_grad_moments_final(const double* __restrict__ partials, int blocks,
                                                            double* __restrict__ acc) {
    __shared__ double red[2][256];
    double a0 = 0.0, a1 = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) {
        a0 += partials[2 * b];
        a1 += partials[2 * b + 1];
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        acc[0] += red[0][0];
        acc[1] = red[1][0];
    }
}

// The step counter of a replayed (graph-captured) Adam step: t = ++*step unless *skip, and the
// bias corrections 1 - beta^t rounded from double, as the host computes them for a given step.
__global__ void k_adam_count(int32_t* __restrict__ step, const uint32_t* __restrict__ skip, float beta1, float beta2,
                             float* __restrict__ state) {
    const bool sk = skip && *skip;
    state[0] = sk ? 1.0f : 0.0f;
    if (sk) return;
    const int32_t t = *step + 1;
    *step = t;
    state[1] = (float)(1.0 - pow((double)beta1, (double)t));
    state[2] = (float)(1.0 - pow((double)beta2, (double)t));
}

void launch_adam_count(int32_t* step, const uint32_t* skip, float beta1, float beta2, float* state, hipStream_t s) {
    hipLaunchKernelGGL(k_adam_count, dim3(1), dim3(1), 0, s, step, skip, beta1, beta2, state);
}

void launch_adam(float* means, float* scales, float* quats, float* opac, float* sh, const GradArgs& gr, float* mom,
                 int64_t P, int sh_degree, const AdamArgs& a, hipStream_t s, const float* state) {
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const int64_t n = P * (11 + 3 * K);
    if (!n) return;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (n <= (int64_t(1) << 32) - 256)   // no index of the grid wraps
        hipLaunchKernelGGL(k_adam<uint32_t>, grid, dim3(256), 0, s, means, scales, quats, opac, sh, gr.means,
                           gr.scales, gr.quats, gr.opac, gr.sh, reinterpret_cast<float2*>(mom), P, K, a, state);
    else
        hipLaunchKernelGGL(k_adam<uint64_t>, grid, dim3(256), 0, s, means, scales, quats, opac, sh, gr.means,
                           gr.scales, gr.quats, gr.opac, gr.sh, reinterpret_cast<float2*>(mom), P, K, a, state);
}

void launch_gather_rows(const int32_t* src, int64_t n, int64_t width, const float* in, float* out, hipStream_t s) {
    if (!n || !width) return;
    const dim3 grid((unsigned)((n * width + 255) / 256));
    if (n * width <= (int64_t(1) << 32) - 256)
        hipLaunchKernelGGL(k_gather_rows<uint32_t>, grid, dim3(256), 0, s, src, n, width, in, out);
    else
        hipLaunchKernelGGL(k_gather_rows<uint64_t>, grid, dim3(256), 0, s, src, n, width, in, out);
}

size_t moment_blocks(int64_t n) {
    return (size_t)std::max<int64_t>(1, std::min<int64_t>((n + 2047) / 2048, kMomentBlocks));
}

void launch_grad_moments(const GradSegments& g, double* sum, double* acc, double* partials, hipStream_t s) {
    const int64_t n = g.end[4];
    const int blocks = (int)moment_blocks(n);
    if (n) hipLaunchKernelGGL(k_grad_moments, dim3((unsigned)blocks), dim3(256), 0, s, g, sum, partials);
    hipLaunchKernelGGL(k_grad_moments_final, dim3(1), dim3(256), 0, s, partials, n ? blocks : 0, acc);
}

}  // namespace mvgs
