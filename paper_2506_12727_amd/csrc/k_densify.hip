// Multi-view adaptive density control (paper Sec. 5.2.2): from the per-view statistics of the
// backward (Eqs. 13-14) decide per Gaussian whether to split it (mean E1 above a threshold and a
// large scale), clone it (mean E2 above a threshold and a small scale), keep it or prune it (low
// opacity), then write the new set with every original's outputs in a row, in original order.
// Split children are drawn from the parent (mean + R (s * z) with caller-supplied normals z) with
// scales divided by 1.6. The decisions are single-precision comparisons.
#include "mvgs_kernels.h"

namespace mvgs {

constexpr uint8_t kPrune = 0, kKeep = 1, kClone = 2, kSplit = 3;

__global__ void __launch_bounds__(256) k_adc_classify(const float* __restrict__ scales,
                                                      const float* __restrict__ opac, const float* __restrict__ e1,
                                                      const float* __restrict__ e2,
                                                      const int32_t* __restrict__ count, int64_t P, AdcParams prm,
                                                      uint32_t* __restrict__ n_out, uint8_t* __restrict__ action) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= P) return;
    uint8_t a = kKeep;
    if (opac[g] < prm.min_opacity) {
        a = kPrune;
    } else {
        const float smax = fmaxf(fmaxf(scales[3 * g], scales[3 * g + 1]), scales[3 * g + 2]);
        const bool big = smax > prm.dense_scale;
        const int32_t c = count[g];
        const float m1 = c > 0 ? e1[g] / (float)c : 0.0f;
        const float m2 = c > 0 ? e2[g] / (float)c : 0.0f;
        if (big && m1 > prm.split_threshold) a = kSplit;
        else if (!big && m2 > prm.clone_threshold) a = kClone;
    }
    action[g] = a;
    n_out[g] = a == kPrune ? 0u : (a == kKeep ? 1u : 2u);
}

__global__ void __launch_bounds__(256) k_adc_write(const float* __restrict__ means, const float* __restrict__ scales,
                                                   const float* __restrict__ quats, const float* __restrict__ opac,
                                                   const float* __restrict__ sh, int64_t P, int K,
                                                   const float* __restrict__ normals,
                                                   const uint8_t* __restrict__ action, const uint32_t* __restrict__ off,
                                                   float* __restrict__ o_means, float* __restrict__ o_scales,
                                                   float* __restrict__ o_quats, float* __restrict__ o_opac,
                                                   float* __restrict__ o_sh, int32_t* __restrict__ src) {
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= P) return;
    const uint8_t a = action[g];
    if (a == kPrune) return;
    const int n = a == kKeep ? 1 : 2;
    float R[9];
    if (a == kSplit) {
        float w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
        const float inv = 1.0f / sqrtf(w * w + x * x + y * y + z * z);
        w *= inv; x *= inv; y *= inv; z *= inv;
        R[0] = 1.0f - 2.0f * (y * y + z * z); R[1] = 2.0f * (x * y - w * z); R[2] = 2.0f * (x * z + w * y);
        R[3] = 2.0f * (x * y + w * z); R[4] = 1.0f - 2.0f * (x * x + z * z); R[5] = 2.0f * (y * z - w * x);
        R[6] = 2.0f * (x * z - w * y); R[7] = 2.0f * (y * z + w * x); R[8] = 1.0f - 2.0f * (x * x + y * y);
    }
    for (int k = 0; k < n; ++k) {
        const int64_t o = (int64_t)off[g] + k;
        float s[3] = {scales[3 * g], scales[3 * g + 1], scales[3 * g + 2]};
        float m[3] = {means[3 * g], means[3 * g + 1], means[3 * g + 2]};
        if (a == kSplit) {
            const float* zk = normals + (6 * g + 3 * k);
            const float v0 = s[0] * zk[0], v1 = s[1] * zk[1], v2 = s[2] * zk[2];
#pragma unroll
            for (int i = 0; i < 3; ++i) m[i] += R[3 * i] * v0 + R[3 * i + 1] * v1 + R[3 * i + 2] * v2;
#pragma unroll
            for (int i = 0; i < 3; ++i) s[i] = s[i] / 1.6f;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            o_means[3 * o + i] = m[i];
            o_scales[3 * o + i] = s[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) o_quats[4 * o + i] = quats[4 * g + i];
        o_opac[o] = opac[g];
        for (int i = 0; i < 3 * K; ++i) o_sh[(int64_t)3 * K * o + i] = sh[(int64_t)3 * K * g + i];
        if (src) src[o] = (int32_t)g;
    }
}

void launch_adc_classify(const GaussianArgs& ga, const float* e1, const float* e2, const int32_t* count,
                         const AdcParams& prm, uint32_t* n_out, uint8_t* action, hipStream_t s) {
    if (!ga.P) return;
    hipLaunchKernelGGL(k_adc_classify, dim3((unsigned)((ga.P + 255) / 256)), dim3(256), 0, s, ga.scales, ga.opac, e1,
                       e2, count, ga.P, prm, n_out, action);
}

void launch_adc_write(const GaussianArgs& ga, const float* normals, const uint8_t* action, const uint32_t* off,
                      float* means, float* scales, float* quats, float* opac, float* sh, int32_t* src, hipStream_t s) {
    if (!ga.P) return;
    const int K = (ga.sh_degree + 1) * (ga.sh_degree + 1);
    hipLaunchKernelGGL(k_adc_write, dim3((unsigned)((ga.P + 255) / 256)), dim3(256), 0, s, ga.means, ga.scales,
                       ga.quats, ga.opac, ga.sh, ga.P, K, normals, action, off, means, scales, quats, opac, sh, src);
}

}  // namespace mvgs
