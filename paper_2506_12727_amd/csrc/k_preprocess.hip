// Per-Gaussian preprocessing kernels: participation count, record emission, and the
// backward chain from 2D quantities to the parameters (paper Sec. 3; multi-view
// appendix: participation is decided per view before memory is sized).
//
// One thread per Gaussian loops over all views of the batch, so each Gaussian's
// parameters are read from HBM once per step whatever the number of views; the
// cameras are uniform across the wave and come in through the scalar cache.
#include <algorithm>

#include "mvgs_kernels.h"

namespace mvgs {

__device__ __forceinline__ void load_gaussian(const float* __restrict__ means, const float* __restrict__ scales,
                                              const float* __restrict__ quats, const float* __restrict__ opac,
                                              int64_t g, float mu[3], float s[3], float q[4], float& o) {
    mu[0] = means[3 * g]; mu[1] = means[3 * g + 1]; mu[2] = means[3 * g + 2];
    s[0] = scales[3 * g]; s[1] = scales[3 * g + 1]; s[2] = scales[3 * g + 2];
    const float4 qq = *reinterpret_cast<const float4*>(quats + 4 * g);
    q[0] = qq.x; q[1] = qq.y; q[2] = qq.z; q[3] = qq.w;
    o = opac[g];
}

// Tiles covered by the inclusive pixel range [a, b] (0 <= a <= b) of tiles `tile` pixels wide, a
// power of two (8, 16 or 32): a shift, where an integer division would take a long VALU sequence.
__device__ __forceinline__ int tile_span(int a, int b, int tile) {
    const int sh = __builtin_ctz((unsigned)tile);
    return (b >> sh) - (a >> sh) + 1;
}

// Number of participating views and of covered tiles (summed over views) per Gaussian.
__global__ void __launch_bounds__(256) k_count(const float* __restrict__ means, const float* __restrict__ scales,
                                               const float* __restrict__ quats, const float* __restrict__ opac,
                                               int64_t P, const DevCam* __restrict__ cams, int B, int tile_w,
                                               int tile_h, uint32_t* __restrict__ nrec,
                                               uint32_t* __restrict__ ntiles, uint32_t* __restrict__ key_range) {
    __shared__ uint32_t red[2][4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t kmin = 0xffffffffu, kmax = 0u;   // depth keys of the participating records
    if (g < P) {
        float mu[3], s[3], q[4], o;
        load_gaussian(means, scales, quats, opac, g, mu, s, q, o);
        GaussGeom geo;
        gauss_geom(s, q, o, geo);
        uint32_t n = 0, nt = 0;
        for (int v = 0; v < B; ++v) {
            ProjState st;
            const ProjOut p = project(mu, geo, cams[v], st);
            if (p.ok) {
                n += 1;
                nt += (uint32_t)(tile_span(p.x0, p.x1, tile_w) * tile_span(p.y0, p.y1, tile_h));
                kmin = min(kmin, f2u(p.depth));
                kmax = max(kmax, f2u(p.depth));
            }
        }
        nrec[g] = n;
        ntiles[g] = nt;
    }
    if (!key_range) return;   // (uniform over the workgroup)
    // the workgroup's range; a global atomic only when it widens the range seen so far
    for (int off = 32; off > 0; off >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = kmin;
        red[1][w] = kmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (int)(blockDim.x + 63) >> 6;
        for (int i = 1; i < nw; ++i) {
            kmin = min(kmin, red[0][i]);
            kmax = max(kmax, red[1][i]);
        }
        // the second word holds the complement of the maximum, so that both start at ~0
        if (kmin < __atomic_load_n(key_range, __ATOMIC_RELAXED)) atomicMin(key_range, kmin);
        if (~kmax < __atomic_load_n(key_range + 1, __ATOMIC_RELAXED)) atomicMin(key_range + 1, ~kmax);
    }
}

// Participation pre-pass per view, for admission before anything is sized: the records (1 per
// participating Gaussian) and covered tiles of each view, summed over the Gaussians. One thread per
// Gaussian walks the views; per view a wavefront sum, the workgroup's four wavefront sums added in
// LDS, and one partial per workgroup, view and count (partial[(2 v + c) * blocks + block]); a
// second kernel adds each row of partials. (One 64-bit atomic per wavefront into the same two
// words per view serialised on one L2 channel: 0.4 ms for 1M Gaussians.)
__global__ void __launch_bounds__(256) k_count_views(const float* __restrict__ means,
                                                     const float* __restrict__ scales,
                                                     const float* __restrict__ quats,
                                                     const float* __restrict__ opac, int64_t P,
                                                     const DevCam* __restrict__ cams, int B, int tile_w, int tile_h,
                                                     unsigned long long* __restrict__ partial) {
    __shared__ uint32_t red[2][4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < P;
    const int wave = threadIdx.x >> 6;
    float mu[3] = {0.f, 0.f, 0.f}, s[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f}, o = 0.f;
    if (live) load_gaussian(means, scales, quats, opac, g, mu, s, q, o);
    GaussGeom geo;
    gauss_geom(s, q, o, geo);
    for (int v = 0; v < B; ++v) {
        uint32_t n = 0, nt = 0;
        if (live) {
            ProjState st;
            const ProjOut p = project(mu, geo, cams[v], st);
            if (p.ok) {
                n = 1;
                nt = (uint32_t)(tile_span(p.x0, p.x1, tile_w) * tile_span(p.y0, p.y1, tile_h));
            }
        }
        // at most 256 x 65,536 tiles per workgroup: the sums fit 32 bits
        for (int off = 32; off > 0; off >>= 1) {
            n += (uint32_t)__shfl_xor((int)n, off, 64);
            nt += (uint32_t)__shfl_xor((int)nt, off, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            red[0][wave] = n;
            red[1][wave] = nt;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            const uint32_t* r = red[threadIdx.x];
            partial[(size_t)(2 * v + threadIdx.x) * gridDim.x + blockIdx.x] =
                (unsigned long long)r[0] + r[1] + r[2] + r[3];
        }
        __syncthreads();
    }
}

// counts[k] = sum of row k of the partials (rows of `blocks` values), one workgroup per row
__global__ void __launch_bounds__(256) k_sum_rows_u64(const unsigned long long* __restrict__ partial,
                                                      uint32_t blocks, unsigned long long* __restrict__ counts) {
    __shared__ unsigned long long red[4];
    const unsigned long long* row = partial + (size_t)blockIdx.x * blocks;
    unsigned long long s = 0;
    for (uint32_t i = threadIdx.x; i < blocks; i += 256) s += row[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// The per-record arrays beside the record itself: view, depth key and covered-tile rectangle
// (first global tile id, width | height << 16; the view's tiles per row follow from the id).
__device__ __forceinline__ void record_side(const BlendRec& r, const DevCam* __restrict__ cams, int tile_w,
                                            int tile_h, uint32_t i, uint32_t* __restrict__ depth_key,
                                            uint2* __restrict__ tile_rect, uint16_t* __restrict__ rec_view) {
    const DevCam& c = cams[r.view];
    const uint32_t x0 = r.boxx & 0xffffu, x1 = r.boxx >> 16, y0 = r.boxy & 0xffffu, y1 = r.boxy >> 16;
    const uint32_t sw = (uint32_t)__builtin_ctz((unsigned)tile_w), shh = (uint32_t)__builtin_ctz((unsigned)tile_h);
    const uint32_t tx0 = x0 >> sw, ty0 = y0 >> shh;   // tiles are 8, 16 or 32 pixels
    const uint32_t tw_n = (x1 >> sw) - tx0 + 1, th_n = (y1 >> shh) - ty0 + 1;
    rec_view[i] = (uint16_t)r.view;
    depth_key[i] = r.depth_bits;
    tile_rect[i] = make_uint2(c.tile_base + ty0 * (uint32_t)c.tiles_x + tx0, tw_n | (th_n << 16));
}

// Records of every participating (view, Gaussian), written in (Gaussian, view) order at
// rec_off[g]. Also the depth sort key and the covered-tile rectangle of each record. One
// wavefront per workgroup: its 64 Gaussians own one contiguous run of records, which is staged in
// LDS while the lanes project view after view and then written out by consecutive lanes (each
// lane's own records lie a Gaussian's worth of views apart, so direct stores would leave lines
// half written). A run a little longer than the stage goes through it in two windows: the second
// repeats, for the lanes whose records straddle the two, the participation tests of the views
// before it, and evaluates colours and assembles only its own records. A run longer still (many
// views per Gaussian) is written directly: with two windows of about half the lanes each, the
// wavefront's serial time would double.
constexpr uint32_t kRecStage = 512;   // records (32 KiB)

// The record of a participating (view, Gaussian): its projection p, colour from the SH
// coefficients along the view direction (clamped at 0), opacity o.
template <int D>
__device__ __forceinline__ BlendRec make_record(const ProjOut& p, const float (&mu)[3], float o,
                                                const float (&coef)[(D + 1) * (D + 1)][3], const DevCam& c,
                                                uint32_t g, uint32_t v) {
    constexpr int K = (D + 1) * (D + 1);
    float dx = mu[0] - c.campos[0], dy = mu[1] - c.campos[1], dz = mu[2] - c.campos[2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    dx *= il; dy *= il; dz *= il;
    float Y[16];
    sh_basis<D>(dx, dy, dz, Y);
    float rgb[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float a = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) a = __builtin_fmaf(coef[k][ch], Y[k], a);
        rgb[ch] = a > 0.0f ? a : 0.0f;
    }
    BlendRec r;
    r.boxx = (uint32_t)p.x0 | ((uint32_t)p.x1 << 16);
    r.boxy = (uint32_t)p.y0 | ((uint32_t)p.y1 << 16);
    r.mx = p.mx; r.my = p.my;
    r.hca = p.hca * kLog2e; r.nb = p.nb * kLog2e; r.hcc = p.hcc * kLog2e; r.o = o;
    r.cut = p.cut * kLog2e; r.unused = 0.0f; r.r = rgb[0]; r.g = rgb[1];
    r.b = rgb[2];
    r.gid = g;
    r.view = v;
    r.depth_bits = f2u(p.depth);
    return r;
}

template <int D>
__global__ void __launch_bounds__(64) k_records(const float* __restrict__ means, const float* __restrict__ scales,
                                                const float* __restrict__ quats, const float* __restrict__ opac,
                                                const float* __restrict__ sh, int64_t P,
                                                const DevCam* __restrict__ cams, int B, int tile_w, int tile_h,
                                                const uint32_t* __restrict__ rec_off, BlendRec* __restrict__ recs,
                                                uint32_t* __restrict__ depth_key, uint2* __restrict__ tile_rect,
                                                uint16_t* __restrict__ rec_view,
                                                const uint32_t* __restrict__ overflow) {
    __shared__ BlendRec stage[kRecStage];
    constexpr int K = (D + 1) * (D + 1);
    if (overflow && *overflow) return;
    const int64_t g0 = (int64_t)blockIdx.x * 64;
    const int64_t g1 = g0 + 64 < P ? g0 + 64 : P;
    const uint32_t base = rec_off[g0], n_run = rec_off[g1] - base;
    const int64_t g = g0 + threadIdx.x;
    const bool here = g < P;
    float mu[3] = {0.0f, 0.0f, 0.0f}, s[3] = {0.0f, 0.0f, 0.0f}, q[4] = {1.0f, 0.0f, 0.0f, 0.0f}, o = 0.0f;
    float coef[K][3];
    uint32_t out0 = 0, out_end = 0;
    if (here) {
        load_gaussian(means, scales, quats, opac, g, mu, s, q, o);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) coef[k][ch] = sh[(g * K + k) * 3 + ch];
        out0 = rec_off[g];
        out_end = rec_off[g + 1];
    }
    GaussGeom geo;
    gauss_geom(s, q, o, geo);
    const bool staged = n_run <= kRecStage + kRecStage / 4;   // uniform over the workgroup
    if (!staged) {
        if (!here) return;
        uint32_t out = out0;
        for (int v = 0; v < B && out < out_end; ++v) {
            const DevCam& c = cams[v];
            ProjState st;
            const ProjOut p = project(mu, geo, c, st);
            if (!p.ok) continue;
            const BlendRec r = make_record<D>(p, mu, o, coef, c, (uint32_t)g, (uint32_t)v);
            recs[out] = r;
            record_side(r, cams, tile_w, tile_h, out, depth_key, tile_rect, rec_view);
            ++out;
        }
        return;
    }
    for (uint32_t w0 = 0; w0 < n_run; w0 += kRecStage) {
        const uint32_t lo = base + w0, hi = base + min(n_run, w0 + kRecStage);
        if (here && out0 < hi && out_end > lo) {
            uint32_t out = out0;
            for (int v = 0; v < B && out < out_end && out < hi; ++v) {
                const DevCam& c = cams[v];
                ProjState st;
                const ProjOut p = project(mu, geo, c, st);
                if (!p.ok) continue;
                if (out >= lo) stage[out - lo] = make_record<D>(p, mu, o, coef, c, (uint32_t)g, (uint32_t)v);
                ++out;
            }
        }
        __syncthreads();
        const uint32_t n = hi - lo;
        const uint4* src = reinterpret_cast<const uint4*>(stage);
        uint4* dst = reinterpret_cast<uint4*>(recs + lo);
        for (uint32_t i = threadIdx.x; i < 4 * n; i += 64) dst[i] = src[i];
        for (uint32_t i = threadIdx.x; i < n; i += 64)
            record_side(stage[i], cams, tile_w, tile_h, lo + i, depth_key, tile_rect, rec_view);
        __syncthreads();   // the stage is reused by the next window
    }
}

// Backward chain per Gaussian over its records (2D gradients -> parameters), summed over
// views; densification statistics in each view's normalised device coordinates.
template <int D>
__global__ void __launch_bounds__(256) k_preprocess_bwd(
    const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, int64_t P, const DevCam* __restrict__ cams,
    const uint32_t* __restrict__ rec_off, const uint16_t* __restrict__ rec_view, const float* __restrict__ acc,
    float* __restrict__ g_means, float* __restrict__ g_scales, float* __restrict__ g_quats,
    float* __restrict__ g_opac, float* __restrict__ g_sh, float* __restrict__ e1, float* __restrict__ e2,
    int32_t* __restrict__ count, const uint32_t* __restrict__ overflow) {
    constexpr int K = (D + 1) * (D + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P) return;
    float mu[3], s[3], q[4], o;
    load_gaussian(means, scales, quats, opac, g, mu, s, q, o);
    float coef[K][3], dcoef[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            coef[k][ch] = sh[(g * K + k) * 3 + ch];
            dcoef[k][ch] = 0.0f;
        }
    float dmu[3] = {0, 0, 0}, ds[3] = {0, 0, 0}, dq[4] = {0, 0, 0, 0}, dop = 0.0f;
    float se1 = 0.0f, se2 = 0.0f;
    const uint32_t r0 = rec_off[g], r1 = (overflow && *overflow) ? r0 : rec_off[g + 1];
    GaussGeom geo;
    gauss_geom(s, q, o, geo);
    for (uint32_t ri = r0; ri < r1; ++ri) {
        const uint32_t v = rec_view[ri];
        const DevCam& c = cams[v];
        const float4 a0 = *reinterpret_cast<const float4*>(acc + (size_t)ri * kAccStride);
        const float4 a1 = *reinterpret_cast<const float4*>(acc + (size_t)ri * kAccStride + 4);
        const float4 a2 = *reinterpret_cast<const float4*>(acc + (size_t)ri * kAccStride + 8);
        const float gmx = a0.x, gmy = a0.y, gca = a0.z, gcb = a0.w;
        const float gcc = a1.x, gop = a1.y, gr = a1.z, gg = a1.w;
        const float gb = a2.x, ge1 = a2.y;
        ProjState st;
        (void)project(mu, geo, c, st);
        dop += gop;
        // statistics (NDC = pixel gradient times (W/2, H/2))
        const float nx = gmx * 0.5f * (float)c.W, ny = gmy * 0.5f * (float)c.H;
        se2 += sqrtf(nx * nx + ny * ny);
        se1 += ge1;

        // conic -> Sigma': dL/dSigma' = -Q G Q with G = [[gca, gcb/2], [gcb/2, gcc]]
        const float Q00 = st.ca, Q01 = st.cb, Q11 = st.cc;
        const float G00 = gca, G01 = 0.5f * gcb, G11 = gcc;
        const float QG00 = Q00 * G00 + Q01 * G01, QG01 = Q00 * G01 + Q01 * G11;
        const float QG10 = Q01 * G00 + Q11 * G01, QG11 = Q01 * G01 + Q11 * G11;
        const float Gs00 = -(QG00 * Q00 + QG01 * Q01);
        const float Gs01 = -(QG00 * Q01 + QG01 * Q11);
        const float Gs11 = -(QG10 * Q01 + QG11 * Q11);
        // Sigma' = T Sigma T^T + 0.3 I: dT = 2 Gs T Sigma, dSigma = T^T Gs T
        const float Sm[9] = {st.S[0], st.S[1], st.S[2], st.S[1], st.S[3], st.S[4], st.S[2], st.S[4], st.S[5]};
        float TS0[3], TS1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            TS0[k] = st.T0[0] * Sm[k] + st.T0[1] * Sm[3 + k] + st.T0[2] * Sm[6 + k];
            TS1[k] = st.T1[0] * Sm[k] + st.T1[1] * Sm[3 + k] + st.T1[2] * Sm[6 + k];
        }
        float dT0[3], dT1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dT0[k] = 2.0f * (Gs00 * TS0[k] + Gs01 * TS1[k]);
            dT1[k] = 2.0f * (Gs01 * TS0[k] + Gs11 * TS1[k]);
        }
        float dSig[9];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                dSig[3 * k + m] = st.T0[k] * (Gs00 * st.T0[m] + Gs01 * st.T1[m]) +
                                  st.T1[k] * (Gs01 * st.T0[m] + Gs11 * st.T1[m]);
        // T = J W with J = [[j00, 0, j02], [0, j11, j12]]
        float dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dJ00 += dT0[k] * c.R[k];
            dJ02 += dT0[k] * c.R[6 + k];
            dJ11 += dT1[k] * c.R[3 + k];
            dJ12 += dT1[k] * c.R[6 + k];
        }
        const float iz = st.iz, iz2 = iz * iz, iz3 = iz2 * iz;
        const float x = st.tx, y = st.ty;
        float dtc[3];
        dtc[0] = gmx * c.fx * iz - dJ02 * c.fx * iz2;
        dtc[1] = gmy * c.fy * iz - dJ12 * c.fy * iz2;
        dtc[2] = -gmx * c.fx * x * iz2 - gmy * c.fy * y * iz2 - dJ00 * c.fx * iz2 + dJ02 * 2.0f * c.fx * x * iz3 -
                 dJ11 * c.fy * iz2 + dJ12 * 2.0f * c.fy * y * iz3;
#pragma unroll
        for (int k = 0; k < 3; ++k) dmu[k] += c.R[k] * dtc[0] + c.R[3 + k] * dtc[1] + c.R[6 + k] * dtc[2];
        // Sigma = M M^T, M = rot diag(s): dM = 2 dSigma_sym M
        float M[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) M[3 * i + j] = st.rot[3 * i + j] * s[j];
        float drot[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                float v_ = 0.0f;
#pragma unroll
                for (int k = 0; k < 3; ++k) v_ += (dSig[3 * i + k] + dSig[3 * k + i]) * M[3 * k + j];
                ds[j] += v_ * st.rot[3 * i + j];
                drot[3 * i + j] = v_ * s[j];
            }
        const float w = st.qw, qx = st.qx, qy = st.qy, qz = st.qz;
        float dqn[4];
        dqn[0] = -2 * qz * drot[1] + 2 * qy * drot[2] + 2 * qz * drot[3] - 2 * qx * drot[5] - 2 * qy * drot[6] +
                 2 * qx * drot[7];
        dqn[1] = 2 * qy * drot[1] + 2 * qz * drot[2] + 2 * qy * drot[3] - 4 * qx * drot[4] - 2 * w * drot[5] +
                 2 * qz * drot[6] + 2 * w * drot[7] - 4 * qx * drot[8];
        dqn[2] = -4 * qy * drot[0] + 2 * qx * drot[1] + 2 * w * drot[2] + 2 * qx * drot[3] + 2 * qz * drot[5] -
                 2 * w * drot[6] + 2 * qz * drot[7] - 4 * qy * drot[8];
        dqn[3] = -4 * qz * drot[0] - 2 * w * drot[1] + 2 * qx * drot[2] + 2 * w * drot[3] - 4 * qz * drot[4] +
                 2 * qy * drot[5] + 2 * qx * drot[6] + 2 * qy * drot[7];
        const float qd = w * dqn[0] + qx * dqn[1] + qy * dqn[2] + qz * dqn[3];
        dq[0] += (dqn[0] - w * qd) * st.qinv;
        dq[1] += (dqn[1] - qx * qd) * st.qinv;
        dq[2] += (dqn[2] - qy * qd) * st.qinv;
        dq[3] += (dqn[3] - qz * qd) * st.qinv;
        // colour
        float ex = mu[0] - c.campos[0], ey = mu[1] - c.campos[1], ez = mu[2] - c.campos[2];
        const float il = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
        ex *= il; ey *= il; ez *= il;
        float Y[16], dY[16][3];
        sh_basis<D>(ex, ey, ez, Y);
        sh_basis_grad<D>(ex, ey, ez, dY);
        const float grgb[3] = {gr, gg, gb};
        float gch[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float raw = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) raw = __builtin_fmaf(coef[k][ch], Y[k], raw);
            gch[ch] = raw > 0.0f ? grgb[ch] : 0.0f;   // the clamp at 0 passes no gradient
        }
        // d colour / d direction: sum over k of (sum over channels gch coef) dY_k
        float dd[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float wk = gch[0] * coef[k][0] + gch[1] * coef[k][1] + gch[2] * coef[k][2];
            dd[0] += wk * dY[k][0];
            dd[1] += wk * dY[k][1];
            dd[2] += wk * dY[k][2];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) dcoef[k][ch] += gch[ch] * Y[k];
        }
        const float ddot = dd[0] * ex + dd[1] * ey + dd[2] * ez;
        dmu[0] += (dd[0] - ex * ddot) * il;
        dmu[1] += (dd[1] - ey * ddot) * il;
        dmu[2] += (dd[2] - ez * ddot) * il;
    }
    g_means[3 * g] = dmu[0]; g_means[3 * g + 1] = dmu[1]; g_means[3 * g + 2] = dmu[2];
    g_scales[3 * g] = ds[0]; g_scales[3 * g + 1] = ds[1]; g_scales[3 * g + 2] = ds[2];
    *reinterpret_cast<float4*>(g_quats + 4 * g) = make_float4(dq[0], dq[1], dq[2], dq[3]);
    g_opac[g] = dop;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) g_sh[(g * K + k) * 3 + ch] = dcoef[k][ch];
    if (e1) {
        e1[g] += se1;
        e2[g] += se2;
        count[g] += (int32_t)(r1 - r0);
    }
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------
void launch_count(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th, uint32_t* nrec,
                  uint32_t* ntiles, hipStream_t s, uint32_t* key_range) {
    const unsigned blocks = (unsigned)((ga.P + 255) / 256);
    if (!blocks) return;
    hipLaunchKernelGGL(k_count, dim3(blocks), dim3(256), 0, s, ga.means, ga.scales, ga.quats, ga.opac, ga.P, cams,
                       B, tw, th, nrec, ntiles, key_range);
}

__global__ void k_fill_u64_small(unsigned long long* __restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// views per launch of the pre-pass (bounds its scratch to 2 x 64 partials per workgroup)
constexpr int kCountViewsChunk = 64;

size_t count_views_scratch_bytes(int64_t P, int B) {
    return sizeof(unsigned long long) * 2 * (size_t)std::min(B, kCountViewsChunk) *
           (size_t)std::max<int64_t>((P + 255) / 256, 1);
}

void launch_count_views(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th,
                        unsigned long long* counts, unsigned long long* scratch, hipStream_t s) {
    const unsigned blocks = (unsigned)((ga.P + 255) / 256);
    if (!blocks) {
        hipLaunchKernelGGL(k_fill_u64_small, dim3(1), dim3(64), 0, s, counts, 2 * B);
        return;
    }
    for (int v0 = 0; v0 < B; v0 += kCountViewsChunk) {
        const int nb = std::min(kCountViewsChunk, B - v0);
        hipLaunchKernelGGL(k_count_views, dim3(blocks), dim3(256), 0, s, ga.means, ga.scales, ga.quats, ga.opac,
                           ga.P, cams + v0, nb, tw, th, scratch);
        hipLaunchKernelGGL(k_sum_rows_u64, dim3(2 * nb), dim3(256), 0, s, (const unsigned long long*)scratch, blocks,
                           counts + 2 * (size_t)v0);
    }
}

void launch_records(const GaussianArgs& ga, const DevCam* cams, int B, int tw, int th, const uint32_t* rec_off,
                    BlendRec* recs, uint32_t* depth_key, uint2* tile_rect, uint16_t* rec_view, hipStream_t s,
                    const uint32_t* overflow) {
    const unsigned blocks = (unsigned)((ga.P + 63) / 64);
    if (!blocks) return;
#define MVGS_REC(D)                                                                                             \
    hipLaunchKernelGGL(k_records<D>, dim3(blocks), dim3(64), 0, s, ga.means, ga.scales, ga.quats, ga.opac,      \
                       ga.sh, ga.P, cams, B, tw, th, rec_off, recs, depth_key, tile_rect, rec_view, overflow)
    switch (ga.sh_degree) {
        case 0: MVGS_REC(0); break;
        case 1: MVGS_REC(1); break;
        case 2: MVGS_REC(2); break;
        default: MVGS_REC(3); break;
    }
#undef MVGS_REC
}

void launch_preprocess_bwd(const GaussianArgs& ga, const DevCam* cams, const uint32_t* rec_off,
                           const uint16_t* rec_view, const float* acc, const GradArgs& gr, hipStream_t s,
                           const uint32_t* overflow) {
    const unsigned blocks = (unsigned)((ga.P + 255) / 256);
    if (!blocks) return;
#define MVGS_PB(D)                                                                                              \
    hipLaunchKernelGGL(k_preprocess_bwd<D>, dim3(blocks), dim3(256), 0, s, ga.means, ga.scales, ga.quats,       \
                       ga.opac, ga.sh, ga.P, cams, rec_off, rec_view, acc, gr.means, gr.scales, gr.quats, gr.opac,  \
                       gr.sh, gr.e1, gr.e2, gr.count, overflow)
    switch (ga.sh_degree) {
        case 0: MVGS_PB(0); break;
        case 1: MVGS_PB(1); break;
        case 2: MVGS_PB(2); break;
        default: MVGS_PB(3); break;
    }
#undef MVGS_PB
}

}  // namespace mvgs
