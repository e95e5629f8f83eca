// Device-side types and the single-precision projection shared by the mvgs kernels.
//
// Everything here is compiled with -ffp-contract=off: a fused multiply-add appears
// only where __builtin_fmaf is written, so the projection below is one fixed
// sequence of IEEE operations (division and square root correctly rounded). Its
// discrete outputs -- participation, pixel box, tile rectangle, depth key and the
// per-pixel cut test -- are therefore reproducible bit for bit by any
// implementation of the same sequence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mvgs {

// Per-record accumulator stride (floats) of the blend backward:
// dmx, dmy, dca, dcb, dcc, dopacity, dr, dg, db, E1 term, 2 spare.
constexpr int kAccStride = 12;

constexpr float kNear = 0.2f;          // near plane (camera-space z)
constexpr float kDilation = 0.3f;      // px^2 added to the 2D covariance diagonal
constexpr float kPowerFloor = -4.5f;   // 3-sigma ellipse: power = -0.5 d^T conic d >= -4.5
constexpr float kAlphaMin = 255.0f;    // alpha >= 1/255  <=>  power >= -ln(255 o)
constexpr float kAlphaMax = 0.99f;     // alpha clamp
constexpr float kTStop = 1e-4f;        // stop before transmittance falls below this

// One camera as the kernels see it.
struct DevCam {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float bg[3];
    float campos[3];         // camera centre -R^T t
    int32_t W, H;
    int32_t tiles_x, tiles_y;
    uint32_t tile_base;      // global id of this view's first tile
    uint32_t pix_base;       // offset of this view's first pixel in per-pixel arrays
};

// the view holding global tile id `tile` (views in increasing tile_base)
__device__ __forceinline__ int find_view(const DevCam* __restrict__ cams, int B, uint32_t tile) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cams[mid].tile_base <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Blend record of one participating (view, Gaussian): 64 bytes, four dwordx4. The exponent is
// held in base 2 (every term times log2 e), so that a pixel's weight is one exp2 of its power.
struct alignas(16) BlendRec {
    uint32_t boxx;   // x0 | x1 << 16 (inclusive pixel box)
    uint32_t boxy;   // y0 | y1 << 16
    float mx, my;    // projected mean (pixels)
    float hca, nb, hcc, o;   // log2 e times (-0.5*conic_xx, -conic_xy, -0.5*conic_yy); opacity
    float cut, unused, r, g; // cut threshold on that base-2 power (the clamp is min(o G, 0.99)); colour
    float b;
    uint32_t gid;    // Gaussian index
    uint32_t view;
    uint32_t depth_bits;   // IEEE bits of the camera-space depth
};
static_assert(sizeof(BlendRec) == 64, "BlendRec must be 64 bytes");

__device__ __forceinline__ uint32_t f2u(float f) { return __float_as_uint(f); }

// ln(x) for the opacity thresholds: x = 2^e m, m in [sqrt(1/2), sqrt(2)],
// ln m = 2 atanh(s) with s = (m-1)/(m+1), series through s^9. Non-positive or NaN -> -inf.
__device__ __forceinline__ float ln_threshold(float x) {
    if (!(x > 0.0f)) return -__builtin_inff();
    if (x == __builtin_inff()) return __builtin_inff();
    int e = 0;
    uint32_t b = __float_as_uint(x);
    if (b < 0x00800000u) {
        x = x * 8388608.0f;  // 2^23, exact
        b = __float_as_uint(x);
        e = -23;
    }
    e += (int)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x007fffffu) | 0x3f800000u);
    if (m > 1.41421356f) {
        m = m * 0.5f;
        e += 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float s2 = s * s;
    float p = 0.111111111f;
    p = __builtin_fmaf(p, s2, 0.142857143f);
    p = __builtin_fmaf(p, s2, 0.2f);
    p = __builtin_fmaf(p, s2, 0.333333333f);
    const float s_2 = s + s;
    const float lnm = __builtin_fmaf(s_2 * s2, p, s_2);
    return __builtin_fmaf((float)e, 0.693147182f, lnm);
}

// Quantities of the projection that the backward reuses.
struct ProjState {
    float tx, ty, tz, iz;
    float qw, qx, qy, qz, qinv;       // normalised quaternion and 1/|q|
    float rot[9];                     // rotation of the normalised quaternion
    float S[6];                       // Sigma: xx xy xz yy yz zz
    float T0[3], T1[3];               // J W (rows)
    float a, b, c;                    // dilated Sigma' entries
    float ca, cb, cc;                 // conic
};

struct ProjOut {
    bool ok;
    float mx, my, depth;
    float hca, nb, hcc, cut;
    int32_t x0, x1, y0, y1;
};

// The view-independent part of the projection (paper Sec. 3): normalised quaternion, its
// rotation, Sigma = R S S^T R^T, and the cut threshold of the opacity. Computed once
// per Gaussian; project() below then works view by view. The operations are those of the fixed
// order described at the top of this file, only not repeated per view.
struct GaussGeom {
    bool ok;                          // the quaternion is not degenerate
    float qw, qx, qy, qz, qinv;
    float rot[9];
    float S[6];                       // Sigma: xx xy xz yy yz zz
    float cut;
};

__device__ __forceinline__ void gauss_geom(const float s[3], const float q[4], float o, GaussGeom& g) {
    const float n2 = __builtin_fmaf(q[0], q[0], __builtin_fmaf(q[1], q[1], __builtin_fmaf(q[2], q[2], q[3] * q[3])));
    g.ok = n2 > 0.0f;
    const float inv = 1.0f / sqrtf(n2);
    g.qinv = inv;
    const float qw = q[0] * inv, qx = q[1] * inv, qy = q[2] * inv, qz = q[3] * inv;
    g.qw = qw; g.qx = qx; g.qy = qy; g.qz = qz;
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    float* r = g.rot;
    r[0] = 1.0f - 2.0f * (yy + zz);
    r[1] = 2.0f * (xy - wz);
    r[2] = 2.0f * (xz + wy);
    r[3] = 2.0f * (xy + wz);
    r[4] = 1.0f - 2.0f * (xx + zz);
    r[5] = 2.0f * (yz - wx);
    r[6] = 2.0f * (xz - wy);
    r[7] = 2.0f * (yz + wx);
    r[8] = 1.0f - 2.0f * (xx + yy);
    float M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[3 * i + j] = r[3 * i + j] * s[j];
    g.S[0] = __builtin_fmaf(M[0], M[0], __builtin_fmaf(M[1], M[1], M[2] * M[2]));
    g.S[1] = __builtin_fmaf(M[0], M[3], __builtin_fmaf(M[1], M[4], M[2] * M[5]));
    g.S[2] = __builtin_fmaf(M[0], M[6], __builtin_fmaf(M[1], M[7], M[2] * M[8]));
    g.S[3] = __builtin_fmaf(M[3], M[3], __builtin_fmaf(M[4], M[4], M[5] * M[5]));
    g.S[4] = __builtin_fmaf(M[3], M[6], __builtin_fmaf(M[4], M[7], M[5] * M[8]));
    g.S[5] = __builtin_fmaf(M[6], M[6], __builtin_fmaf(M[7], M[7], M[8] * M[8]));
    const float lc = -ln_threshold(kAlphaMin * o);
    g.cut = (lc > kPowerFloor) ? lc : kPowerFloor;
}

// EWA projection of one Gaussian (its view-independent part in g) into one camera (paper Sec. 3),
// in the fixed operation order described at the top of this file.
__device__ __forceinline__ ProjOut project(const float mu[3], const GaussGeom& g, const DevCam& c, ProjState& st) {
    ProjOut out;
    out.ok = false;
    const float tx = __builtin_fmaf(c.R[0], mu[0], __builtin_fmaf(c.R[1], mu[1], __builtin_fmaf(c.R[2], mu[2], c.t[0])));
    const float ty = __builtin_fmaf(c.R[3], mu[0], __builtin_fmaf(c.R[4], mu[1], __builtin_fmaf(c.R[5], mu[2], c.t[1])));
    const float tz = __builtin_fmaf(c.R[6], mu[0], __builtin_fmaf(c.R[7], mu[1], __builtin_fmaf(c.R[8], mu[2], c.t[2])));
    out.depth = tz;
    st.tx = tx; st.ty = ty; st.tz = tz;
    if (!(tz > kNear)) return out;
    const float iz = 1.0f / tz;
    st.iz = iz;
    const float u = c.fx * tx;
    const float w = c.fy * ty;
    out.mx = __builtin_fmaf(u, iz, c.cx);
    out.my = __builtin_fmaf(w, iz, c.cy);

    if (!g.ok) return out;
    st.qinv = g.qinv;
    st.qw = g.qw; st.qx = g.qx; st.qy = g.qy; st.qz = g.qz;
#pragma unroll
    for (int k = 0; k < 9; ++k) st.rot[k] = g.rot[k];
    const float S00 = g.S[0], S01 = g.S[1], S02 = g.S[2], S11 = g.S[3], S12 = g.S[4], S22 = g.S[5];
    st.S[0] = S00; st.S[1] = S01; st.S[2] = S02; st.S[3] = S11; st.S[4] = S12; st.S[5] = S22;
    const float Sm[9] = {S00, S01, S02, S01, S11, S12, S02, S12, S22};

    const float j00 = c.fx * iz;
    const float j11 = c.fy * iz;
    const float j02 = -(j00 * (tx * iz));
    const float j12 = -(j11 * (ty * iz));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        st.T0[k] = __builtin_fmaf(j00, c.R[k], j02 * c.R[6 + k]);
        st.T1[k] = __builtin_fmaf(j11, c.R[3 + k], j12 * c.R[6 + k]);
    }
    float U0[3], U1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        U0[k] = __builtin_fmaf(st.T0[0], Sm[k], __builtin_fmaf(st.T0[1], Sm[3 + k], st.T0[2] * Sm[6 + k]));
        U1[k] = __builtin_fmaf(st.T1[0], Sm[k], __builtin_fmaf(st.T1[1], Sm[3 + k], st.T1[2] * Sm[6 + k]));
    }
    const float a = __builtin_fmaf(U0[0], st.T0[0], __builtin_fmaf(U0[1], st.T0[1], U0[2] * st.T0[2])) + kDilation;
    const float b = __builtin_fmaf(U0[0], st.T1[0], __builtin_fmaf(U0[1], st.T1[1], U0[2] * st.T1[2]));
    const float cq = __builtin_fmaf(U1[0], st.T1[0], __builtin_fmaf(U1[1], st.T1[1], U1[2] * st.T1[2])) + kDilation;
    st.a = a; st.b = b; st.c = cq;

    const float det = __builtin_fmaf(a, cq, -(b * b));
    if (!(det > 0.0f)) return out;
    const float idet = 1.0f / det;
    const float ca = cq * idet;
    const float cb = -(b * idet);
    const float cc = a * idet;
    st.ca = ca; st.cb = cb; st.cc = cc;
    out.hca = -0.5f * ca;
    out.nb = -cb;
    out.hcc = -0.5f * cc;

    out.cut = g.cut;

    // footprint: per-axis half-extents of the cut ellipse {d : -0.5 d^T conic d >= cut},
    // sqrt(-2 cut Sigma'_xx) and sqrt(-2 cut Sigma'_yy), in whole pixels
    const float nc = -2.0f * out.cut;
    const float rx = ceilf(sqrtf(nc * a));
    const float ry = ceilf(sqrtf(nc * cq));

    float x0 = floorf(out.mx - rx), x1 = floorf(out.mx + rx);
    float y0 = floorf(out.my - ry), y1 = floorf(out.my + ry);
    const float wmax = (float)(c.W - 1), hmax = (float)(c.H - 1);
    if (x0 < 0.0f) x0 = 0.0f;
    if (y0 < 0.0f) y0 = 0.0f;
    if (x1 > wmax) x1 = wmax;
    if (y1 > hmax) y1 = hmax;
    if (!(x0 <= x1) || !(y0 <= y1)) return out;
    out.x0 = (int32_t)x0;
    out.x1 = (int32_t)x1;
    out.y0 = (int32_t)y0;
    out.y1 = (int32_t)y1;
    out.ok = true;
    return out;
}

// The projection of one Gaussian into one camera from its parameters.
__device__ __forceinline__ ProjOut project(const float mu[3], const float s[3], const float q[4], float o,
                                           const DevCam& c, ProjState& st) {
    GaussGeom g;
    gauss_geom(s, q, o, g);
    return project(mu, g, c, st);
}

// power = -0.5 d^T conic d at pixel (px, py), d = pixel centre - mean: the cut test's operand,
// evaluated as dy (hcc dy + nb dx) + hca dx dx. The column terms (PowerX) are shared by every
// pixel of a lane's column.
struct PowerX {
    float dx, ax, bx;
};

__device__ __forceinline__ PowerX power_x(float px, float mx, float hca, float nb) {
    const float dx = px - mx;
    return PowerX{dx, (hca * dx) * dx, nb * dx};
}

__device__ __forceinline__ float power_dy(const PowerX& t, float dy, float hcc) {
    return __builtin_fmaf(dy, __builtin_fmaf(hcc, dy, t.bx), t.ax);
}

__device__ __forceinline__ float power_y(const PowerX& t, float py, float my, float hcc) {
    return power_dy(t, py - my, hcc);
}

__device__ __forceinline__ float pixel_power(float px, float py, float mx, float my, float hca, float nb, float hcc) {
    return power_y(power_x(px, mx, hca, nb), py, my, hcc);
}

// ---------------------------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, Condon-Shortley phase, index l^2 + l + m
// (Cartesian polynomials on the unit direction (x, y, z)).
// ---------------------------------------------------------------------------------------------
constexpr float kSH0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float kSH1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float kSH2a = 1.0925484305920792f;   // sqrt(15 / (4 pi))
constexpr float kSH2b = 0.31539156525252005f;  // sqrt(5 / (16 pi))
constexpr float kSH2c = 0.54627421529603959f;  // sqrt(15 / (16 pi))
constexpr float kSH3a = 0.59004358992664352f;  // sqrt(35 / (32 pi))
constexpr float kSH3b = 2.8906114426405538f;   // sqrt(105 / (4 pi))
constexpr float kSH3c = 0.45704579946446572f;  // sqrt(21 / (32 pi))
constexpr float kSH3d = 0.37317633259011546f;  // sqrt(7 / (16 pi))
constexpr float kSH3e = 1.4453057213202769f;   // sqrt(105 / (16 pi))

template <int D>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
    Y[0] = kSH0;
    if (D >= 1) {
        Y[1] = -kSH1 * y;
        Y[2] = kSH1 * z;
        Y[3] = -kSH1 * x;
    }
    if (D >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = kSH2a * x * y;
        Y[5] = -kSH2a * y * z;
        Y[6] = kSH2b * (2.0f * zz - xx - yy);
        Y[7] = -kSH2a * x * z;
        Y[8] = kSH2c * (xx - yy);
        if (D >= 3) {
            Y[9] = -kSH3a * y * (3.0f * xx - yy);
            Y[10] = kSH3b * x * y * z;
            Y[11] = -kSH3c * y * (4.0f * zz - xx - yy);
            Y[12] = kSH3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -kSH3c * x * (4.0f * zz - xx - yy);
            Y[14] = kSH3e * z * (xx - yy);
            Y[15] = -kSH3a * x * (xx - 3.0f * yy);
        }
    }
}

// Gradient of each basis polynomial above with respect to (x, y, z): dY[k] = (d/dx, d/dy, d/dz).
template <int D>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float (*dY)[3]) {
    dY[0][0] = dY[0][1] = dY[0][2] = 0.0f;
    if (D >= 1) {
        dY[1][0] = 0.0f; dY[1][1] = -kSH1; dY[1][2] = 0.0f;
        dY[2][0] = 0.0f; dY[2][1] = 0.0f; dY[2][2] = kSH1;
        dY[3][0] = -kSH1; dY[3][1] = 0.0f; dY[3][2] = 0.0f;
    }
    if (D >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        dY[4][0] = kSH2a * y; dY[4][1] = kSH2a * x; dY[4][2] = 0.0f;
        dY[5][0] = 0.0f; dY[5][1] = -kSH2a * z; dY[5][2] = -kSH2a * y;
        dY[6][0] = -2.0f * kSH2b * x; dY[6][1] = -2.0f * kSH2b * y; dY[6][2] = 4.0f * kSH2b * z;
        dY[7][0] = -kSH2a * z; dY[7][1] = 0.0f; dY[7][2] = -kSH2a * x;
        dY[8][0] = 2.0f * kSH2c * x; dY[8][1] = -2.0f * kSH2c * y; dY[8][2] = 0.0f;
        if (D >= 3) {
            dY[9][0] = -kSH3a * 6.0f * x * y;
            dY[9][1] = -kSH3a * (3.0f * xx - 3.0f * yy);
            dY[9][2] = 0.0f;
            dY[10][0] = kSH3b * y * z; dY[10][1] = kSH3b * x * z; dY[10][2] = kSH3b * x * y;
            dY[11][0] = kSH3c * 2.0f * x * y;
            dY[11][1] = -kSH3c * (4.0f * zz - xx - 3.0f * yy);
            dY[11][2] = -kSH3c * 8.0f * y * z;
            dY[12][0] = -kSH3d * 6.0f * x * z;
            dY[12][1] = -kSH3d * 6.0f * y * z;
            dY[12][2] = kSH3d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
            dY[13][0] = -kSH3c * (4.0f * zz - 3.0f * xx - yy);
            dY[13][1] = kSH3c * 2.0f * x * y;
            dY[13][2] = -kSH3c * 8.0f * x * z;
            dY[14][0] = kSH3e * 2.0f * x * z; dY[14][1] = -kSH3e * 2.0f * y * z; dY[14][2] = kSH3e * (xx - yy);
            dY[15][0] = -kSH3a * (3.0f * xx - 3.0f * yy);
            dY[15][1] = kSH3a * 6.0f * x * y;
            dY[15][2] = 0.0f;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of m below this lane
__device__ __forceinline__ int rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Order LDS traffic of one wavefront without a workgroup barrier.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 64 lanes with DPP row operations; every lane receives the total.
__device__ __forceinline__ float wave_sum(float v) {
    // within rows of 16 lanes
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xf, 0xf, false)); // row_shr:1
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x112, 0xf, 0xf, false)); // row_shr:2
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x114, 0xf, 0xf, false)); // row_shr:4 (after 1,2 partial sums of 4)
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x118, 0xf, 0xf, false)); // row_shr:8
    // lane 15 of each row now holds its row sum; combine rows
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x142, 0xa, 0xf, false)); // row_bcast:15
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x143, 0xc, 0xf, false)); // row_bcast:31
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

}  // namespace mvgs
