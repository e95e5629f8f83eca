// Device helpers shared by the full-tile blend kernels and the partial-rendering kernels:
// record loads through the scalar unit, candidate culling, the per-pixel forward step of
// Eq. 1, the per-pixel reverse step and the wavefront reduction of per-Gaussian sums.
#pragma once

#include "mvgs_kernels.h"

namespace mvgs {


// Contiguous tile runs per XCD: block b is dispatched to XCD b % 8.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7u, k = b >> 3;
    const uint32_t q = n >> 3, rem = n & 7u;
    return x * q + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ bool box_misses(uint32_t bx, uint32_t by, int sx0, int sx1, int sy0, int sy1) {
    return (int)(bx & 0xffffu) > sx1 || (int)(bx >> 16) < sx0 || (int)(by & 0xffffu) > sy1 || (int)(by >> 16) < sy0;
}

// a record's exponent is in base 2 already (BlendRec)
__device__ __forceinline__ float weight_of(float power2) { return __builtin_amdgcn_exp2f(power2); }

// Wavefront-uniform copy of the fields the walks use.
struct RecS {
    float mx, my, hca, nb, hcc, o, cut, r, g, b, z;
};

__device__ __forceinline__ RecS load_rec(const BlendRec* __restrict__ recs, uint32_t r) {
    const BlendRec* R = recs + r;
    RecS s;
    s.mx = R->mx; s.my = R->my; s.hca = R->hca; s.nb = R->nb; s.hcc = R->hcc; s.o = R->o;
    s.cut = R->cut; s.r = R->r; s.g = R->g; s.b = R->b;
    s.z = __uint_as_float(R->depth_bits);
    return s;
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Largest power -0.5 d^T conic d over the rectangle [xa, xb] x [ya, yb] of pixel centres (d = p - mean),
// with power(d) = dx (hca dx + nb dy) + hcc dy^2, concave: 0 if the mean is inside, else the best of
// the four edges, each maximised in closed form and clamped to the edge. Also returns the size of
// the terms at that point, which bounds its rounding error.
__device__ __forceinline__ float rect_max_power(float mx, float my, float hca, float nb, float hcc, float xa,
                                               float xb, float ya, float yb, float& mag) {
    const float ax = xa - mx, bx = xb - mx, ay = ya - my, by = yb - my;
    if (ax <= 0.0f && bx >= 0.0f && ay <= 0.0f && by >= 0.0f) {
        mag = 0.0f;
        return 0.0f;
    }
    float best = -__builtin_inff();
    mag = 0.0f;
    // The stationary points only choose where on an edge to evaluate the quadratic; near them it
    // is flat, so the hardware reciprocal (about 1 ulp) moves the value by far less than the slack.
    const float ry = -nb * __builtin_amdgcn_rcpf(2.0f * hcc), rx = -nb * __builtin_amdgcn_rcpf(2.0f * hca);
    // edges x = const: maximise over dy at dy* = -nb dx / (2 hcc)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dx = e ? bx : ax;
        float dy = ry * dx;
        dy = fminf(fmaxf(dy, ay), by);
        const float t1 = hca * dx * dx, t2 = nb * dx * dy, t3 = hcc * dy * dy;
        const float p = t1 + t2 + t3;
        if (p > best) {
            best = p;
            mag = fabsf(t1) + fabsf(t2) + fabsf(t3);
        }
    }
    // edges y = const: maximise over dx at dx* = -nb dy / (2 hca)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float dy = e ? by : ay;
        float dx = rx * dy;
        dx = fminf(fmaxf(dx, ax), bx);
        const float t1 = hca * dx * dx, t2 = nb * dx * dy, t3 = hcc * dy * dy;
        const float p = t1 + t2 + t3;
        if (p > best) {
            best = p;
            mag = fabsf(t1) + fabsf(t2) + fabsf(t3);
        }
    }
    return best;
}

// Candidate window: lane k looks at list entry base + k and keeps it if the Gaussian's cut ellipse
// reaches a pixel centre of the wavefront's sub-tile: first the pixel box, then the ellipse itself.
// The ellipse test only ever keeps too much (a slack far above float32 rounding), so culling never
// changes a result; it only spares the wavefront Gaussians that no pixel of its sub-tile accepts.
// window_load issues the loads the test starts with (the entry and its record's pixel box and mean),
// so that a walk can have the next window's in flight while it blends the current one (the full-tile
// forward does: 0.661 -> 0.645 ms on the 1M x 8 batch; the backward gained nothing from it).
struct WindowPre {
    uint32_t rl;   // the entry's record (0 past the end)
    float4 q0;     // its pixel box and mean
    bool in;
};

__device__ __forceinline__ WindowPre window_load(const uint32_t* __restrict__ vals,
                                                 const BlendRec* __restrict__ recs, uint32_t base, uint32_t end,
                                                 int lane) {
    WindowPre w;
    const uint32_t idx = base + (uint32_t)lane;
    w.in = idx < end;
    w.rl = 0;
    w.q0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (w.in) {
        w.rl = vals[idx];
        w.q0 = *reinterpret_cast<const float4*>(recs + w.rl);
    }
    return w;
}

__device__ __forceinline__ uint64_t window_test(const WindowPre& w, const BlendRec* __restrict__ recs, int sx0,
                                                int sx1, int sy0, int sy1) {
    bool keep = false;
    if (w.in) {
        keep = !box_misses(__float_as_uint(w.q0.x), __float_as_uint(w.q0.y), sx0, sx1, sy0, sy1);
        if (keep) {
            const float4 q1 = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(recs + w.rl) + 4);
            const float cut = reinterpret_cast<const float*>(recs + w.rl)[8];
            float mag;
            const float pm = rect_max_power(w.q0.z, w.q0.w, q1.x, q1.y, q1.z, (float)sx0 + 0.5f, (float)sx1 + 0.5f,
                                            (float)sy0 + 0.5f, (float)sy1 + 0.5f, mag);
            keep = pm >= cut - (1e-2f + 1e-5f * mag);
        }
    }
    return ballot64(keep);
}

__device__ __forceinline__ uint64_t window_mask(const uint32_t* __restrict__ vals, const BlendRec* __restrict__ recs,
                                                uint32_t base, uint32_t end, int lane, int sx0, int sx1, int sy0,
                                                int sy1, uint32_t& rl) {
    const WindowPre w = window_load(vals, recs, base, end, lane);
    rl = w.rl;
    return window_test(w, recs, sx0, sx1, sy0, sy1);
}

// Bounding rectangle [ax0, ax1] x [ay0, ay1] of the pixels of a wavefront's SW-wide sub-tile (at
// sx0, sy0; lane l owns column l % SW and rows l / SW + (64 / SW) k, k < PPL) whose bit is set in
// the ballots m[k] (pixel k of each lane); at least one bit must be set. Scalar work only: the
// walks shrink the rectangle their candidates are culled against to the pixels that can still
// take a Gaussian (live in the forward, before their last contributor in the backward), so a
// candidate that reaches only stopped or finished pixels is not loaded.
template <int PPL, int SW>
__device__ __forceinline__ void active_rect(const uint64_t (&m)[PPL], int sx0, int sy0, int& ax0, int& ax1, int& ay0,
                                            int& ay1) {
    constexpr int ROWS = 64 / SW;
    constexpr uint64_t kCols = (1ull << SW) - 1ull;
    uint64_t cols = 0;
    uint32_t rows = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k)
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const uint64_t c = (m[k] >> (r * SW)) & kCols;
            cols |= c;
            rows |= (c != 0ull ? 1u : 0u) << (r + ROWS * k);
        }
    ax0 = sx0 + __builtin_ctzll(cols);
    ax1 = sx0 + 63 - __builtin_clzll(cols);
    ay0 = sy0 + __builtin_ctz(rows);
    ay1 = sy0 + 31 - __builtin_clz(rows);
}

// T carries the pixel's state in its sign: a stopped (or unselected) pixel holds -T, so one
// comparison tells a live pixel and no separate flag has to be kept per candidate. Transmittance
// is |T| (at least 1e-4 while live).
struct FwdPix {
    float T, C0, C1, C2;
    uint32_t last;
    float D;   // blended camera-space depth (accumulated only where asked for)
};

__device__ __forceinline__ bool pix_live(const FwdPix& st) { return st.T > 0.0f; }

// One Gaussian of Eq. 1 for one pixel (skipped when the pixel has stopped or the cut test fails:
// the power is computed for every lane and both tests share one branch).
template <bool DEPTH>
__device__ __forceinline__ void blend_step(FwdPix& st, const RecS& q, const PowerX& t, float py, uint32_t pos) {
    const float power = power_y(t, py, q.my, q.hcc);
    if (pix_live(st) & (power >= q.cut)) {
        const float alpha = fminf(q.o * weight_of(power), kAlphaMax);
        const float Tn = __builtin_fmaf(-st.T, alpha, st.T);
        if (Tn < kTStop) {
            st.T = -st.T;
        } else {
            const float w = alpha * st.T;
            st.C0 = __builtin_fmaf(q.r, w, st.C0);
            st.C1 = __builtin_fmaf(q.g, w, st.C1);
            st.C2 = __builtin_fmaf(q.b, w, st.C2);
            if (DEPTH) st.D = __builtin_fmaf(q.z, w, st.D);
            st.T = Tn;
            st.last = pos + 1;
        }
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

struct BwdPix {
    float T, dC0, dC1, dC2, Rb0, Rb1, Rb2;
    float py;
    uint32_t last;
};

// Per-lane sums of one Gaussian's gradient contributions over the lane's pixels. Without E1 the
// field o first holds s0 = sum dpow, with dpow = dalpha alpha = w (dC . (c - behind)) for an
// unclamped pixel, and s1 = sum dpow dy, s2 = sum dpow dy^2 (the lane's pixels share dx);
// unblend_step expands them once, the opacity gradient sum dalpha G being s0 / o.
struct BwdSum {
    float mx, my, ca, cb, cc, o, r, g, b, e1;
    float s1, s2;
    bool contrib;
};

// CHECK = false: the caller knows pos < st.last for every pixel that can contribute (a pixel
// without contributors holds T = 0 and dC = 0, so it adds nothing).
template <bool E1, bool CHECK>
__device__ __forceinline__ void unblend_pixel(BwdPix& st, BwdSum& a, const RecS& q, uint32_t pos, const PowerX& t,
                                              float half_w, float half_h) {
    const float dx = t.dx, dy = st.py - q.my;
    const float power = power_dy(t, dy, q.hcc);
    if (!((!CHECK | (pos < st.last)) & (power >= q.cut))) return;   // one branch for both tests
    a.contrib = true;
    const float G = weight_of(power);
    const float oG = q.o * G;
    const bool clamped = oG > kAlphaMax;   // the forward's min(o G, kAlphaMax), decided alike
    const float alpha = clamped ? kAlphaMax : oG;
    st.T = st.T * __builtin_amdgcn_rcpf(1.0f - alpha);   // transmittance in front of this Gaussian
    const float w = alpha * st.T;
    a.r = __builtin_fmaf(st.dC0, w, a.r);
    a.g = __builtin_fmaf(st.dC1, w, a.g);
    a.b = __builtin_fmaf(st.dC2, w, a.b);
    // fused: the build keeps contraction off, so the dot product is written with explicit FMAs
    const float dot = __builtin_fmaf(st.dC0, q.r - st.Rb0, __builtin_fmaf(st.dC1, q.g - st.Rb1, st.dC2 * (q.b - st.Rb2)));
    st.Rb0 = __builtin_fmaf(q.r - st.Rb0, alpha, st.Rb0);
    st.Rb1 = __builtin_fmaf(q.g - st.Rb1, alpha, st.Rb1);
    st.Rb2 = __builtin_fmaf(q.b - st.Rb2, alpha, st.Rb2);
    if (clamped) return;
    if (E1) {
        const float dalpha = st.T * dot;
        a.o = __builtin_fmaf(dalpha, G, a.o);
        const float dpow = dalpha * alpha;
        // the per-pixel positional gradient is needed for its norm (natural-log conic terms)
        const float ca = (-2.0f * kLn2) * q.hca, cbq = -kLn2 * q.nb, cc = (-2.0f * kLn2) * q.hcc;
        const float gx = dpow * (ca * dx + cbq * dy);
        const float gy = dpow * (cbq * dx + cc * dy);
        a.mx += gx;
        a.my += gy;
        a.ca = __builtin_fmaf(-0.5f * dpow, dx * dx, a.ca);
        a.cb = __builtin_fmaf(-dpow, dx * dy, a.cb);
        a.cc = __builtin_fmaf(-0.5f * dpow, dy * dy, a.cc);
        const float nx = gx * half_w, ny = gy * half_h;
        a.e1 += sqrtf(nx * nx + ny * ny);
    } else {
        const float dpow = w * dot;
        const float dpy = dpow * dy;
        a.o += dpow;
        a.s1 += dpy;
        a.s2 = __builtin_fmaf(dpy, dy, a.s2);
    }
}

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_mov(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old), __builtin_bit_cast(int, v),
                                                                 CTRL, ROW_MASK, BANK_MASK, false));
}

// One halving step of the transposed reduction: of the pair (a, b) a lane keeps a if `hi` is false
// and b otherwise, and adds the same member from its partner across the exchange `xchg`.
template <typename X>
__device__ __forceinline__ float keep_add(float a, float b, bool hi, X xchg) {
    const float send = hi ? a : b;
    const float keep = hi ? b : a;
    return keep + xchg(send);
}

// Sum of ten per-lane values over the wavefront in one pass of halving exchanges (xor 32, 16, 8,
// 4 move half of the values each, xor 2 and 1 finish): afterwards the first lane of quad q holds
// the total of value kQuadValue[q]. Returns that total; *idx receives the value index (or -1).
__device__ __forceinline__ float wave_sum10(const float (&v)[10], int lane, uint32_t bperm32, int* idx) {
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4;
    auto x32 = [&](float t) { return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute((int)bperm32,
                                                                                            __builtin_bit_cast(int, t))); };
    // swizzle bit mode: and_mask 0x1f, xor_mask 0x10 -> lane ^ 16 within each half
    auto x16 = [&](float t) { return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, t),
                                                                                           0x401f)); };
    auto x8 = [&](float t) { return dpp_mov<0x128, 0xf, 0xf>(0.0f, t); };  // row_ror:8 -> lane ^ 8 in a row
    auto x4 = [&](float t) {
        const float up = dpp_mov<0x104, 0xf, 0x5>(0.0f, t);   // row_shl:4 into banks 0, 2 (lane + 4)
        return dpp_mov<0x114, 0xf, 0xa>(up, t);              // row_shr:4 into banks 1, 3 (lane - 4)
    };
    const float r0 = keep_add(v[0], v[1], b5, x32);
    const float r1 = keep_add(v[2], v[3], b5, x32);
    const float r2 = keep_add(v[4], v[5], b5, x32);
    const float r3 = keep_add(v[6], v[7], b5, x32);
    const float r4 = keep_add(v[8], v[9], b5, x32);
    const float s0 = keep_add(r0, r1, b4, x16);
    const float s1 = keep_add(r2, r3, b4, x16);
    const float s2 = keep_add(r4, 0.0f, b4, x16);
    const float u0 = keep_add(s0, s1, b3, x8);
    const float u1 = keep_add(s2, 0.0f, b3, x8);
    float x = keep_add(u0, u1, b2, x4);
    x += dpp_mov<0x4e, 0xf, 0xf>(0.0f, x);   // quad_perm [2,3,0,1]
    x += dpp_mov<0xb1, 0xf, 0xf>(0.0f, x);   // quad_perm [1,0,3,2]
    // value held by lane groups: bit2 = 0 -> u0 (bit3 picks s0/s1), bit2 = 1 -> u1 (s2 if bit3 = 0)
    int k = -1;
    if ((lane & 3) == 0) {
        if (!b2) k = (b3 ? 4 : 0) + (b5 ? 1 : 0) + (b4 ? 2 : 0);
        else if (!b3 && !b4) k = 8 + (b5 ? 1 : 0);
    }
    *idx = k;
    return x;
}

// One Gaussian of the reverse walk for all of this lane's pixels, summed over the wavefront and
// added to the record's accumulators with one atomic instruction.
template <bool E1, int PPL, bool CHECK>
__device__ __forceinline__ void unblend_step(BwdPix (&st)[PPL], const RecS& q, uint32_t r, uint32_t pos, float px,
                                             float half_w, float half_h, int lane, uint32_t bperm32,
                                             float* __restrict__ acc) {
    BwdSum a{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false};
    const PowerX t = power_x(px, q.mx, q.hca, q.nb);
#pragma unroll
    for (int k = 0; k < PPL; ++k) unblend_pixel<E1, CHECK>(st[k], a, q, pos, t, half_w, half_h);
    if (ballot64(a.contrib) == 0) return;
    if (!E1) {
        // sum over the lane's pixels of dpow (ca dx + cb dy, cb dx + cc dy) and -dpow (dx^2 / 2,
        // dx dy, dy^2 / 2), with ca = -2 hca, cb = -nb, cc = -2 hcc in natural-log units (the
        // record's base-2 terms times ln 2)
        const float dx = t.dx;
        const float s0 = a.o, s1 = a.s1, s2 = a.s2;
        a.o = s0 * __builtin_amdgcn_rcpf(q.o);
        const float ca = (-2.0f * kLn2) * q.hca, cb = -kLn2 * q.nb, cc = (-2.0f * kLn2) * q.hcc;
        a.mx = __builtin_fmaf(ca * dx, s0, cb * s1);
        a.my = __builtin_fmaf(cb * dx, s0, cc * s1);
        a.ca = -0.5f * dx * dx * s0;
        a.cb = -dx * s1;
        a.cc = -0.5f * s2;
    }
    const float v[10] = {a.mx, a.my, a.ca, a.cb, a.cc, a.o, a.r, a.g, a.b, E1 ? a.e1 : 0.0f};
    int k;
    const float total = wave_sum10(v, lane, bperm32, &k);
    if (k >= 0 && (E1 || k < 9)) unsafeAtomicAdd(acc + (size_t)r * kAccStride + k, total);
}

// Front-to-back walk of one wavefront over the sorted list [rg.x, rg.y) of its (view, tile): each
// lane blends its PPL pixels (px, py[k]); candidates are culled against the pixel rectangle
// [sx0, sx1] x [sy0, sy1] that holds every pixel of the wavefront. Ends when all lanes stopped.
template <int PPL, bool DEPTH = false>
__device__ __forceinline__ void walk_forward(FwdPix (&st)[PPL], float px, const float (&py)[PPL], uint2 rg,
                                             const uint32_t* __restrict__ vals, const BlendRec* __restrict__ recs,
                                             int lane, int sx0, int sx1, int sy0, int sy1) {
    for (uint32_t base = rg.x; base < rg.y; base += 64) {
        bool live = false;
#pragma unroll
        for (int k = 0; k < PPL; ++k) live |= pix_live(st[k]);
        if (ballot64(live) == 0) break;
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
            const PowerX t0 = power_x(px, q0.mx, q0.hca, q0.nb);
#pragma unroll
            for (int k = 0; k < PPL; ++k) blend_step<DEPTH>(st[k], q0, t0, py[k], base + (uint32_t)j0);
            if (h1) {
                const PowerX t1 = power_x(px, q1.mx, q1.hca, q1.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<DEPTH>(st[k], q1, t1, py[k], base + (uint32_t)j1);
            }
            if (h2) {
                const PowerX t2 = power_x(px, q2.mx, q2.hca, q2.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<DEPTH>(st[k], q2, t2, py[k], base + (uint32_t)j2);
            }
            if (h3) {
                const PowerX t3 = power_x(px, q3.mx, q3.hca, q3.nb);
#pragma unroll
                for (int k = 0; k < PPL; ++k) blend_step<DEPTH>(st[k], q3, t3, py[k], base + (uint32_t)j3);
            }
        }
    }
}

// The surviving candidates m of one window (list positions base + j), highest position first, up
// to four records per round trip through the scalar cache.
template <bool E1, int PPL, bool CHECK>
__device__ __forceinline__ void unblend_window(BwdPix (&st)[PPL], float px, uint64_t m, uint32_t rl, uint32_t base,
                                               const BlendRec* __restrict__ recs, int lane, uint32_t bperm32,
                                               float half_w, float half_h, float* __restrict__ acc) {
    while (m) {
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
        unblend_step<E1, PPL, CHECK>(st, q0, r0, base + (uint32_t)j0, px, half_w, half_h, lane, bperm32, acc);
        if (h1) unblend_step<E1, PPL, CHECK>(st, q1, r1, base + (uint32_t)j1, px, half_w, half_h, lane, bperm32, acc);
        if (h2) unblend_step<E1, PPL, CHECK>(st, q2, r2, base + (uint32_t)j2, px, half_w, half_h, lane, bperm32, acc);
        if (h3) unblend_step<E1, PPL, CHECK>(st, q3, r3, base + (uint32_t)j3, px, half_w, half_h, lane, bperm32, acc);
    }
}

// Reverse walk of one wavefront from list position hi_end down to rg.x (Eq. 1 differentiated):
// per Gaussian, the lanes' contributions are summed over the wavefront and added to the record's
// accumulators with one atomic instruction. SW > 0: the lanes' pixels form an SW-wide sub-tile
// (see active_rect) and each window of candidates is culled against the pixels whose last
// contributor lies above it; SW = 0: against the fixed rectangle [sx0, sx1] x [sy0, sy1].
// lo_end: every pixel of the wavefront either has its last contributor at or above lo_end or
// has none (and then T = 0, dC = 0); without E1, windows below it skip the per-pixel position
// test. 0 keeps the test everywhere.
template <bool E1, int PPL, int SW = 0>
__device__ __forceinline__ void walk_backward(BwdPix (&st)[PPL], float px, uint32_t hi_end, uint32_t lo_end, uint2 rg,
                                              const uint32_t* __restrict__ vals, const BlendRec* __restrict__ recs,
                                              int lane, int sx0, int sx1, int sy0, int sy1, float half_w,
                                              float half_h, float* __restrict__ acc) {
    const uint32_t bperm32 = (uint32_t)((lane ^ 32) << 2);

    for (uint32_t top = hi_end; top > rg.x;) {
        const uint32_t base = top - rg.x > 64u ? top - 64u : rg.x;
        int ax0 = sx0, ax1 = sx1, ay0 = sy0, ay1 = sy1;
        if constexpr (SW > 0) {
            uint64_t am[PPL];
            uint64_t any = 0;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                am[k] = ballot64(st[k].last > base);
                any |= am[k];
            }
            if (any == 0) {   // no pixel takes a Gaussian at or above base
                top = base;
                continue;
            }
            active_rect<PPL, SW>(am, sx0, sy0, ax0, ax1, ay0, ay1);
        }
        uint32_t rl;
        const uint64_t m = window_mask(vals, recs, base, top, lane, ax0, ax1, ay0, ay1, rl);
        if (!E1 && top <= lo_end)   // with E1 the second copy of the loop costs occupancy
            unblend_window<E1, PPL, false>(st, px, m, rl, base, recs, lane, bperm32, half_w, half_h, acc);
        else
            unblend_window<E1, PPL, true>(st, px, m, rl, base, recs, lane, bperm32, half_w, half_h, acc);
        top = base;
    }
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace mvgs
