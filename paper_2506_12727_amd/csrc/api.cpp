// Host runtime of libmvgs: contexts, frames, argument validation, workspace and the
// launch sequence of each public call (see include/mvgs.h for the contract).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mvgs.h"
#include "mvgs_kernels.h"

using namespace mvgs;

namespace {

// Where device memory comes from: the caller's callbacks (mvgs_options.alloc / free), else
// hipMalloc / hipFree.
struct Allocator {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*free)(void*, void*) = nullptr;
    void* ctx = nullptr;
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    const Allocator* al = nullptr;   // the owning context's allocator
};

hipError_t dev_alloc(const Allocator* al, void** p, size_t n) {
    if (al && al->alloc) {
        *p = al->alloc(n, al->ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, n);
}

hipError_t dev_free(const Allocator* al, void* p) {
    if (al && al->free) {
        al->free(p, al->ctx);
        return hipSuccess;
    }
    return hipFree(p);
}

// Capacity a grow-only buffer has after it is asked for `bytes`: unchanged if it already fits,
// else at least a quarter more than before, in whole 4 KiB pages.
size_t grown_capacity(size_t cap, size_t bytes) {
    if (bytes <= cap && cap) return cap;
    size_t n = std::max<size_t>(bytes, 256);
    n = std::max(n, cap + cap / 4);
    return (n + 4095) & ~(size_t)4095;
}
size_t grown_capacity(const DevBuf& b, size_t bytes) { return grown_capacity(b.p ? b.cap : 0, bytes); }

// Grow-only device buffer. Growing frees the old allocation first: hipFree waits for the device;
// a caller's free callback gets the block while work that used it may still be queued on the
// call's stream (the contract of mvgs_options.free: reuse in stream order).
hipError_t ensure(DevBuf& b, size_t bytes) {
    if (bytes <= b.cap && b.p) return hipSuccess;
    const size_t n = grown_capacity(b, bytes);
    if (b.p) {
        hipError_t e = dev_free(b.al, b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.cap = 0;
    }
    hipError_t e = dev_alloc(b.al, &b.p, n);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.cap = n;
    return hipSuccess;
}

void release(DevBuf& b) {
    if (b.p) (void)dev_free(b.al, b.p);
    b.p = nullptr;
    b.cap = 0;
}

template <typename T>
T* as(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

int bits_for(uint64_t n) {  // bits needed to hold values 0..n-1
    int b = 0;
    while (b < 64 && ((uint64_t)1 << b) < n) ++b;
    return b;
}

// Pinned host staging with device twins, used round-robin; a slot is reused only after
// the event recorded behind its last consumer has completed.
struct UploadRing {
    static constexpr int kSlots = 16;
    struct Slot {
        void* host = nullptr;
        DevBuf dev;
        size_t cap = 0;
        hipEvent_t ev = nullptr;
        bool pending = false;
    };
    Slot slots[kSlots];
    int next = 0;
    std::vector<int> used;
    // Staging recorded into a stream capture: one dedicated buffer pair per upload, kept until the
    // context is destroyed, so that every replay of the graph copies the same host memory.
    struct Sticky {
        void* host = nullptr;
        void* dev = nullptr;
        size_t bytes = 0;
    };
    std::vector<Sticky> sticky;

    hipError_t put_sticky(const void* src, size_t bytes, hipStream_t s, void** dev_out, void** host_out) {
        Sticky st;
        st.bytes = std::max<size_t>(bytes, 256);
        // allocations are not stream work; let them through the capture like a caching allocator does
        hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
        hipError_t e = hipThreadExchangeStreamCaptureMode(&mode);
        if (e != hipSuccess) return e;
        e = hipHostMalloc(&st.host, st.bytes, hipHostMallocDefault);
        if (e == hipSuccess) {
            e = hipMalloc(&st.dev, st.bytes);
            if (e != hipSuccess) (void)hipHostFree(st.host);
        }
        hipStreamCaptureMode back = mode;
        (void)hipThreadExchangeStreamCaptureMode(&back);
        if (e != hipSuccess) return e;
        sticky.push_back(st);
        memcpy(st.host, src, bytes);
        e = hipMemcpyAsync(st.dev, st.host, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        *dev_out = st.dev;
        if (host_out) *host_out = st.host;
        return hipSuccess;
    }

    hipError_t put(const void* src, size_t bytes, hipStream_t s, void** dev_out, bool capturing = false,
                   void** host_out = nullptr) {
        if (capturing) return put_sticky(src, bytes, s, dev_out, host_out);
        if (host_out) *host_out = nullptr;
        Slot& sl = slots[next];
        const int idx = next;
        next = (next + 1) % kSlots;
        if (sl.pending) {
            hipError_t e = hipEventSynchronize(sl.ev);
            if (e != hipSuccess) return e;
            sl.pending = false;
        }
        if (!sl.ev) {
            hipError_t e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
            if (e != hipSuccess) return e;
        }
        if (sl.cap < bytes) {
            if (sl.host) (void)hipHostFree(sl.host);
            sl.host = nullptr;
            size_t n = std::max<size_t>(bytes, 4096);
            hipError_t e = hipHostMalloc(&sl.host, n, hipHostMallocDefault);
            if (e != hipSuccess) return e;
            sl.cap = n;
        }
        hipError_t e = ensure(sl.dev, bytes);
        if (e != hipSuccess) return e;
        memcpy(sl.host, src, bytes);
        e = hipMemcpyAsync(sl.dev.p, sl.host, bytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return e;
        used.push_back(idx);
        *dev_out = sl.dev.p;
        return hipSuccess;
    }
    // record completion behind everything enqueued so far on `s` for the slots used by this call
    hipError_t seal(hipStream_t s) {
        hipError_t r = hipSuccess;
        for (int idx : used) {
            hipError_t e = hipEventRecord(slots[idx].ev, s);
            if (e != hipSuccess) r = e;
            else slots[idx].pending = true;
        }
        used.clear();
        return r;
    }
    void destroy() {
        for (auto& st : sticky) {
            if (st.host) (void)hipHostFree(st.host);
            if (st.dev) (void)hipFree(st.dev);
        }
        sticky.clear();
        for (auto& sl : slots) {
            if (sl.pending) (void)hipEventSynchronize(sl.ev);
            if (sl.ev) (void)hipEventDestroy(sl.ev);
            if (sl.host) (void)hipHostFree(sl.host);
            release(sl.dev);
        }
    }
};

}  // namespace

constexpr int kModeFull = -1;  // otherwise MVGS_PARTIAL_COMPACT or MVGS_PARTIAL_MASKED

struct mvgs_frame {
    mvgs_context* ctx = nullptr;
    bool in_use = false;
    uint16_t gen = 0;   // generation of the handle: advanced at each release (see frame_handle)
    int B = 0;
    std::vector<DevCam> hcams;
    uint32_t n_tiles = 0, n_pixels = 0;
    int64_t P = 0;
    int sh_degree = 0;
    int ppl = 1;   // pixels per lane of the full-tile blend kernels (the backward uses the forward's)
    uint32_t V = 0;
    uint64_t K = 0;
    int final_buf = 0;
    bool key16 = false;   // the pair keys are 16-bit tile ids (at most 65,536 tiles)
    int depth_bits = 0, tile_bits = 0;   // key bits the depth and tile sorts ordered
    size_t need_bytes = 0;  // device bytes the forward that made this frame asked for
    // partial rendering: kModeFull renders every pixel; the others a selection (t_final and
    // n_last then hold one entry per selected pixel in thread-efficient mode)
    int mode = kModeFull;
    uint32_t n_sel = 0, n_tasks = 0;
    // capacity mode: sizes are known on the host only after mvgs_frame_check; dtot holds the
    // call's totals (u64 records, pairs, error words) and at byte 32 the clamped counts and the
    // overflow word
    bool capacity = false, checked = true;
    void* cam_stage = nullptr;   // host staging of the cameras when the forward was captured
    // thread-efficient partial frames: whether the selection covers the views' common image plane
    // once (then the merged plane has a 3D loss), and the blended depth per selected pixel
    bool partition = false;
    DevBuf cams, recs, rec_off, rec_view, keys[2], vals[2], ranges, t_final, n_last;
    DevBuf sel_off, sel_pix, mask, task_n, task_off, tasks, dtot, depth, plane_mask;

    template <typename Fn>
    void each_buffer(Fn fn) {
        DevBuf* bufs[] = {&cams, &recs, &rec_off, &rec_view, &keys[0], &keys[1], &vals[0], &vals[1], &ranges,
                          &t_final, &n_last, &sel_off, &sel_pix, &mask, &task_n, &task_off, &tasks, &dtot, &depth,
                          &plane_mask};
        for (DevBuf* b : bufs) fn(*b);
    }
};

struct mvgs_context {
    int device = 0;
    Allocator alloc;   // every DevBuf of the context and of its frames points here
    int tw = 16, th = 16, ppl = 2;
    bool ppl_auto = false;   // pixels per lane chosen per frame (blend_auto_ppl)
    std::string err;
    std::vector<mvgs_frame*> frames;
    DevBuf nrec, ntiles, totals, scan_scratch, depth_key[2], rec_vals[2], tile_rect, sorted_rect;
    DevBuf sort_scratch, acc, loss_scratch, loss3d_scratch, adc_n, adc_off, adc_act, moment_partials;
    DevBuf adam_state;   // 3 words of a device-counted Adam step (allocated with the first device use)
    DevBuf view_counts;  // per-view records and pairs of mvgs_count_views
    size_t limit = 0;  // 0: no workspace limit
    uint64_t cap_v = 0, cap_k = 0;  // capacity mode when non-zero
    // capacity mode: the window of depth keys the depth sort orders, [dwin_base, dwin_base +
    // 2^dwin_bits), set by mvgs_frame_check from the keys of the frames it checks
    uint32_t dwin_base = 0;
    int dwin_bits = 32;
    bool capturing = false;         // the current call's stream is being captured into a graph
    uint64_t* pinned_totals = nullptr;
    uint64_t* pinned_counts = nullptr;   // readback of mvgs_count_views (grown as needed)
    size_t pinned_counts_n = 0;
    bool device_used = false;
    UploadRing ring;

    // opt-in stage timing
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<Mark> marks;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[MVGS_STAGE_COUNT] = {0};
    int64_t prof_calls[MVGS_STAGE_COUNT] = {0};
    DevBuf work;

    template <typename Fn>
    void each_buffer(Fn fn) {
        DevBuf* bufs[] = {&nrec, &ntiles, &totals, &scan_scratch, &depth_key[0], &depth_key[1], &rec_vals[0],
                          &rec_vals[1], &tile_rect, &sorted_rect, &sort_scratch, &acc,
                          &loss_scratch, &loss3d_scratch, &adc_n, &adc_off, &adc_act,
                          &moment_partials, &work, &adam_state, &view_counts};
        for (DevBuf* b : bufs) fn(*b);
        for (auto& sl : ring.slots) fn(sl.dev);
        for (mvgs_frame* f : frames) f->each_buffer(fn);
    }
    // device bytes held now: workspace, upload staging and every frame, live or pooled
    size_t held() {
        size_t n = 0;
        each_buffer([&](DevBuf& b) { n += b.cap; });
        return n;
    }

    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // returns a mark index (or -1 when profiling is off)
    int stage_begin(int stage, hipStream_t s) {
        if (!prof || capturing) return -1;
        Mark m{stage, take_event(), take_event()};
        if (!m.a || !m.b || hipEventRecord(m.a, s) != hipSuccess) return -1;
        marks.push_back(m);
        return (int)marks.size() - 1;
    }
    void stage_end(int idx, hipStream_t s) {
        if (idx >= 0) (void)hipEventRecord(marks[idx].b, s);
    }

    // called first by every call that enqueues work: notes whether the stream is being captured
    bool begin(hipStream_t s) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
        return capturing;
    }

    // first device use: remember the device, allocate the pinned readback slot
    hipError_t bind_device() {
        if (device_used) return hipSuccess;
        hipError_t e = hipGetDevice(&device);
        if (e != hipSuccess) return e;
        e = hipHostMalloc((void**)&pinned_totals, 8 * sizeof(uint64_t), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        e = ensure(adam_state, 256);
        if (e != hipSuccess) return e;
        device_used = true;
        return hipSuccess;
    }

    int fail(int code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        return fail(e == hipErrorOutOfMemory ? MVGS_ENOMEM : MVGS_EHIP, "%s: %s", what, hipGetErrorString(e));
    }
};

namespace {

struct Need {
    DevBuf* buf;
    size_t bytes;
};

// Grows every listed buffer (each listed once) to its size, unless the context would then hold
// more than its workspace limit: then nothing is allocated and MVGS_ECAPACITY is returned.
int grow_all(mvgs_context* ctx, const Need* need, int count) {
    if (ctx->capturing) {
        for (int i = 0; i < count; ++i)
            if (need[i].bytes && grown_capacity(*need[i].buf, need[i].bytes) != need[i].buf->cap)
                return ctx->fail(MVGS_ECAPACITY, "the call would allocate device memory during stream capture: "
                                                 "make the same call once before capturing");
        return MVGS_OK;
    }
    if (ctx->limit) {
        size_t planned = ctx->held();
        for (int i = 0; i < count; ++i)
            if (need[i].bytes) planned += grown_capacity(*need[i].buf, need[i].bytes) - need[i].buf->cap;
        if (planned > ctx->limit)
            return ctx->fail(MVGS_ECAPACITY, "the call needs the context to hold %zu device bytes; its limit is %zu",
                             planned, ctx->limit);
    }
    for (int i = 0; i < count; ++i) {
        if (!need[i].bytes) continue;
        hipError_t e = ensure(*need[i].buf, need[i].bytes);
        if (e != hipSuccess) return ctx->hip_fail(e, "workspace allocation");
    }
    return MVGS_OK;
}

size_t need_sum(const Need* need, int count) {
    size_t n = 0;
    for (int i = 0; i < count; ++i) n += need[i].bytes;
    return n;
}

}  // namespace

#define HIPCHK(ctx, call)                                     \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, #call); \
    } while (0)

#define LAUNCHCHK(ctx, what)                                  \
    do {                                                      \
        hipError_t e_ = hipGetLastError();                    \
        if (e_ != hipSuccess) return (ctx)->hip_fail(e_, what); \
    } while (0)

namespace {

int validate_cams(mvgs_context* ctx, const mvgs_camera* cams, int32_t B, int tw, int th, uint32_t* n_tiles,
                  uint32_t* n_pixels) {
    if (!cams) return ctx->fail(MVGS_EINVAL, "cams is NULL");
    if (B < 1 || B > MVGS_MAX_VIEWS) return ctx->fail(MVGS_EINVAL, "B=%d outside [1, %d]", B, MVGS_MAX_VIEWS);
    uint64_t tiles = 0, pix = 0;
    for (int v = 0; v < B; ++v) {
        const mvgs_camera& c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
            return ctx->fail(MVGS_EINVAL, "view %d: size %dx%d outside [1, 65535]", v, c.width, c.height);
        if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
            return ctx->fail(MVGS_EINVAL, "view %d: focal lengths must be finite and > 0", v);
        const uint64_t t = (uint64_t)((c.width + tw - 1) / tw) * (uint64_t)((c.height + th - 1) / th);
        if (t > MVGS_MAX_TILES_PER_VIEW)
            return ctx->fail(MVGS_EINVAL, "view %d: %llu tiles exceed %d", v, (unsigned long long)t,
                             MVGS_MAX_TILES_PER_VIEW);
        tiles += t;
        pix += (uint64_t)c.width * c.height;
    }
    if (pix >= (1ull << 32)) return ctx->fail(MVGS_EINVAL, "total pixels %llu reach 2^32", (unsigned long long)pix);
    if (tiles >= (1ull << 32)) return ctx->fail(MVGS_EINVAL, "total tiles reach 2^32");
    *n_tiles = (uint32_t)tiles;
    *n_pixels = (uint32_t)pix;
    return MVGS_OK;
}

int validate_gaussians(mvgs_context* ctx, const mvgs_gaussians* g) {
    if (!g) return ctx->fail(MVGS_EINVAL, "gaussians is NULL");
    if (g->P < 0 || g->P >= (1ll << 31)) return ctx->fail(MVGS_EINVAL, "P=%lld outside [0, 2^31)", (long long)g->P);
    if (g->sh_degree < 0 || g->sh_degree > 3) return ctx->fail(MVGS_EINVAL, "sh_degree=%d outside [0, 3]", g->sh_degree);
    if (g->P > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
        return ctx->fail(MVGS_EINVAL, "a Gaussian parameter pointer is NULL");
    return MVGS_OK;
}

GaussianArgs gargs(const mvgs_gaussians* g) {
    GaussianArgs a;
    a.means = g->means;
    a.scales = g->scales;
    a.quats = g->quats;
    a.opac = g->opacities;
    a.sh = g->sh;
    a.P = g->P;
    a.sh_degree = g->sh_degree;
    return a;
}

void build_cams(const mvgs_camera* cams, int B, int tw, int th, std::vector<DevCam>& out) {
    out.resize(B);
    uint32_t tb = 0, pb = 0;
    for (int v = 0; v < B; ++v) {
        const mvgs_camera& c = cams[v];
        DevCam& d = out[v];
        memcpy(d.R, c.R, sizeof(d.R));
        memcpy(d.t, c.t, sizeof(d.t));
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        memcpy(d.bg, c.bg, sizeof(d.bg));
        for (int i = 0; i < 3; ++i) {
            const double p = -((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]);
            d.campos[i] = (float)p;
        }
        d.W = c.width;
        d.H = c.height;
        d.tiles_x = (c.width + tw - 1) / tw;
        d.tiles_y = (c.height + th - 1) / th;
        d.tile_base = tb;
        d.pix_base = pb;
        tb += (uint32_t)(d.tiles_x * d.tiles_y);
        pb += (uint32_t)(c.width * c.height);
    }
}

// Frame handles. Frame objects are pooled per context and reused, so a raw pointer would let a
// handle kept past mvgs_frame_release name whatever frame the object holds next. A handle is
// therefore the object's address (below 2^48 in user space) with the object's 16-bit generation
// in the top bits; releasing a frame advances its generation, and every call resolves the handle
// through frame_of, which rejects a handle whose generation is not the object's current one (a
// stale handle aliases a new frame only after exactly a multiple of 65,536 reuses of its object).
constexpr uintptr_t kFrameAddrMask = ((uintptr_t)1 << 48) - 1;

mvgs_frame* frame_handle(mvgs_frame* f) {
    return reinterpret_cast<mvgs_frame*>(reinterpret_cast<uintptr_t>(f) | ((uintptr_t)f->gen << 48));
}

mvgs_frame* frame_of(const mvgs_frame* handle) {
    const uintptr_t h = reinterpret_cast<uintptr_t>(handle);
    mvgs_frame* f = reinterpret_cast<mvgs_frame*>(h & kFrameAddrMask);
    if (!f || f->gen != (uint16_t)(h >> 48) || !f->in_use) return nullptr;
    return f;
}

mvgs_frame* acquire_frame(mvgs_context* ctx) {
    for (mvgs_frame* f : ctx->frames)
        if (!f->in_use) {
            f->in_use = true;
            return f;
        }
    mvgs_frame* f = new (std::nothrow) mvgs_frame();
    if (!f) return nullptr;
    if (reinterpret_cast<uintptr_t>(f) & ~kFrameAddrMask) {   // no room for the generation
        delete f;
        return nullptr;
    }
    f->each_buffer([&](DevBuf& b) { b.al = &ctx->alloc; });
    f->ctx = ctx;
    f->in_use = true;
    ctx->frames.push_back(f);
    return f;
}


}  // namespace

extern "C" {

const char* mvgs_status_string(int status) {
    switch (status) {
        case MVGS_OK: return "ok";
        case MVGS_EINVAL: return "invalid argument";
        case MVGS_ENOMEM: return "out of memory";
        case MVGS_ECAPACITY: return "size limit exceeded";
        case MVGS_EHIP: return "HIP runtime error";
        case MVGS_ERETRY: return "make the call again";
        default: return "unknown status";
    }
}

const char* mvgs_last_error(const mvgs_context* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

int mvgs_create(mvgs_context** out, const mvgs_options* opt) {
    if (!out) return MVGS_EINVAL;
    *out = nullptr;
    int tw = 16, th = 16, ppl = 0;
    int64_t limit = 0, cap_v = 0, cap_k = 0;
    if (opt) {
        if (opt->tile_w) tw = opt->tile_w;
        if (opt->tile_h) th = opt->tile_h;
        ppl = opt->pixels_per_lane;
        limit = opt->workspace_limit;
        cap_v = opt->capacity_records;
        cap_k = opt->capacity_pairs;
        if (opt->reserved0) return MVGS_EINVAL;
        if ((opt->alloc == nullptr) != (opt->free == nullptr)) return MVGS_EINVAL;
    }
    if (limit < 0 || cap_v < 0 || cap_k < 0 || (cap_v == 0) != (cap_k == 0) || cap_v >= (1ll << 32) ||
        cap_k >= (1ll << 32))
        return MVGS_EINVAL;
    const bool ppl_auto = ppl == 0;
    if (ppl == 0) ppl = blend_default_ppl(tw, th);
    if (!blend_supported(tw, th, ppl)) return MVGS_EINVAL;
    mvgs_context* ctx = new (std::nothrow) mvgs_context();
    if (!ctx) return MVGS_ENOMEM;
    ctx->tw = tw;
    ctx->th = th;
    ctx->ppl = ppl;
    ctx->ppl_auto = ppl_auto;
    ctx->limit = (size_t)limit;
    ctx->cap_v = (uint64_t)cap_v;
    ctx->cap_k = (uint64_t)cap_k;
    if (opt) {
        ctx->alloc.alloc = opt->alloc;
        ctx->alloc.free = opt->free;
        ctx->alloc.ctx = opt->alloc_ctx;
    }
    ctx->each_buffer([&](DevBuf& b) { b.al = &ctx->alloc; });
    // no HIP call here: device resources are created by the first call that needs them
    *out = ctx;
    return MVGS_OK;
}

void mvgs_destroy(mvgs_context* ctx) {
    if (!ctx) return;
    if (ctx->device_used) (void)hipDeviceSynchronize();
    ctx->ring.destroy();
    ctx->each_buffer([](DevBuf& b) { release(b); });
    for (mvgs_frame* f : ctx->frames) delete f;
    for (auto& m : ctx->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->pinned_totals) (void)hipHostFree(ctx->pinned_totals);
    if (ctx->pinned_counts) (void)hipHostFree(ctx->pinned_counts);
    delete ctx;
}

}  // extern "C"

namespace {

// A lane's pixels share its walk over the tile's list, so more pixels per lane means fewer
// wavefronts: fewer walks over the same lists, but also less latency hiding. Take the most
// pixels per lane the tile allows that still launches kMinBlendWaves wavefronts (16 per CU); a
// frame with fewer tiles than that takes one pixel per lane.
constexpr uint64_t kMinBlendWaves = 4096;
static int blend_auto_ppl(int tw, int th, uint32_t n_tiles) {
    for (int ppl = blend_default_ppl(tw, th); ppl > 1; ppl >>= 1)
        if ((uint64_t)n_tiles * (uint64_t)(tw * th / (64 * ppl)) >= kMinBlendWaves) return ppl;
    return 1;
}

// Capacity-mode frames keep on the device (dtot, 64 bytes): the call's totals (u64 records, pairs,
// error words, selection tasks) at [0, 32), at [32, 44) the clamped record and pair counts and
// the void word (bit 0 capacity overflow, bit 1 rejected selection, bit 2 tasks over their bound,
// bit 3 depth keys outside the sort window), and at [48, 56) the depth keys' (min, ~max).
const uint32_t* frame_eff(const mvgs_frame* f) {
    return f->capacity ? reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(f->dtot.p) + 32) : nullptr;
}
const uint32_t* frame_void(const mvgs_frame* f) { return f->capacity ? frame_eff(f) + 2 : nullptr; }
const uint32_t* frame_tasks(const mvgs_frame* f) {
    return f->capacity ? reinterpret_cast<const uint32_t*>(static_cast<const uint8_t*>(f->dtot.p) + 24) : nullptr;
}

SelBlendArgs sel_args(mvgs_frame* f) {
    SelBlendArgs sa{};
    sa.cams = as<DevCam>(f->cams);
    sa.B = f->B;
    sa.ranges = as<uint2>(f->ranges);
    sa.vals = as<uint32_t>(f->vals[f->final_buf]);
    sa.recs = as<BlendRec>(f->recs);
    sa.sel_off = as<uint32_t>(f->sel_off);
    sa.sel_pix = as<uint32_t>(f->sel_pix);
    sa.tasks = as<uint2>(f->tasks);
    sa.n_tasks = f->n_tasks;
    sa.t_sel = as<float>(f->t_final);
    sa.last_sel = as<uint32_t>(f->n_last);
    sa.depth_sel = as<float>(f->depth);
    if (f->capacity) {
        sa.n_dev = frame_tasks(f);
        sa.void_word = frame_void(f);
    }
    return sa;
}

struct SelIn {
    const uint32_t* off;
    const uint32_t* pix;
    uint32_t n_sel;
    int mode;
};

// What a forward's buffers are sized by.
struct FwdSizes {
    int B = 0;
    size_t P = 0;
    uint32_t n_tiles = 0, n_pixels = 0;
    bool cap = false;
    const SelIn* sel = nullptr;
    size_t task_cap = 0;     // tasks of thread-efficient partial rendering: one per segment + one per 64 pixels
    size_t mask_words = 0;   // pixel bit mask of a selection
    bool want_plane = false; // a selection over views of one size: plane mask of the merged image
    size_t plane_words = 0;
};

FwdSizes fwd_sizes(const mvgs_camera* cams, int B, size_t P, uint32_t n_tiles, uint32_t n_pixels, bool cap,
                   const SelIn* sel) {
    FwdSizes z;
    z.B = B;
    z.P = P;
    z.n_tiles = n_tiles;
    z.n_pixels = n_pixels;
    z.cap = cap;
    z.sel = sel;
    z.task_cap = sel ? (size_t)n_tiles + sel->n_sel / 64 + 1 : 0;
    z.mask_words = ((size_t)n_pixels + 31) / 32;
    bool same_size = true;
    for (int v = 1; v < B; ++v)
        same_size = same_size && cams[v].width == cams[0].width && cams[v].height == cams[0].height;
    z.plane_words = ((size_t)cams[0].width * cams[0].height + 31) / 32;
    z.want_plane = sel && same_size;
    return z;
}

constexpr int kMaxNeed = 24;

// Buffers a forward grows before the participation pre-pass (sized by P, tiles, pixels).
int fwd_needs_pre(mvgs_context* ctx, mvgs_frame* f, const FwdSizes& z, Need* n) {
    const SelIn* sel = z.sel;
    const size_t P = z.P;
    int k = 0;
    n[k++] = {&f->cams, sizeof(DevCam) * z.B};
    n[k++] = {&ctx->nrec, sizeof(uint32_t) * (P + 1)};
    n[k++] = {&ctx->ntiles, sizeof(uint32_t) * (P + 1)};
    n[k++] = {&ctx->totals, sizeof(uint64_t) * 8};
    n[k++] = {&f->dtot, z.cap ? (size_t)64 : (size_t)0};
    n[k++] = {&f->rec_off, sizeof(uint32_t) * (P + 1)};
    n[k++] = {&ctx->scan_scratch, scan_scratch_bytes(std::max<size_t>(P + 1, z.n_tiles))};
    n[k++] = {&f->sel_off, sel ? sizeof(uint32_t) * ((size_t)z.n_tiles + 1) : 0};
    n[k++] = {&f->sel_pix, sel ? sizeof(uint32_t) * std::max<size_t>(sel->n_sel, 1) : 0};
    n[k++] = {&f->mask, sel ? sizeof(uint32_t) * z.mask_words : 0};
    n[k++] = {&f->task_n, sel ? sizeof(uint32_t) * z.n_tiles : 0};
    n[k++] = {&f->task_off, sel ? sizeof(uint32_t) * z.n_tiles : 0};
    n[k++] = {&f->tasks, sel ? sizeof(uint2) * z.task_cap : 0};
    n[k++] = {&f->plane_mask, z.want_plane ? sizeof(uint32_t) * z.plane_words : 0};
    return k;
}

// Buffers a forward grows once it knows V records and K pairs (exact, or the capacities).
int fwd_needs_post(mvgs_context* ctx, mvgs_frame* f, const FwdSizes& z, uint32_t V, uint32_t K, Need* n) {
    const SelIn* sel = z.sel;
    const size_t V1 = std::max<uint32_t>(V, 1), K1 = std::max<uint32_t>(K, 1);
    // per-pixel blend state: every pixel, or every selected pixel in thread-efficient mode
    const bool compact = sel && sel->mode == MVGS_PARTIAL_COMPACT;
    const size_t n_px_state = compact ? sel->n_sel : z.n_pixels;
    int k = 0;
    n[k++] = {&f->recs, sizeof(BlendRec) * V1};
    n[k++] = {&f->rec_view, sizeof(uint16_t) * V1};
    n[k++] = {&ctx->depth_key[0], sizeof(uint32_t) * V1};
    n[k++] = {&ctx->depth_key[1], sizeof(uint32_t) * V1};
    n[k++] = {&ctx->rec_vals[0], sizeof(uint32_t) * V1};
    n[k++] = {&ctx->rec_vals[1], sizeof(uint32_t) * V1};
    n[k++] = {&ctx->tile_rect, sizeof(uint2) * V1};
    n[k++] = {&ctx->sorted_rect, sizeof(uint2) * V1};
    n[k++] = {&f->keys[0], sizeof(uint32_t) * K1};
    n[k++] = {&f->keys[1], sizeof(uint32_t) * K1};
    n[k++] = {&f->vals[0], sizeof(uint32_t) * K1};
    n[k++] = {&f->vals[1], sizeof(uint32_t) * K1};
    n[k++] = {&f->ranges, sizeof(uint2) * std::max<uint32_t>(z.n_tiles, 1)};
    n[k++] = {&f->t_final, sizeof(float) * std::max<size_t>(n_px_state, 1)};
    n[k++] = {&f->n_last, sizeof(uint32_t) * std::max<size_t>(n_px_state, 1)};
    n[k++] = {&f->depth, compact ? sizeof(float) * std::max<size_t>(sel->n_sel, 1) : (size_t)0};
    n[k++] = {&ctx->sort_scratch, std::max(radix_scratch_bytes(V), emit_sort_scratch_bytes(V, K))};
    return k;
}

// Buffers of the loss and of the backward.
uint64_t ssim_tiles_of(const mvgs_camera* cams, int B) {
    uint64_t n = 0;
    for (int v = 0; v < B; ++v) n += ssim_tiles(cams[v].width, cams[v].height);
    return n;
}
int loss_needs(mvgs_context* ctx, const mvgs_camera* cams, int B, uint32_t n_pixels, bool dssim, Need* n) {
    n[0] = {&ctx->loss_scratch, loss_scratch_bytes(n_pixels, dssim ? ssim_tiles_of(cams, B) : 0)};
    return 1;
}
int backward_needs(mvgs_context* ctx, uint32_t V, Need* n) {
    n[0] = {&ctx->acc, sizeof(float) * kAccStride * std::max<uint32_t>(V, 1)};
    return 1;
}

int forward_impl(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams, int32_t B,
                 float* const* images, mvgs_frame** frame, const SelIn* sel) {
    if (!ctx) return MVGS_EINVAL;
    if (!frame) return ctx->fail(MVGS_EINVAL, "frame output is NULL");
    *frame = nullptr;
    int st = validate_gaussians(ctx, g);
    if (st) return st;
    uint32_t n_tiles = 0, n_pixels = 0;
    st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    if (!images) return ctx->fail(MVGS_EINVAL, "images is NULL");
    for (int v = 0; v < B; ++v)
        if (!images[v]) return ctx->fail(MVGS_EINVAL, "images[%d] is NULL", v);

    hipStream_t s = (hipStream_t)stream;
    const int tw = ctx->tw, th = ctx->th;
    const bool cap = ctx->cap_v > 0;
    if (ctx->begin(s) && (!cap || !ctx->device_used))
        return ctx->fail(MVGS_EINVAL, "a forward can be captured only on a context with capacities, after one "
                                      "call outside the capture");
    HIPCHK(ctx, ctx->bind_device());
    mvgs_frame* f = acquire_frame(ctx);
    if (!f) return ctx->fail(MVGS_ENOMEM, "frame allocation failed");
    f->B = B;
    f->P = g->P;
    f->sh_degree = g->sh_degree;
    f->n_tiles = n_tiles;
    f->n_pixels = n_pixels;
    f->mode = sel ? sel->mode : kModeFull;
    f->n_sel = sel ? sel->n_sel : 0;
    f->n_tasks = 0;
    f->partition = false;
    f->capacity = cap;
    f->checked = !cap;
    f->cam_stage = nullptr;
    build_cams(cams, B, tw, th, f->hcams);
    const GaussianArgs ga = gargs(g);
    const size_t P = (size_t)g->P;

    auto bail = [&](int code) {
        f->in_use = false;
        return code;
    };
#define FCHK(call)                                                   \
    do {                                                             \
        hipError_t e_ = (call);                                      \
        if (e_ != hipSuccess) return bail(ctx->hip_fail(e_, #call)); \
    } while (0)

    const bool fresh_totals = !ctx->totals.p;
    const FwdSizes z = fwd_sizes(cams, B, (size_t)g->P, n_tiles, n_pixels, cap, sel);
    const size_t task_cap = z.task_cap, mask_words = z.mask_words, plane_words = z.plane_words;
    const bool want_plane = z.want_plane;
    Need need1[kMaxNeed];
    const int n_need1 = fwd_needs_pre(ctx, f, z, need1);
    st = grow_all(ctx, need1, n_need1);
    if (st) return bail(st);
    if (fresh_totals) fill_u32(as<uint32_t>(ctx->totals), 16, 0u, s);
    void* img_ptrs = nullptr;
    {
        void* dcams = nullptr;
        FCHK(ctx->ring.put(f->hcams.data(), sizeof(DevCam) * B, s, &dcams, ctx->capturing, &f->cam_stage));
        FCHK(hipMemcpyAsync(f->cams.p, dcams, sizeof(DevCam) * B, hipMemcpyDeviceToDevice, s));
        FCHK(ctx->ring.put(images, sizeof(float*) * B, s, &img_ptrs, ctx->capturing));
    }
    const DevCam* dcam = as<DevCam>(f->cams);

    // participation and sizes
    int mk = ctx->stage_begin(0, s);
    fill_u32(as<uint32_t>(ctx->nrec) + P, 1, 0u, s);
    // the range of the records' depth keys (totals[6]: min, ~max), read at the synchronization
    // below so that the depth sort covers only the bits in which keys differ (capacity mode:
    // checked against the context's window on the device)
    uint32_t* key_range = reinterpret_cast<uint32_t*>(as<uint64_t>(ctx->totals) + 6);
    fill_u32(key_range, 2, ~0u, s);
    launch_count(ga, dcam, B, tw, th, as<uint32_t>(ctx->nrec), as<uint32_t>(ctx->ntiles), s, key_range);
    scan_exclusive_u32(as<uint32_t>(ctx->nrec), as<uint32_t>(f->rec_off), P + 1, as<uint64_t>(ctx->totals),
                       ctx->scan_scratch.p, s);
    reduce_sum_u32(as<uint32_t>(ctx->ntiles), P, as<uint64_t>(ctx->totals) + 1, nullptr, s);
    uint32_t* sel_err = reinterpret_cast<uint32_t*>(as<uint64_t>(ctx->totals) + 2) + 1;
    if (sel) {
        // the selection: private copy, checks, pixel mask, wavefront tasks
        if (n_tiles) FCHK(hipMemcpyAsync(f->sel_off.p, sel->off, sizeof(uint32_t) * ((size_t)n_tiles + 1),
                                         hipMemcpyDeviceToDevice, s));
        if (sel->n_sel) FCHK(hipMemcpyAsync(f->sel_pix.p, sel->pix, sizeof(uint32_t) * sel->n_sel,
                                            hipMemcpyDeviceToDevice, s));
        fill_u32(as<uint32_t>(f->mask), mask_words, 0u, s);
        if (want_plane) fill_u32(as<uint32_t>(f->plane_mask), plane_words, 0u, s);
        fill_u32(sel_err, 1, 0u, s);
        fill_u32(reinterpret_cast<uint32_t*>(as<uint64_t>(ctx->totals) + 3), 2, 0u, s);
        if (n_tiles) {
            launch_sel_check(dcam, B, n_tiles, tw, th, as<uint32_t>(f->sel_off), as<uint32_t>(f->sel_pix),
                             sel->n_sel, as<uint32_t>(f->mask), want_plane ? as<uint32_t>(f->plane_mask) : nullptr,
                             as<uint32_t>(f->task_n), sel_err, s);
            scan_exclusive_u32(as<uint32_t>(f->task_n), as<uint32_t>(f->task_off), n_tiles,
                               as<uint64_t>(ctx->totals) + 3, ctx->scan_scratch.p, s);
            launch_sel_tasks(n_tiles, as<uint32_t>(f->task_n), as<uint32_t>(f->task_off), (uint32_t)task_cap,
                             as<uint2>(f->tasks), s);
        }
    }
    ctx->stage_end(mk, s);
    FCHK(hipGetLastError());
    uint64_t V64 = ctx->cap_v, K64 = ctx->cap_k;
    uint32_t depth_base = 0;   // the depth sort orders key - depth_base on depth_bits bits
    int depth_bits = 32;
    const uint32_t* eff = nullptr;   // capacity mode: device (records, pairs) of this call
    const uint32_t* ovf = nullptr;   // capacity mode: device overflow word
    if (cap) {
        uint32_t* e32 = reinterpret_cast<uint32_t*>(static_cast<uint8_t*>(f->dtot.p) + 32);
        depth_base = ctx->dwin_base;
        depth_bits = ctx->dwin_bits;
        launch_capacity_clamp(as<uint64_t>(ctx->totals), ctx->cap_v, ctx->cap_k, e32, e32 + 2, s, key_range,
                              depth_base, depth_bits, e32 + 4);
        if (sel) {
            // the grid of the selection kernels is the task bound; the count stays on the device
            launch_sel_void(sel_err, as<uint64_t>(ctx->totals) + 3, (uint32_t)task_cap, e32, e32 + 2, s);
            f->n_tasks = (uint32_t)task_cap;
            // a selection of W H pixels is taken as a partition of the plane; mvgs_frame_check
            // reports it if a plane position is selected in two views
            f->partition = want_plane && (uint64_t)sel->n_sel == (uint64_t)cams[0].width * (uint64_t)cams[0].height;
        }
        // this call's totals and error words, for the selection kernels and mvgs_frame_check
        FCHK(hipMemcpyAsync(f->dtot.p, ctx->totals.p, 4 * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        eff = e32;
        ovf = e32 + 2;
        f->V = 0;
        f->K = 0;
    } else {
        FCHK(hipMemcpyAsync(ctx->pinned_totals, ctx->totals.p, 7 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        FCHK(hipStreamSynchronize(s));
        V64 = ctx->pinned_totals[0];
        K64 = ctx->pinned_totals[1];
        const uint32_t kmin = (uint32_t)ctx->pinned_totals[6], kmax = ~(uint32_t)(ctx->pinned_totals[6] >> 32);
        if (V64 > 0 && kmin <= kmax) {
            depth_base = kmin;
            depth_bits = kmax > kmin ? 32 - __builtin_clz(kmax - kmin) : 1;
        }
        if (sel) {
            const uint32_t e = (uint32_t)(ctx->pinned_totals[2] >> 32);
            f->partition = want_plane && !(e & kSelPlaneOverlap) &&
                           (uint64_t)sel->n_sel == (uint64_t)cams[0].width * (uint64_t)cams[0].height;
            if (e & kSelErrors) {
                (void)ctx->ring.seal(s);
                return bail(ctx->fail(MVGS_EINVAL, "pixel selection rejected:%s%s%s%s",
                                      (e & kSelBadOffsets) ? " offsets do not rise from 0 to n_sel;" : "",
                                      (e & kSelTooLong) ? " a segment holds more pixels than a tile;" : "",
                                      (e & kSelOutside) ? " a pixel lies outside its (view, tile);" : "",
                                      (e & kSelDuplicate) ? " a pixel is selected twice;" : ""));
            }
            const uint64_t nt = ctx->pinned_totals[3];
            if (nt > task_cap) {
                (void)ctx->ring.seal(s);
                return bail(ctx->fail(MVGS_EHIP, "selection tasks %llu exceed their bound", (unsigned long long)nt));
            }
            f->n_tasks = (uint32_t)nt;
        }
        if (V64 >= (1ull << 32) || K64 >= (1ull << 32)) {
            (void)ctx->ring.seal(s);
            return bail(ctx->fail(MVGS_ECAPACITY, "records %llu or pairs %llu reach 2^32", (unsigned long long)V64,
                                  (unsigned long long)K64));
        }
        f->V = (uint32_t)V64;
        f->K = (uint32_t)K64;
    }
    // exact sizes, or in capacity mode the capacities (grids are then sized by them and the
    // kernels read the actual counts from eff)
    const uint32_t V = (uint32_t)V64, K = (uint32_t)K64;

    // records, sorts, ranges and per-pixel state
    Need need2[kMaxNeed];
    const int n_need2 = fwd_needs_post(ctx, f, z, V, K, need2);
    st = grow_all(ctx, need2, n_need2);
    if (st) {
        (void)ctx->ring.seal(s);
        return bail(st);
    }
    f->need_bytes = need_sum(need1, n_need1) + need_sum(need2, n_need2);

    mk = ctx->stage_begin(1, s);
    launch_records(ga, dcam, B, tw, th, as<uint32_t>(f->rec_off), as<BlendRec>(f->recs),
                   as<uint32_t>(ctx->depth_key[0]), as<uint2>(ctx->tile_rect), as<uint16_t>(f->rec_view), s, ovf);
    ctx->stage_end(mk, s);
    mk = ctx->stage_begin(2, s);
    uint32_t* dk[2] = {as<uint32_t>(ctx->depth_key[0]), as<uint32_t>(ctx->depth_key[1])};
    uint32_t* dv[2] = {as<uint32_t>(ctx->rec_vals[0]), as<uint32_t>(ctx->rec_vals[1])};
    // the records' tile rectangles travel with their depth keys
    uint2* rect[2] = {as<uint2>(ctx->tile_rect), as<uint2>(ctx->sorted_rect)};
    // (only the order is used: the last pass writes no keys)
    const int dcur =
        radix_sort_u32(dk, dv, true, V, depth_bits, ctx->sort_scratch.p, s, eff, depth_base, rect, false);
    const uint32_t* sorted_rec = dv[dcur];
    ctx->stage_end(mk, s);

    // pairs in depth order, emitted into their places after the first pass of the stable sort by
    // global tile id, then the other passes
    mk = ctx->stage_begin(3, s);
    const int tile_bits = bits_for(n_tiles);
    f->depth_bits = depth_bits;
    f->tile_bits = tile_bits;
    f->key16 = tile_bits <= 16;
    emit_pairs_first_pass(sorted_rec, rect[dcur], dcam, B, V, eff, f->keys[0].p, f->key16, as<uint32_t>(f->vals[0]),
                          K, eff ? eff + 1 : nullptr, tile_bits, ctx->sort_scratch.p, s);
    ctx->stage_end(mk, s);
    mk = ctx->stage_begin(4, s);
    void* pk[2] = {f->keys[0].p, f->keys[1].p};
    uint32_t* pv[2] = {as<uint32_t>(f->vals[0]), as<uint32_t>(f->vals[1])};
    f->final_buf = sort_pairs_rest(pk, f->key16, pv, K, eff ? eff + 1 : nullptr, tile_bits, ctx->sort_scratch.p, s);
    ctx->stage_end(mk, s);
    mk = ctx->stage_begin(5, s);
    launch_ranges(pk[f->final_buf], f->key16, K, n_tiles, as<uint2>(f->ranges), s, eff ? eff + 1 : nullptr);
    ctx->stage_end(mk, s);

    // blend every pixel of every view
    BlendFwdArgs a;
    a.cams = dcam;
    a.B = B;
    a.n_tiles = n_tiles;
    a.ranges = as<uint2>(f->ranges);
    a.vals = pv[f->final_buf];
    a.recs = as<BlendRec>(f->recs);
    a.images = (float* const*)img_ptrs;
    a.t_final = as<float>(f->t_final);
    a.n_last = as<uint32_t>(f->n_last);
    a.mask = f->mode == MVGS_PARTIAL_MASKED ? as<uint32_t>(f->mask) : nullptr;
    mk = ctx->stage_begin(6, s);
    if (f->mode == MVGS_PARTIAL_COMPACT) {
        SelBlendArgs sa = sel_args(f);
        sa.images = a.images;
        launch_blend_fwd_sel(sa, s);
    } else {
        f->ppl = ctx->ppl_auto ? blend_auto_ppl(tw, th, n_tiles) : ctx->ppl;
        launch_blend_fwd(a, tw, th, f->ppl, s);
    }
    ctx->stage_end(mk, s);
    FCHK(hipGetLastError());
    FCHK(ctx->ring.seal(s));
    *frame = frame_handle(f);
    return MVGS_OK;
#undef FCHK
}

}  // namespace

extern "C" {

int mvgs_forward(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams, int32_t B,
                 float* const* images, mvgs_frame** frame) {
    return forward_impl(ctx, stream, g, cams, B, images, frame, nullptr);
}

int mvgs_forward_partial(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams,
                         int32_t B, const uint32_t* sel_offsets, const uint32_t* sel_pixels, int64_t n_sel,
                         int32_t mode, float* const* images, mvgs_frame** frame) {
    if (!ctx) return MVGS_EINVAL;
    if (mode != MVGS_PARTIAL_COMPACT && mode != MVGS_PARTIAL_MASKED)
        return ctx->fail(MVGS_EINVAL, "mode %d is not MVGS_PARTIAL_COMPACT or MVGS_PARTIAL_MASKED", mode);
    if (n_sel < 0 || n_sel >= (1ll << 32)) return ctx->fail(MVGS_EINVAL, "n_sel=%lld outside [0, 2^32)", (long long)n_sel);
    if (!sel_offsets || (n_sel > 0 && !sel_pixels)) return ctx->fail(MVGS_EINVAL, "selection array is NULL");
    const SelIn sel{sel_offsets, sel_pixels, (uint32_t)n_sel, mode};
    return forward_impl(ctx, stream, g, cams, B, images, frame, &sel);
}

int mvgs_count_views(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_camera* cams, int32_t B,
                     int64_t* records, int64_t* pairs) {
    if (!ctx) return MVGS_EINVAL;
    int st = validate_gaussians(ctx, g);
    if (st) return st;
    uint32_t n_tiles = 0, n_pixels = 0;
    st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    if (!records || !pairs) return ctx->fail(MVGS_EINVAL, "records or pairs is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (ctx->begin(s)) return ctx->fail(MVGS_EINVAL, "mvgs_count_views synchronizes and cannot be captured");
    HIPCHK(ctx, ctx->bind_device());
    // the counts, then the per-workgroup partials of the pre-pass
    const size_t counts_b = (sizeof(unsigned long long) * 2 * (size_t)B + 255) & ~(size_t)255;
    const Need need[] = {{&ctx->view_counts, counts_b + count_views_scratch_bytes(g->P, B)}};
    st = grow_all(ctx, need, 1);
    if (st) return st;
    std::vector<DevCam> hc;
    build_cams(cams, B, ctx->tw, ctx->th, hc);
    void* dcams = nullptr;
    HIPCHK(ctx, ctx->ring.put(hc.data(), sizeof(DevCam) * B, s, &dcams));
    unsigned long long* dc = as<unsigned long long>(ctx->view_counts);
    launch_count_views(gargs(g), (const DevCam*)dcams, B, ctx->tw, ctx->th, dc,
                       reinterpret_cast<unsigned long long*>(static_cast<uint8_t*>(ctx->view_counts.p) + counts_b), s);
    LAUNCHCHK(ctx, "participation pre-pass");
    // read back through pinned memory (a pageable destination costs a staged copy)
    if (ctx->pinned_counts_n < 2 * (size_t)B) {
        if (ctx->pinned_counts) HIPCHK(ctx, hipHostFree(ctx->pinned_counts));
        ctx->pinned_counts = nullptr;
        ctx->pinned_counts_n = 0;
        const size_t n = std::max<size_t>(2 * (size_t)B, 64);
        HIPCHK(ctx, hipHostMalloc((void**)&ctx->pinned_counts, n * sizeof(uint64_t), hipHostMallocDefault));
        ctx->pinned_counts_n = n;
    }
    const uint64_t* hv = ctx->pinned_counts;
    HIPCHK(ctx, hipMemcpyAsync(ctx->pinned_counts, dc, sizeof(unsigned long long) * 2 * (size_t)B,
                               hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, ctx->ring.seal(s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (int v = 0; v < B; ++v) {
        records[v] = (int64_t)hv[2 * (size_t)v];
        pairs[v] = (int64_t)hv[2 * (size_t)v + 1];
    }
    return MVGS_OK;
}

int mvgs_workspace_bound(mvgs_context* ctx, const mvgs_camera* cams, int32_t B, int64_t P, int64_t records,
                         int64_t pairs, int32_t work, int64_t* bytes) {
    if (!ctx) return MVGS_EINVAL;
    if (!bytes) return ctx->fail(MVGS_EINVAL, "bytes is NULL");
    uint32_t n_tiles = 0, n_pixels = 0;
    int st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    if (P < 0 || P >= (1ll << 31)) return ctx->fail(MVGS_EINVAL, "P=%lld outside [0, 2^31)", (long long)P);
    if (records < 0 || records > P * (int64_t)B || pairs < 0)
        return ctx->fail(MVGS_EINVAL, "records %lld or pairs %lld impossible for %lld Gaussians and %d views",
                         (long long)records, (long long)pairs, (long long)P, B);
    if (work & ~(MVGS_WORK_LOSS | MVGS_WORK_LOSS_DSSIM | MVGS_WORK_BACKWARD))
        return ctx->fail(MVGS_EINVAL, "unknown work flags 0x%x", work);
    const bool cap = ctx->cap_v > 0;
    if (!cap && (records >= (1ll << 32) || pairs >= (1ll << 32)))
        return ctx->fail(MVGS_ECAPACITY, "records %lld or pairs %lld reach 2^32", (long long)records, (long long)pairs);
    const uint32_t V = cap ? (uint32_t)ctx->cap_v : (uint32_t)records;
    const uint32_t K = cap ? (uint32_t)ctx->cap_k : (uint32_t)pairs;
    // the frame the forward would take: the first free one of the pool, else a new (empty) one
    mvgs_frame fresh;
    mvgs_frame* f = &fresh;
    for (mvgs_frame* q : ctx->frames)
        if (!q->in_use) {
            f = q;
            break;
        }
    // replay the calls' growth in order on simulated capacities
    std::vector<std::pair<const DevBuf*, size_t>> caps;
    size_t held = ctx->held();
    auto grow = [&](const DevBuf* b, size_t want) {
        if (!want) return;
        size_t c = b->p ? b->cap : 0;
        auto it = std::find_if(caps.begin(), caps.end(), [&](const std::pair<const DevBuf*, size_t>& e) {
            return e.first == b;
        });
        if (it != caps.end()) c = it->second;
        const size_t n = grown_capacity(c, want);
        if (n == c) return;
        held += n - c;
        if (it != caps.end()) it->second = n;
        else caps.emplace_back(b, n);
    };
    auto grow_list = [&](const Need* n, int k) {
        for (int i = 0; i < k; ++i) grow(n[i].buf, n[i].bytes);
    };
    int ring_next = ctx->ring.next;
    auto ring_put = [&](size_t b) { grow(&ctx->ring.slots[ring_next].dev, b); ring_next = (ring_next + 1) % UploadRing::kSlots; };
    if (!ctx->device_used) grow(&ctx->adam_state, 256);
    const FwdSizes z = fwd_sizes(cams, B, (size_t)P, n_tiles, n_pixels, cap, nullptr);
    Need n[kMaxNeed];
    grow_list(n, fwd_needs_pre(ctx, f, z, n));
    ring_put(sizeof(DevCam) * B);
    ring_put(sizeof(float*) * B);
    grow_list(n, fwd_needs_post(ctx, f, z, V, K, n));
    if (work & (MVGS_WORK_LOSS | MVGS_WORK_LOSS_DSSIM)) {
        grow_list(n, loss_needs(ctx, cams, B, n_pixels, (work & MVGS_WORK_LOSS_DSSIM) != 0, n));
        ring_put(sizeof(LossView) * B);
    }
    if (work & MVGS_WORK_BACKWARD) {
        grow_list(n, backward_needs(ctx, V, n));
        ring_put(sizeof(float*) * B);
    }
    *bytes = (int64_t)held;
    return MVGS_OK;
}

int mvgs_subsample(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B, const uint32_t* keys,
                   uint32_t* sel_offsets, uint32_t* sel_pixels) {
    if (!ctx) return MVGS_EINVAL;
    uint32_t n_tiles = 0, n_pixels = 0;
    int st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    for (int v = 1; v < B; ++v)
        if (cams[v].width != cams[0].width || cams[v].height != cams[0].height)
            return ctx->fail(MVGS_EINVAL, "view %d is %dx%d, view 0 is %dx%d: sub-sampling needs one size", v,
                             cams[v].width, cams[v].height, cams[0].width, cams[0].height);
    if (!keys || !sel_offsets || !sel_pixels) return ctx->fail(MVGS_EINVAL, "a sub-sampling buffer is NULL");
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    HIPCHK(ctx, ctx->bind_device());
    const Need need[] = {{&ctx->scan_scratch, scan_scratch_bytes(n_tiles)}};
    st = grow_all(ctx, need, 1);
    if (st) return st;
    launch_subsample(keys, cams[0].width, cams[0].height, B, ctx->tw, ctx->th, sel_offsets, sel_pixels,
                     ctx->scan_scratch.p, s);
    LAUNCHCHK(ctx, "sub-sampling kernels");
    return MVGS_OK;
}

int mvgs_loss(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B, const float* const* images,
              const float* const* targets, float w_l1, float w_dssim, float* loss_dev, float* const* dl_dimages) {
    if (!ctx) return MVGS_EINVAL;
    uint32_t n_tiles = 0, n_pixels = 0;
    int st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    if (!images || !targets || !dl_dimages || !loss_dev) return ctx->fail(MVGS_EINVAL, "a loss buffer is NULL");
    if (!std::isfinite(w_l1) || !std::isfinite(w_dssim)) return ctx->fail(MVGS_EINVAL, "loss weights must be finite");
    std::vector<LossView> lv(B);
    uint32_t pb = 0;
    for (int v = 0; v < B; ++v) {
        if (!images[v] || !targets[v] || !dl_dimages[v]) return ctx->fail(MVGS_EINVAL, "view %d: NULL image", v);
        lv[v].img = images[v];
        lv[v].tgt = targets[v];
        lv[v].grad = dl_dimages[v];
        lv[v].W = cams[v].width;
        lv[v].H = cams[v].height;
        lv[v].pix_base = pb;
        lv[v].pad = 0;
        const uint32_t hw = (uint32_t)(cams[v].width * cams[v].height);
        pb += hw;
    }
    hipStream_t s = (hipStream_t)stream;
    if (ctx->begin(s) && !ctx->device_used)
        return ctx->fail(MVGS_EINVAL, "make the call once before capturing it");
    HIPCHK(ctx, ctx->bind_device());
    Need need[2];
    st = grow_all(ctx, need, loss_needs(ctx, cams, B, n_pixels, w_dssim != 0.0f, need));
    if (st) return st;
    void* dviews = nullptr;
    HIPCHK(ctx, ctx->ring.put(lv.data(), sizeof(LossView) * B, s, &dviews, ctx->capturing));
    const int mk = ctx->stage_begin(7, s);
    launch_loss((const LossView*)dviews, lv.data(), B, n_pixels, w_l1, w_dssim, loss_dev, ctx->loss_scratch.p, s);
    ctx->stage_end(mk, s);
    LAUNCHCHK(ctx, "loss kernels");
    HIPCHK(ctx, ctx->ring.seal(s));
    return MVGS_OK;
}

// Device memory of mvgs_loss_noalloc: a fixed array in the library's code object, one copy on each
// GPU, held until the process ends. Host code never passes `scratch` itself (on the host the name
// stands for a host-side shadow, not the device array): each device's address is looked up once
// with hipGetSymbolAddress and that address is used everywhere.
static __device__ __align__(256) unsigned char scratch[MVGS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};

// the current device's copy of `scratch` (looked up at the first call on that device)
hipError_t scratch_for_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}
}  // namespace

int mvgs_loss_noalloc(mvgs_context* ctx, void* stream, const mvgs_camera* cams, int32_t B, const float* const* images,
                      const float* const* targets, float w_l1, float w_dssim, float* loss_dev,
                      float* const* dl_dimages) {
    if (!ctx) return MVGS_EINVAL;
    uint32_t n_tiles = 0, n_pixels = 0;
    int st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    if (!images || !targets || !dl_dimages || !loss_dev) return ctx->fail(MVGS_EINVAL, "a loss buffer is NULL");
    if (!std::isfinite(w_l1) || !std::isfinite(w_dssim)) return ctx->fail(MVGS_EINVAL, "loss weights must be finite");
    if (B > kLossArgViews)
        return ctx->fail(MVGS_ECAPACITY, "mvgs_loss_noalloc takes at most %d views (B=%d)", kLossArgViews, B);
    std::vector<LossView> lv(B);
    uint32_t pb = 0;
    for (int v = 0; v < B; ++v) {
        if (!images[v] || !targets[v] || !dl_dimages[v]) return ctx->fail(MVGS_EINVAL, "view %d: NULL image", v);
        lv[v].img = images[v];
        lv[v].tgt = targets[v];
        lv[v].grad = dl_dimages[v];
        lv[v].W = cams[v].width;
        lv[v].H = cams[v].height;
        lv[v].pix_base = pb;
        lv[v].pad = 0;
        const uint32_t hw = (uint32_t)(cams[v].width * cams[v].height);
        pb += hw;
    }
    // scratch layout: view table, then the loss partials
    const auto up256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t views_b = up256(sizeof(LossView) * (size_t)B);
    const size_t need = views_b + loss_scratch_bytes(n_pixels, w_dssim != 0.0f ? ssim_tiles_of(cams, B) : 0);
    if (need > (size_t)MVGS_NOALLOC_SCRATCH_BYTES)
        return ctx->fail(MVGS_ECAPACITY,
                         "mvgs_loss_noalloc: %zu scratch bytes needed (%u pixels%s), above its %d-byte maximum", need,
                         n_pixels, w_dssim != 0.0f ? ", D-SSIM" : "", MVGS_NOALLOC_SCRATCH_BYTES);
    void* base = nullptr;
    HIPCHK(ctx, scratch_for_current_device(&base));
    hipStream_t s = (hipStream_t)stream;
    uint8_t* p = (uint8_t*)base;
    LossView* dviews = (LossView*)p;
    // every partial and chunk sum is written before it is read: nothing to clear
    launch_put_loss_views(lv.data(), B, dviews, s);
    launch_loss(dviews, lv.data(), B, n_pixels, w_l1, w_dssim, loss_dev, p + views_b, s);
    LAUNCHCHK(ctx, "loss kernels");
    return MVGS_OK;
}

int mvgs_adapt_density(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const float* e1, const float* e2,
                       const int32_t* count, const float* normals, const mvgs_adc_params* prm,
                       const mvgs_gaussians_out* out, int32_t* src, int64_t capacity, int64_t* n_out) {
    if (!ctx) return MVGS_EINVAL;
    int st = validate_gaussians(ctx, g);
    if (st) return st;
    if (!prm || !out || !n_out) return ctx->fail(MVGS_EINVAL, "params, outputs or n_out is NULL");
    if (g->P > 0 && (!e1 || !e2 || !count || !normals))
        return ctx->fail(MVGS_EINVAL, "statistics or normals are NULL");
    if (capacity < 0) return ctx->fail(MVGS_EINVAL, "capacity < 0");
    if (!(prm->dense_scale >= 0.0f) || !std::isfinite(prm->split_threshold) || !std::isfinite(prm->clone_threshold) ||
        !std::isfinite(prm->min_opacity))
        return ctx->fail(MVGS_EINVAL, "densification parameters must be finite (dense_scale >= 0)");
    *n_out = 0;
    hipStream_t s = (hipStream_t)stream;
    if (ctx->begin(s)) return ctx->fail(MVGS_EINVAL, "mvgs_adapt_density synchronizes and cannot be captured");
    HIPCHK(ctx, ctx->bind_device());
    const size_t P = (size_t)g->P;
    const Need need[] = {{&ctx->adc_n, sizeof(uint32_t) * (P + 1)},
                         {&ctx->adc_off, sizeof(uint32_t) * (P + 1)},
                         {&ctx->adc_act, std::max<size_t>(P, 1)},
                         {&ctx->totals, sizeof(uint64_t) * 8},
                         {&ctx->scan_scratch, scan_scratch_bytes(P + 1)}};
    const bool fresh_totals = !ctx->totals.p;
    st = grow_all(ctx, need, 5);
    if (st) return st;
    if (fresh_totals) fill_u32(as<uint32_t>(ctx->totals), 16, 0u, s);
    AdcParams ap{prm->split_threshold, prm->clone_threshold, prm->dense_scale, prm->min_opacity};
    const GaussianArgs ga = gargs(g);
    uint64_t* total = as<uint64_t>(ctx->totals) + 4;
    if (P) {
        launch_adc_classify(ga, e1, e2, count, ap, as<uint32_t>(ctx->adc_n), as<uint8_t>(ctx->adc_act), s);
        scan_exclusive_u32(as<uint32_t>(ctx->adc_n), as<uint32_t>(ctx->adc_off), P, total, ctx->scan_scratch.p, s);
    } else {
        fill_u32(reinterpret_cast<uint32_t*>(total), 2, 0u, s);
    }
    LAUNCHCHK(ctx, "densification classify");
    HIPCHK(ctx, hipMemcpyAsync(ctx->pinned_totals, total, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const int64_t n = (int64_t)ctx->pinned_totals[0];
    *n_out = n;
    if (n > capacity)
        return ctx->fail(MVGS_ECAPACITY, "densification makes %lld Gaussians; the outputs hold %lld", (long long)n,
                         (long long)capacity);
    if (n > 0 && (!out->means || !out->scales || !out->quats || !out->opacities || !out->sh))
        return ctx->fail(MVGS_EINVAL, "an output pointer is NULL");
    launch_adc_write(ga, normals, as<uint8_t>(ctx->adc_act), as<uint32_t>(ctx->adc_off), out->means, out->scales,
                     out->quats, out->opacities, out->sh, src, s);
    LAUNCHCHK(ctx, "densification write");
    return MVGS_OK;
}

static int grads_present(const mvgs_grads* gr, int64_t P) {
    return gr && (P == 0 || (gr->means && gr->scales && gr->quats && gr->opacities && gr->sh));
}

int mvgs_adam_step(mvgs_context* ctx, void* stream, int64_t P, int32_t sh_degree, const mvgs_gaussians_out* params,
                   const mvgs_grads* grads, float* moments, const mvgs_adam_params* prm) {
    if (!ctx) return MVGS_EINVAL;
    if (P < 0 || P >= (1ll << 31)) return ctx->fail(MVGS_EINVAL, "P=%lld outside [0, 2^31)", (long long)P);
    if (sh_degree < 0 || sh_degree > 3) return ctx->fail(MVGS_EINVAL, "sh_degree=%d outside [0, 3]", sh_degree);
    if (!params || !prm || !grads_present(grads, P))
        return ctx->fail(MVGS_EINVAL, "params, grads or adam parameters are NULL");
    if (P > 0 && (!params->means || !params->scales || !params->quats || !params->opacities || !params->sh ||
                  !moments))
        return ctx->fail(MVGS_EINVAL, "a parameter or moment pointer is NULL");
    if (!prm->step_dev && prm->step < 1) return ctx->fail(MVGS_EINVAL, "step=%d must be >= 1", prm->step);
    if (prm->skip_dev && !prm->step_dev) return ctx->fail(MVGS_EINVAL, "skip_dev needs step_dev");
    if (!(prm->beta1 >= 0.0f && prm->beta1 < 1.0f && prm->beta2 >= 0.0f && prm->beta2 < 1.0f && prm->eps >= 0.0f))
        return ctx->fail(MVGS_EINVAL, "betas must lie in [0, 1) and eps >= 0");
    const float lrs[6] = {prm->lr_means, prm->lr_scales, prm->lr_quats, prm->lr_opacities, prm->lr_sh_dc,
                          prm->lr_sh_rest};
    for (float l : lrs)
        if (!std::isfinite(l)) return ctx->fail(MVGS_EINVAL, "learning rates must be finite");
    const int32_t t = prm->step_dev ? 1 : prm->step;   // (counted on the device: checked for t = 1)
    AdamArgs a{lrs[0], lrs[1], lrs[2], lrs[3], lrs[4], lrs[5], prm->beta1, prm->beta2, prm->eps,
               (float)(1.0 - std::pow((double)prm->beta1, t)), (float)(1.0 - std::pow((double)prm->beta2, t))};
    if (!(a.bc1 > 0.0f) || !(a.bc2 > 0.0f)) return ctx->fail(MVGS_EINVAL, "a bias correction is zero");
    GradArgs gr{};
    gr.means = grads->means;
    gr.scales = grads->scales;
    gr.quats = grads->quats;
    gr.opac = grads->opacities;
    gr.sh = grads->sh;
    HIPCHK(ctx, ctx->bind_device());
    float* state = nullptr;
    if (prm->step_dev) {
        state = as<float>(ctx->adam_state);
        launch_adam_count(prm->step_dev, prm->skip_dev, prm->beta1, prm->beta2, state, (hipStream_t)stream);
    }
    launch_adam(params->means, params->scales, params->quats, params->opacities, params->sh, gr, moments, P, sh_degree,
                a, (hipStream_t)stream, state);
    LAUNCHCHK(ctx, "adam step");
    return MVGS_OK;
}

int mvgs_gather_rows(mvgs_context* ctx, void* stream, const int32_t* src, int64_t n, int64_t width, const float* in,
                     float* out) {
    if (!ctx) return MVGS_EINVAL;
    if (n < 0 || width < 0 || (width > 0 && n > (int64_t(1) << 40) / width))
        return ctx->fail(MVGS_EINVAL, "n=%lld, width=%lld out of range", (long long)n, (long long)width);
    if (n > 0 && width > 0 && (!src || !in || !out)) return ctx->fail(MVGS_EINVAL, "src, in or out is NULL");
    HIPCHK(ctx, ctx->bind_device());
    launch_gather_rows(src, n, width, in, out, (hipStream_t)stream);
    LAUNCHCHK(ctx, "row gather");
    return MVGS_OK;
}

}  // extern "C"

namespace {

int check_moment_args(mvgs_context* ctx, int64_t P, int32_t sh_degree, const mvgs_grads* grads, const double* sum,
                      const double* acc) {
    if (P < 0 || P >= (1ll << 31)) return ctx->fail(MVGS_EINVAL, "P=%lld outside [0, 2^31)", (long long)P);
    if (sh_degree < 0 || sh_degree > 3) return ctx->fail(MVGS_EINVAL, "sh_degree=%d outside [0, 3]", sh_degree);
    if (!grads_present(grads, P) || !acc || (P > 0 && !sum))
        return ctx->fail(MVGS_EINVAL, "grads, sum or acc is NULL");
    return MVGS_OK;
}

// the five gradient tensors as one vector: means | scales | quats | opacities | SH
GradSegments moment_segments(int64_t P, int32_t sh_degree, const mvgs_grads* grads) {
    const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
    GradSegments gs;
    const float* seg[5] = {grads->means, grads->scales, grads->quats, grads->opacities, grads->sh};
    const int64_t width[5] = {3, 3, 4, 1, 3 * K};
    int64_t at = 0;
    for (int k = 0; k < 5; ++k) {
        gs.x[k] = seg[k];
        at += P * width[k];
        gs.end[k] = at;
    }
    return gs;
}

}  // namespace

extern "C" {

int mvgs_grad_moments(mvgs_context* ctx, void* stream, int64_t P, int32_t sh_degree, const mvgs_grads* grads,
                      double* sum, double* acc) {
    if (!ctx) return MVGS_EINVAL;
    int st = check_moment_args(ctx, P, sh_degree, grads, sum, acc);
    if (st) return st;
    HIPCHK(ctx, ctx->bind_device());
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    const Need need[] = {{&ctx->moment_partials, sizeof(double) * 2 * kMomentBlocks}};
    st = grow_all(ctx, need, 1);
    if (st) return st;
    launch_grad_moments(moment_segments(P, sh_degree, grads), sum, acc, as<double>(ctx->moment_partials), s);
    LAUNCHCHK(ctx, "gradient moments");
    return MVGS_OK;
}

int mvgs_loss_3d(mvgs_context* ctx, void* stream, const mvgs_frame* frame, const float* image, const float* target,
                 float w_l1, float w_dssim, float* loss_dev, float* dl_dimage) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx) return MVGS_EINVAL;
    if (!frame || frame->ctx != ctx || !frame->in_use) return ctx->fail(MVGS_EINVAL, "frame is not live on this context");
    if (frame->mode != MVGS_PARTIAL_COMPACT || !frame->partition)
        return ctx->fail(MVGS_EINVAL, "the 3D loss needs a thread-efficient partial frame whose selection covers the "
                                      "views' image plane once (as mvgs_subsample makes)");
    if (!image || !target || !loss_dev || !dl_dimage) return ctx->fail(MVGS_EINVAL, "a loss buffer is NULL");
    if (!std::isfinite(w_l1) || !std::isfinite(w_dssim)) return ctx->fail(MVGS_EINVAL, "loss weights must be finite");
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    const int W = f->hcams[0].W, H = f->hcams[0].H;
    const Need need[] = {{&ctx->loss3d_scratch, loss3d_scratch_bytes(W, H)}};
    int st = grow_all(ctx, need, 1);
    if (st) return st;
    const int mk = ctx->stage_begin(7, s);
    launch_loss3d(as<DevCam>(f->cams), f->B, f->n_tiles, as<uint32_t>(f->sel_off), as<uint32_t>(f->sel_pix),
                  as<float>(f->t_final), as<float>(f->depth), W, H, image, target, w_l1, w_dssim, loss_dev, dl_dimage,
                  ctx->loss3d_scratch.p, s, frame_void(f));
    ctx->stage_end(mk, s);
    LAUNCHCHK(ctx, "3D loss kernels");
    return MVGS_OK;
}

int mvgs_export_depth(mvgs_context* ctx, void* stream, const mvgs_frame* frame, float* const* depth) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use || !depth) return MVGS_EINVAL;
    if (frame->mode != MVGS_PARTIAL_COMPACT)
        return ctx->fail(MVGS_EINVAL, "depth is rendered by thread-efficient partial frames only");
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    for (int v = 0; v < f->B; ++v)
        if (!depth[v]) return ctx->fail(MVGS_EINVAL, "depth[%d] is NULL", v);
    void* dptrs = nullptr;
    HIPCHK(ctx, ctx->ring.put(depth, sizeof(float*) * f->B, s, &dptrs, ctx->capturing));
    launch_sel_scatter(as<DevCam>(f->cams), f->B, f->n_tiles, as<uint32_t>(f->sel_off), as<uint32_t>(f->sel_pix),
                       as<float>(f->depth), (float* const*)dptrs, s, frame_void(f));
    LAUNCHCHK(ctx, "depth scatter");
    HIPCHK(ctx, ctx->ring.seal(s));
    return MVGS_OK;
}

int mvgs_backward(mvgs_context* ctx, void* stream, const mvgs_gaussians* g, const mvgs_frame* frame,
                  const float* const* dl_dimages, mvgs_grads* grads, mvgs_densify* densify) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx) return MVGS_EINVAL;
    int st = validate_gaussians(ctx, g);
    if (st) return st;
    if (!frame || frame->ctx != ctx || !frame->in_use) return ctx->fail(MVGS_EINVAL, "frame is not live on this context");
    if (frame->P != g->P || frame->sh_degree != g->sh_degree)
        return ctx->fail(MVGS_EINVAL, "gaussians do not match the frame (P or sh_degree)");
    if (!dl_dimages || !grads) return ctx->fail(MVGS_EINVAL, "dl_dimages or grads is NULL");
    for (int v = 0; v < frame->B; ++v)
        if (!dl_dimages[v]) return ctx->fail(MVGS_EINVAL, "dl_dimages[%d] is NULL", v);
    if (g->P > 0 && (!grads->means || !grads->scales || !grads->quats || !grads->opacities || !grads->sh))
        return ctx->fail(MVGS_EINVAL, "a gradient pointer is NULL");
    if (densify && (!densify->e1 || !densify->e2 || !densify->count))
        return ctx->fail(MVGS_EINVAL, "a densify pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    // records: exact, or in capacity mode bounded by the capacity with the count on the device
    const uint32_t V = f->capacity ? (uint32_t)ctx->cap_v : f->V;
    const uint32_t* eff = frame_eff(f);
    const uint32_t* ovf = frame_void(f);
    Need need[1];
    st = grow_all(ctx, need, backward_needs(ctx, V, need));
    if (st) return st;
    fill_u32_count(as<uint32_t>(ctx->acc), V, eff, kAccStride, 0u, s);
    void* dptrs = nullptr;
    HIPCHK(ctx, ctx->ring.put(dl_dimages, sizeof(float*) * f->B, s, &dptrs, ctx->capturing));
    BlendBwdArgs a;
    a.cams = as<DevCam>(f->cams);
    a.B = f->B;
    a.n_tiles = f->n_tiles;
    a.ranges = as<uint2>(f->ranges);
    a.vals = as<uint32_t>(f->vals[f->final_buf]);
    a.recs = as<BlendRec>(f->recs);
    a.dl_dimg = (const float* const*)dptrs;
    a.t_final = as<float>(f->t_final);
    a.n_last = as<uint32_t>(f->n_last);
    a.acc = as<float>(ctx->acc);
    a.want_e1 = densify != nullptr;
    a.mask = f->mode == MVGS_PARTIAL_MASKED ? as<uint32_t>(f->mask) : nullptr;
    int mk = ctx->stage_begin(8, s);
    if (f->mode == MVGS_PARTIAL_COMPACT) {
        SelBlendArgs sa = sel_args(f);
        sa.dl_dimg = a.dl_dimg;
        sa.acc = a.acc;
        sa.want_e1 = a.want_e1;
        launch_blend_bwd_sel(sa, s);
    } else {
        launch_blend_bwd(a, ctx->tw, ctx->th, f->ppl, s);
    }
    ctx->stage_end(mk, s);
    GradArgs gr;
    gr.means = grads->means;
    gr.scales = grads->scales;
    gr.quats = grads->quats;
    gr.opac = grads->opacities;
    gr.sh = grads->sh;
    gr.e1 = densify ? densify->e1 : nullptr;
    gr.e2 = densify ? densify->e2 : nullptr;
    gr.count = densify ? densify->count : nullptr;
    mk = ctx->stage_begin(9, s);
    launch_preprocess_bwd(gargs(g), as<DevCam>(f->cams), as<uint32_t>(f->rec_off), as<uint16_t>(f->rec_view),
                          as<float>(ctx->acc), gr, s, ovf);
    ctx->stage_end(mk, s);
    LAUNCHCHK(ctx, "backward kernels");
    HIPCHK(ctx, ctx->ring.seal(s));
    return MVGS_OK;
}

int mvgs_frame_release(mvgs_context* ctx, mvgs_frame* frame) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx) return MVGS_EINVAL;
    frame->in_use = false;
    ++frame->gen;
    return MVGS_OK;
}

int mvgs_set_workspace_limit(mvgs_context* ctx, int64_t bytes) {
    if (!ctx || bytes < 0) return MVGS_EINVAL;
    ctx->limit = (size_t)bytes;
    return MVGS_OK;
}

int mvgs_memory_held(mvgs_context* ctx, int64_t* bytes) {
    if (!ctx || !bytes) return MVGS_EINVAL;
    *bytes = (int64_t)ctx->held();
    return MVGS_OK;
}

int mvgs_frame_workspace(const mvgs_frame* frame, int64_t* bytes) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!frame || !bytes) return MVGS_EINVAL;
    *bytes = (int64_t)frame->need_bytes;
    return MVGS_OK;
}

int mvgs_frame_check(mvgs_context* ctx, void* stream, mvgs_frame* frame) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use) return MVGS_EINVAL;
    if (!frame->capacity) return MVGS_OK;
    hipStream_t s = (hipStream_t)stream;
    if (ctx->begin(s)) return ctx->fail(MVGS_EINVAL, "mvgs_frame_check synchronizes and cannot be captured");
    HIPCHK(ctx, hipMemcpyAsync(ctx->pinned_totals, frame->dtot.p, 56, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    const uint64_t V = ctx->pinned_totals[0], K = ctx->pinned_totals[1];
    const uint32_t* e32 = reinterpret_cast<const uint32_t*>(ctx->pinned_totals + 4);
    // the depth-sort window of later forwards: around this frame's keys, whole 8-bit passes
    const uint32_t kmin = e32[4], kmax = ~e32[5];
    if (V > 0 && kmin <= kmax) {   // (the count kernel finds the range whatever else happened)
        const uint32_t range = kmax - kmin;
        const int need = range ? 32 - __builtin_clz(range) : 1;
        const int bits = std::min(32, 8 * ((need + 7) / 8));
        if (bits >= 32) {
            ctx->dwin_base = 0;
            ctx->dwin_bits = 32;
        } else {
            const uint32_t margin = (uint32_t)((((uint64_t)1 << bits) - 1 - range) / 2);
            ctx->dwin_base = kmin >= margin ? kmin - margin : 0u;
            ctx->dwin_bits = bits;
        }
    }
    if (e32[2] & 8u) {
        frame->checked = false;
        return ctx->fail(MVGS_ERETRY, "the depth keys left the sort window that the call was made with; the "
                                      "context's window now fits them: make the call again (capture again)");
    }
    const uint32_t sel_e = frame->mode == kModeFull ? 0u : (uint32_t)(ctx->pinned_totals[2] >> 32);
    if (e32[2] & 2u) {
        frame->checked = false;
        return ctx->fail(MVGS_EINVAL, "pixel selection rejected:%s%s%s%s",
                         (sel_e & kSelBadOffsets) ? " offsets do not rise from 0 to n_sel;" : "",
                         (sel_e & kSelTooLong) ? " a segment holds more pixels than a tile;" : "",
                         (sel_e & kSelOutside) ? " a pixel lies outside its (view, tile);" : "",
                         (sel_e & kSelDuplicate) ? " a pixel is selected twice;" : "");
    }
    if (e32[2] & 4u) {
        frame->checked = false;
        return ctx->fail(MVGS_EHIP, "selection tasks %llu exceed their bound %u",
                         (unsigned long long)ctx->pinned_totals[3], frame->n_tasks);
    }
    if (e32[2]) {
        frame->checked = false;
        return ctx->fail(MVGS_ECAPACITY, "%llu records and %llu pairs exceed the capacities %llu and %llu",
                         (unsigned long long)V, (unsigned long long)K, (unsigned long long)ctx->cap_v,
                         (unsigned long long)ctx->cap_k);
    }
    if (frame->partition && (sel_e & kSelPlaneOverlap)) {
        frame->checked = false;
        return ctx->fail(MVGS_EINVAL, "the selection holds W H pixels but selects a plane position in two views: "
                                      "it is not a partition of the plane, and the 3D loss and merge of the frame "
                                      "are void");
    }
    frame->V = (uint32_t)V;
    frame->K = (uint32_t)K;
    frame->checked = true;
    return MVGS_OK;
}

int mvgs_frame_void_word(const mvgs_frame* frame, const uint32_t** word) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!frame || !word || !frame->in_use) return MVGS_EINVAL;
    *word = frame_void(frame);
    return MVGS_OK;
}

int mvgs_frame_set_cameras(mvgs_context* ctx, mvgs_frame* frame, const mvgs_camera* cams, int32_t B) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use) return MVGS_EINVAL;
    if (!frame->cam_stage) return ctx->fail(MVGS_EINVAL, "the frame was not made under stream capture");
    if (!cams || B != frame->B) return ctx->fail(MVGS_EINVAL, "expected %d cameras", frame->B);
    uint32_t n_tiles = 0, n_pixels = 0;
    int st = validate_cams(ctx, cams, B, ctx->tw, ctx->th, &n_tiles, &n_pixels);
    if (st) return st;
    for (int v = 0; v < B; ++v)
        if (cams[v].width != frame->hcams[v].W || cams[v].height != frame->hcams[v].H)
            return ctx->fail(MVGS_EINVAL, "view %d changes size: a captured graph keeps its sizes", v);
    build_cams(cams, B, ctx->tw, ctx->th, frame->hcams);
    memcpy(frame->cam_stage, frame->hcams.data(), sizeof(DevCam) * B);
    return MVGS_OK;
}

int mvgs_frame_info(const mvgs_frame* frame, int64_t* n_records, int64_t* n_pairs, int64_t* n_tiles) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!frame) return MVGS_EINVAL;
    if (n_records) *n_records = frame->V;
    if (n_pairs) *n_pairs = (int64_t)frame->K;
    if (n_tiles) *n_tiles = frame->n_tiles;
    return MVGS_OK;
}

int mvgs_frame_sort_info(const mvgs_frame* frame, int32_t* depth_passes, int32_t* tile_passes) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!frame) return MVGS_EINVAL;
    // passes of ceil(bits / 8) even digits (k_sort.hip), none for an empty sort
    auto passes = [](int bits, bool empty) { return empty || bits <= 0 ? 0 : std::max(1, (bits + 7) / 8); };
    const bool cap = frame->capacity;
    const bool no_rec = cap ? frame->ctx->cap_v == 0 : frame->V == 0;
    const bool no_pair = cap ? frame->ctx->cap_k == 0 : frame->K == 0;
    if (depth_passes) *depth_passes = passes(frame->depth_bits, no_rec);
    if (tile_passes) *tile_passes = passes(frame->tile_bits, no_rec || no_pair);
    return MVGS_OK;
}

int mvgs_export_binning(mvgs_context* ctx, void* stream, const mvgs_frame* frame, uint64_t* keys, uint32_t* values,
                        uint32_t* ranges) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use) return MVGS_EINVAL;
    if (!frame->checked) return ctx->fail(MVGS_EINVAL, "call mvgs_frame_check on a capacity-mode frame first");
    hipStream_t s = (hipStream_t)stream;
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    if (keys || values)
        launch_export_keys(f->keys[f->final_buf].p, f->key16, as<uint32_t>(f->vals[f->final_buf]),
                           as<BlendRec>(f->recs), as<DevCam>(f->cams), f->B, (uint32_t)f->K, keys, values, s);
    if (ranges && f->n_tiles)
        HIPCHK(ctx, hipMemcpyAsync(ranges, f->ranges.p, sizeof(uint2) * f->n_tiles, hipMemcpyDeviceToDevice, s));
    LAUNCHCHK(ctx, "export binning");
    return MVGS_OK;
}

int mvgs_export_transmittance(mvgs_context* ctx, void* stream, const mvgs_frame* frame, float* const* t_final) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use || !t_final) return MVGS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    for (int v = 0; v < f->B; ++v)
        if (!t_final[v]) return ctx->fail(MVGS_EINVAL, "t_final[%d] is NULL", v);
    ctx->begin(s);
    if (f->mode == MVGS_PARTIAL_COMPACT) {
        void* dptrs = nullptr;
        HIPCHK(ctx, ctx->ring.put(t_final, sizeof(float*) * f->B, s, &dptrs, ctx->capturing));
        launch_sel_scatter(as<DevCam>(f->cams), f->B, f->n_tiles, as<uint32_t>(f->sel_off),
                           as<uint32_t>(f->sel_pix), as<float>(f->t_final), (float* const*)dptrs, s, frame_void(f));
        LAUNCHCHK(ctx, "transmittance scatter");
        HIPCHK(ctx, ctx->ring.seal(s));
        return MVGS_OK;
    }
    for (int v = 0; v < f->B; ++v) {
        const DevCam& c = f->hcams[v];
        HIPCHK(ctx, hipMemcpyAsync(t_final[v], as<float>(f->t_final) + c.pix_base, sizeof(float) * c.W * c.H,
                                   hipMemcpyDeviceToDevice, s));
    }
    return MVGS_OK;
}

int mvgs_frame_merge(mvgs_context* ctx, void* stream, const mvgs_frame* frame, const float* const* planes,
                     int32_t channels, float* out) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx) return MVGS_EINVAL;
    if (!frame || frame->ctx != ctx || !frame->in_use) return ctx->fail(MVGS_EINVAL, "not a live frame");
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    if (f->mode == kModeFull) return ctx->fail(MVGS_EINVAL, "the frame has no pixel selection");
    if (channels < 1 || channels > 64) return ctx->fail(MVGS_EINVAL, "channels=%d outside [1, 64]", channels);
    if (!planes || !out) return ctx->fail(MVGS_EINVAL, "planes or out is NULL");
    for (int v = 0; v < f->B; ++v) {
        if (!planes[v]) return ctx->fail(MVGS_EINVAL, "planes[%d] is NULL", v);
        if (f->hcams[v].W != f->hcams[0].W || f->hcams[v].H != f->hcams[0].H)
            return ctx->fail(MVGS_EINVAL, "merging needs views of one size");
    }
    hipStream_t s = (hipStream_t)stream;
    ctx->begin(s);
    void* dptrs = nullptr;
    HIPCHK(ctx, ctx->ring.put(planes, sizeof(float*) * f->B, s, &dptrs, ctx->capturing));
    launch_sel_merge(as<DevCam>(f->cams), f->B, f->n_tiles, as<uint32_t>(f->sel_off), as<uint32_t>(f->sel_pix),
                     (const float* const*)dptrs, channels, (uint32_t)(f->hcams[0].W * f->hcams[0].H), out, s,
                     frame_void(f));
    LAUNCHCHK(ctx, "selection merge");
    HIPCHK(ctx, ctx->ring.seal(s));
    return MVGS_OK;
}

static const char* kStageNames[MVGS_STAGE_COUNT] = {"count", "records", "depth_sort", "emit", "tile_sort",
                                                     "ranges", "blend_fwd", "loss", "blend_bwd", "preprocess_bwd"};

const char* mvgs_stage_name(int stage) {
    return (stage >= 0 && stage < MVGS_STAGE_COUNT) ? kStageNames[stage] : "unknown";
}

int mvgs_profile_enable(mvgs_context* ctx, int enable) {
    if (!ctx) return MVGS_EINVAL;
    ctx->prof = enable != 0;
    return MVGS_OK;
}

int mvgs_profile_read(mvgs_context* ctx, double* ms, int64_t* calls) {
    if (!ctx) return MVGS_EINVAL;
    for (auto& m : ctx->marks) {
        HIPCHK(ctx, hipEventSynchronize(m.b));
        float t = 0.0f;
        HIPCHK(ctx, hipEventElapsedTime(&t, m.a, m.b));
        ctx->prof_ms[m.stage] += t;
        ctx->prof_calls[m.stage] += 1;
        ctx->ev_pool.push_back(m.a);
        ctx->ev_pool.push_back(m.b);
    }
    ctx->marks.clear();
    for (int i = 0; i < MVGS_STAGE_COUNT; ++i) {
        if (ms) ms[i] = ctx->prof_ms[i];
        if (calls) calls[i] = ctx->prof_calls[i];
    }
    return MVGS_OK;
}

int mvgs_profile_reset(mvgs_context* ctx) {
    if (!ctx) return MVGS_EINVAL;
    int st = mvgs_profile_read(ctx, nullptr, nullptr);
    for (int i = 0; i < MVGS_STAGE_COUNT; ++i) {
        ctx->prof_ms[i] = 0.0;
        ctx->prof_calls[i] = 0;
    }
    return st;
}

int mvgs_frame_work(mvgs_context* ctx, void* stream, const mvgs_frame* frame, uint64_t* work_dev) {
    frame = frame_of(frame);   // NULL for a released or stale handle
    if (!ctx || !frame || frame->ctx != ctx || !frame->in_use || !work_dev) return MVGS_EINVAL;
    mvgs_frame* f = const_cast<mvgs_frame*>(frame);
    if (f->mode == MVGS_PARTIAL_COMPACT)
        launch_frame_work_sel(as<DevCam>(f->cams), f->B, f->n_tiles, as<uint2>(f->ranges),
                              as<uint32_t>(f->vals[f->final_buf]), as<BlendRec>(f->recs), as<uint32_t>(f->sel_off),
                              as<uint32_t>(f->sel_pix), as<uint32_t>(f->n_last), work_dev, (hipStream_t)stream);
    else
        launch_frame_work(as<DevCam>(f->cams), f->B, as<uint2>(f->ranges), as<uint32_t>(f->vals[f->final_buf]),
                          as<BlendRec>(f->recs), as<uint32_t>(f->n_last), f->n_pixels, ctx->tw, ctx->th, work_dev,
                          (hipStream_t)stream);
    LAUNCHCHK(ctx, "frame work");
    return MVGS_OK;
}

}  // extern "C"
