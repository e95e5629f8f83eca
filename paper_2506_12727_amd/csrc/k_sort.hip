// Scans, the stable LSD radix sort, and the (view, tile, depth) binning built on them.
//
// The multi-view appendix of the paper sorts one 64-bit key per (Gaussian, tile) pair holding
// tile, view and depth. The same order -- by (view, tile), then depth, then Gaussian index --
// is reached here in two cheaper stable sorts: the participating (view, Gaussian) records are
// sorted by their 32-bit depth key (one item per record), pairs are then emitted in that depth
// order and sorted stably by their global tile id (view-major, so (view, tile) in one integer of
// ceil(log2(total tiles)) bits). Ties in depth keep the (Gaussian, view) emission order of the
// records, i.e. ascending Gaussian index within a view.
//
// Radix sort: LSD, digits of at most 8 bits spread evenly over the passes, 8192 items per
// partition (4 wavefronts x 32 rounds x 64 lanes). Each pass reduces, scans, then scatters: one
// workgroup per partition counts its digits (LDS counters) into a digit-major table, one exclusive
// scan of that table gives every (digit, partition) its output base, and one workgroup per
// partition ranks its items stably with wave64 ballots, stages them in LDS in digit order and
// writes them out in contiguous runs. Nothing waits on another workgroup. (A single-sweep pass
// with decoupled look-back was measured slower on this chip: its device-scope look-back latency
// across the XCDs cost more than the extra read of the keys.)
#include <algorithm>

#include "mvgs_kernels.h"

namespace mvgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // 4096

constexpr int kSortWaves = 4;
constexpr int kSortRounds = 32;
constexpr int kSortThreads = kSortWaves * 64;
constexpr int kSortTile = kSortWaves * kSortRounds * 64;  // 8192
constexpr int kRadix = 256;

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, size_t n, uint64_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// exclusive scan of 256 values held one per thread; returns the exclusive prefix, sets *total
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* lds, uint32_t* total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
#pragma unroll
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = (t >= off) ? lds[t - off] : 0u;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    const uint32_t incl = lds[t];
    *total = lds[255];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const uint32_t* __restrict__ in, size_t n,
                                                              const uint32_t* __restrict__ n_dev,
                                                              uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t lds[256];
    n = count_of(n, n_dev);
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    uint32_t total;
    (void)block_exclusive_scan_256(s, lds, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t* in, uint32_t* out, size_t n,
                                                             const uint32_t* __restrict__ n_dev,
                                                             const uint32_t* __restrict__ block_off) {
    __shared__ uint32_t lds[256];
    n = count_of(n, n_dev);
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (base + k < n) ? in[base + k] : 0u;
        s += vals[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan_256(s, lds, &total) + (block_off ? block_off[blockIdx.x] : 0u);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += vals[k];
    }
}

__global__ void __launch_bounds__(256) k_reduce64(const uint32_t* __restrict__ in, size_t n,
                                                  unsigned long long* __restrict__ total) {
    __shared__ unsigned long long part[256];
    unsigned long long s = 0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) s += in[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, part[0]);
}

static size_t div_up(size_t a, size_t b) { return (a + b - 1) / b; }

void fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);

size_t scan_scratch_bytes(size_t n) {
    size_t bytes = 256;
    size_t m = n;
    while (m > (size_t)kScanTile) {
        m = div_up(m, kScanTile);
        bytes += m * sizeof(uint32_t) + 256;
    }
    return bytes;
}

static void fill_u64(uint64_t* p, size_t n, uint64_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, p, n, v);
}

void reduce_sum_u32(const uint32_t* in, size_t n, uint64_t* total64, void* scratch, hipStream_t s) {
    (void)scratch;
    fill_u64(total64, 1, 0, s);
    if (n == 0) return;
    const unsigned blocks = (unsigned)std::min<size_t>(div_up(n, 256), 2048);
    hipLaunchKernelGGL(k_reduce64, dim3(blocks), dim3(256), 0, s, in, n, (unsigned long long*)total64);
}

// n is the bound that sizes the grids; n_dev (device, may be null) the count actually scanned.
static void scan_rec(const uint32_t* in, uint32_t* out, size_t n, const uint32_t* n_dev, uint8_t* scratch,
                     hipStream_t s) {
    const size_t blocks = div_up(n, kScanTile);
    if (blocks <= 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                           (const uint32_t*)nullptr);
        return;
    }
    uint32_t* sums = (uint32_t*)scratch;
    uint8_t* next = scratch + ((blocks * sizeof(uint32_t) + 255) / 256) * 256;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, in, n, n_dev, sums);
    scan_rec(sums, sums, blocks, nullptr, next, s);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                       (const uint32_t*)sums);
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, size_t n, uint64_t* total64, void* scratch,
                        hipStream_t s, const uint32_t* n_dev) {
    if (total64) reduce_sum_u32(in, n, total64, nullptr, s);
    if (n == 0) return;
    scan_rec(in, out, n, n_dev, (uint8_t*)scratch, s);
}

// ---------------------------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------------------------

// lanes of this wave holding the same 8-bit digit (among `valid` lanes)
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t peers = ballot64(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot64(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Reduce-then-scan pass, step 1: per-partition digit counts, digit-major (counts[d * parts + p]),
// so that one exclusive scan of the whole array gives every (digit, partition) its output base.
__global__ void __launch_bounds__(256) k_radix_upsweep(const uint32_t* __restrict__ keys, size_t n,
                                                       const uint32_t* __restrict__ n_dev, int shift, uint32_t mask,
                                                       uint32_t parts, uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    n = count_of(n, n_dev);
    const size_t base = (size_t)blockIdx.x * kSortTile;
    if (base + kSortTile <= n) {
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base);
        for (int j = threadIdx.x; j < kSortTile / 4; j += 256) {
            const uint4 k = k4[j];
            atomicAdd(&h[(k.x >> shift) & mask], 1u);
            atomicAdd(&h[(k.y >> shift) & mask], 1u);
            atomicAdd(&h[(k.z >> shift) & mask], 1u);
            atomicAdd(&h[(k.w >> shift) & mask], 1u);
        }
    } else {
        for (int j = threadIdx.x; j < kSortTile; j += 256) {
            const size_t i = base + j;
            if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    counts[(size_t)threadIdx.x * parts + blockIdx.x] = h[threadIdx.x];
}

// Step 3: rank each partition's items stably with wave64 ballots and scatter them through LDS in
// digit order to the bases the scan gave.
__global__ void __launch_bounds__(kSortThreads) k_radix_downsweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, size_t n, const uint32_t* __restrict__ n_dev, int shift, uint32_t mask,
    uint32_t parts, const uint32_t* __restrict__ offsets) {
    __shared__ uint32_t wcount[kSortWaves][kRadix];
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t scan_tmp[kRadix];
    __shared__ uint32_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int d = threadIdx.x; d < kSortWaves * kRadix; d += kSortThreads) (&wcount[0][0])[d] = 0;
    const uint32_t part = blockIdx.x;
    n = count_of(n, n_dev);
    if ((size_t)part * kSortTile >= n) return;
    gbase[threadIdx.x] = offsets[(size_t)threadIdx.x * parts + part];
    __syncthreads();
    const size_t base = (size_t)part * kSortTile + (size_t)wave * kSortRounds * 64;
    uint32_t key[kSortRounds], val[kSortRounds], rank[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? keys_in[i] : 0xffffffffu;
        val[r] = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = (key[r] >> shift) & mask;
        const uint64_t peers = digit_peers(d, valid);
        const uint32_t below = (uint32_t)rank_below(peers);
        const uint32_t before = wcount[wave][d];
        rank[r] = before + below;
        wave_lds_sync();
        if (valid && below == 0) wcount[wave][d] = before + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) {
            const uint32_t c = wcount[w][d];
            wcount[w][d] = run;
            run += c;
        }
        uint32_t total;
        dstart[d] = block_exclusive_scan_256(run, scan_tmp, &total);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        if (i < n) {
            const uint32_t d = (key[r] >> shift) & mask;
            const uint32_t pos = dstart[d] + wcount[wave][d] + rank[r];
            skey[pos] = key[r];
            sval[pos] = val[r];
        }
    }
    __syncthreads();
    const size_t tile_n = std::min<size_t>((size_t)kSortTile, n - (size_t)part * kSortTile);
    for (int j = threadIdx.x; j < (int)tile_n; j += kSortThreads) {
        const uint32_t k = skey[j];
        const uint32_t d = (k >> shift) & mask;
        const size_t dst = (size_t)gbase[d] + (uint32_t)(j - dstart[d]);
        keys_out[dst] = k;
        vals_out[dst] = sval[j];
    }
}

size_t radix_scratch_bytes(size_t n) {
    const size_t parts = std::max<size_t>(1, div_up(n, kSortTile));
    return align256(parts * kRadix * sizeof(uint32_t)) + scan_scratch_bytes(parts * kRadix);
}

int radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], bool identity_values, size_t n, int bits, void* scratch,
                   hipStream_t s, const uint32_t* n_dev) {
    int cur = 0;
    if (n == 0 || bits <= 0) return cur;
    // fewest 8-bit passes, digits spread evenly over them (fewer distinct digits per workgroup
    // give longer runs of consecutive stores)
    const int passes = (bits + 7) / 8;
    const int dbits = (bits + passes - 1) / passes;
    const uint32_t mask = (1u << dbits) - 1u;
    const size_t parts = div_up(n, kSortTile);
    uint8_t* p = (uint8_t*)scratch;
    uint32_t* counts = (uint32_t*)p;
    p += align256(parts * kRadix * sizeof(uint32_t));
    for (int pass = 0; pass < passes; ++pass) {
        const uint32_t* vin = (pass == 0 && identity_values) ? nullptr : vals[cur];
        hipLaunchKernelGGL(k_radix_upsweep, dim3((unsigned)parts), dim3(256), 0, s, keys[cur], n, n_dev, dbits * pass,
                           mask, (uint32_t)parts, counts);
        scan_exclusive_u32(counts, counts, parts * kRadix, nullptr, p, s, nullptr);
        hipLaunchKernelGGL(k_radix_downsweep, dim3((unsigned)parts), dim3(kSortThreads), 0, s, keys[cur], vin,
                           keys[cur ^ 1], vals[cur ^ 1], n, n_dev, dbits * pass, mask, (uint32_t)parts,
                           (const uint32_t*)counts);
        cur ^= 1;
    }
    return cur;
}

// ---------------------------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t rect_tiles(uint4 r) { return (r.y & 0xffffu) * (r.y >> 16); }

// The one gather of the records' tile rectangles in depth order: pair counts, and the rectangles
// themselves in that order so that pair emission reads them sequentially.
__global__ void k_gather_tile_counts(const uint32_t* __restrict__ sorted_rec, const uint4* __restrict__ rect,
                                     uint32_t n, const uint32_t* __restrict__ n_dev, uint32_t* __restrict__ counts,
                                     uint4* __restrict__ sorted_rect) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (uint32_t)count_of(n, n_dev)) {
        const uint4 r = rect[sorted_rec[i]];
        counts[i] = rect_tiles(r);
        sorted_rect[i] = r;
    }
}

// Load-balanced emission: a workgroup takes 256 consecutive records of the depth order; their
// pairs are contiguous in the output, so the workgroup's lanes walk those pairs in order (each
// store is coalesced across the wavefront) and find their record by binary search over the
// workgroup's prefix sums in LDS. Pair j of a record with a w-tile-wide rectangle is tile
// (tx0 + j mod w, ty0 + j / w), row-major, as a per-record loop would emit them.
constexpr int kEmitThreads = 256;

__global__ void __launch_bounds__(kEmitThreads) k_emit_pairs(const uint32_t* __restrict__ sorted_rec,
                                                             const uint4* __restrict__ sorted_rect,
                                                             const uint32_t* __restrict__ pair_off, uint32_t n,
                                                             uint32_t K, const uint32_t* __restrict__ counts_dev,
                                                             uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_off[kEmitThreads + 1];   // local exclusive offsets (+ total)
    __shared__ uint32_t s_rec[kEmitThreads];
    __shared__ uint32_t s_x[kEmitThreads];         // width in tiles
    __shared__ uint32_t s_base[kEmitThreads];      // global tile id of the first covered tile
    __shared__ uint32_t s_stride[kEmitThreads];    // tiles per row of the record's view
    // counts_dev: (records, pairs) actually present, when the grid is sized by bounds
    if (counts_dev) {
        n = (uint32_t)count_of(n, counts_dev);
        K = (uint32_t)count_of(K, counts_dev + 1);
    }
    const uint32_t i0 = blockIdx.x * kEmitThreads;
    if (i0 >= n) return;
    const uint32_t i = i0 + threadIdx.x;
    const uint32_t base_out = pair_off[i0];
    if (i < n) {
        const uint32_t r = sorted_rec[i];
        const uint4 rc = sorted_rect[i];
        s_rec[threadIdx.x] = r;
        s_x[threadIdx.x] = rc.y & 0xffffu;
        s_base[threadIdx.x] = rc.x;
        s_stride[threadIdx.x] = rc.z;
        s_off[threadIdx.x] = pair_off[i] - base_out;
    }
    const uint32_t last = min(n - i0, (uint32_t)kEmitThreads);
    if (threadIdx.x == 0) s_off[last] = (i0 + last < n ? pair_off[i0 + last] : K) - base_out;
    __syncthreads();
    const uint32_t total = s_off[last];
    for (uint32_t j = threadIdx.x; j < total; j += kEmitThreads) {
        // record k with s_off[k] <= j < s_off[k + 1]
        uint32_t lo = 0, hi = last;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= j) lo = mid;
            else hi = mid;
        }
        const uint32_t t = j - s_off[lo];
        const uint32_t w = s_x[lo];
        // t < 65536, so (t + 0.5) / w in float32 is never within rounding of an integer
        const uint32_t row = (uint32_t)floorf(((float)t + 0.5f) * __builtin_amdgcn_rcpf((float)w));
        const uint32_t col = t - row * w;
        const uint32_t o = base_out + j;
        if (o >= K) break;
        keys[o] = s_base[lo] + row * s_stride[lo] + col;
        vals[o] = s_rec[lo];
    }
}

// [start, end) of each global tile's run in the sorted pair keys, by binary search
__global__ void __launch_bounds__(256) k_ranges_search(const uint32_t* __restrict__ keys, uint32_t K,
                                                       const uint32_t* __restrict__ K_dev, uint32_t n_tiles,
                                                       uint2* __restrict__ ranges) {
    const uint32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= n_tiles) return;
    K = (uint32_t)count_of(K, K_dev);
    uint32_t lo = 0, hi = K;  // first index with keys[i] >= t
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (keys[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    uint32_t lo2 = lo, hi2 = K;  // first index with keys[i] > t
    while (lo2 < hi2) {
        const uint32_t mid = lo2 + ((hi2 - lo2) >> 1);
        if (keys[mid] <= t) lo2 = mid + 1;
        else hi2 = mid;
    }
    ranges[t] = lo2 > lo ? make_uint2(lo, lo2) : make_uint2(0u, 0u);
}

__global__ void k_export_keys(const uint32_t* __restrict__ tile_keys, const uint32_t* __restrict__ vals,
                              const BlendRec* __restrict__ recs, const DevCam* __restrict__ cams, uint32_t K,
                              uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const uint32_t r = vals[i];
    const BlendRec& rec = recs[r];
    const uint32_t local = tile_keys[i] - cams[rec.view].tile_base;
    if (keys_out) keys_out[i] = ((uint64_t)rec.view << 48) | ((uint64_t)local << 32) | (uint64_t)rec.depth_bits;
    if (vals_out) vals_out[i] = rec.gid;
}

void launch_gather_tile_counts(const uint32_t* sorted_rec, const uint4* tile_rect, uint32_t n, uint32_t* counts,
                               uint4* sorted_rect, hipStream_t s, const uint32_t* n_dev) {
    if (!n) return;
    hipLaunchKernelGGL(k_gather_tile_counts, dim3((n + 255) / 256), dim3(256), 0, s, sorted_rec, tile_rect, n,
                       n_dev, counts, sorted_rect);
}

void launch_emit_pairs(const uint32_t* sorted_rec, const uint4* sorted_rect, const uint32_t* pair_off, uint32_t n,
                       uint32_t K, uint32_t* keys, uint32_t* vals, hipStream_t s, const uint32_t* counts_dev) {
    if (!n || !K) return;
    hipLaunchKernelGGL(k_emit_pairs, dim3((n + kEmitThreads - 1) / kEmitThreads), dim3(kEmitThreads), 0, s,
                       sorted_rec, sorted_rect, pair_off, n, K, counts_dev, keys, vals);
}

void launch_ranges(const uint32_t* keys, uint32_t K, uint32_t n_tiles, uint2* ranges, hipStream_t s,
                   const uint32_t* K_dev) {
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_ranges_search, dim3((n_tiles + 255) / 256), dim3(256), 0, s, keys, K, K_dev, n_tiles,
                       ranges);
}

void launch_export_keys(const uint32_t* tile_keys, const uint32_t* vals, const BlendRec* recs,
                        const DevCam* cams, int B, uint32_t K, uint64_t* keys_out, uint32_t* vals_out,
                        hipStream_t s) {
    (void)B;
    if (!K) return;
    hipLaunchKernelGGL(k_export_keys, dim3((K + 255) / 256), dim3(256), 0, s, tile_keys, vals, recs, cams, K,
                       keys_out, vals_out);
}

void fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, p, n, v);
}

__global__ void k_fill_u32_count(uint32_t* __restrict__ p, size_t n, const uint32_t* __restrict__ n_dev, uint32_t per,
                                 uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < (size_t)per * count_of(n, n_dev)) p[i] = v;
}

void fill_u32_count(uint32_t* p, size_t n, const uint32_t* n_dev, uint32_t per, uint32_t v, hipStream_t s) {
    if (!n || !per) return;
    hipLaunchKernelGGL(k_fill_u32_count, dim3((unsigned)div_up(n * per, 256)), dim3(256), 0, s, p, n, n_dev, per, v);
}

// Capacity mode: the records and pairs of this call against the buffers' capacities. Within them,
// eff = (V, K); beyond either, eff = (0, 0) and the overflow word is set, so every later kernel
// does no work and stays inside its buffers.
__global__ void k_capacity_clamp(const unsigned long long* __restrict__ totals, uint64_t cap_v, uint64_t cap_k,
                                 uint32_t* __restrict__ eff, uint32_t* __restrict__ overflow) {
    const uint64_t V = totals[0], K = totals[1];
    const bool over = V > cap_v || K > cap_k;
    eff[0] = over ? 0u : (uint32_t)V;
    eff[1] = over ? 0u : (uint32_t)K;
    overflow[0] = over ? 1u : 0u;
}

void launch_capacity_clamp(const uint64_t* totals, uint64_t cap_v, uint64_t cap_k, uint32_t* eff, uint32_t* overflow,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_capacity_clamp, dim3(1), dim3(1), 0, s, (const unsigned long long*)totals, cap_v, cap_k, eff,
                       overflow);
}

}  // namespace mvgs
