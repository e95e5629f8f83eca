// Scans, the stable LSD radix sort, and the (view, tile, depth) binning built on them.
//
// The multi-view appendix of the paper sorts one 64-bit key per (Gaussian, tile) pair holding
// tile, view and depth. The same order -- by (view, tile), then depth, then Gaussian index --
// is reached here in two cheaper stable sorts: the participating (view, Gaussian) records are
// sorted by their 32-bit depth key (one item per record), pairs are then emitted in that depth
// order and sorted stably by their global tile id (view-major, so (view, tile) in one integer of
// ceil(log2(total tiles)) bits). Ties in depth keep the (Gaussian, view) emission order of the
// records, i.e. ascending Gaussian index within a view. The depth sort orders key - min over only
// the bits in which the keys differ, and the first pass of the tile sort is fused with emission.
//
// Radix sort: LSD, digits of at most 8 bits spread evenly over the passes, 8192 items per
// partition (8 wavefronts x 16 rounds x 64 lanes in the scatter). Each pass reduces, scans, then
// scatters: one workgroup per partition counts its digits (LDS counters) into a digit-major
// table, one exclusive scan of that table gives every (digit, partition) its output base, and one
// workgroup per partition ranks its items stably with wave64 ballots, stages them in LDS in digit
// order and writes them out in contiguous runs. Nothing waits on another workgroup. (A
// single-sweep pass with decoupled look-back was measured slower on this chip: its device-scope
// look-back latency across the XCDs cost more than the extra read of the keys.) The tile ids of
// the pairs are 16-bit keys while a batch has at most 65,536 tiles, 32-bit above.
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
// wavefronts of the downsweeps: 8 x 16 rounds over the same 8192-item partition fit four waves
// per SIMD (4 x 32 rounds: two); the payload's digit bytes share the count table's LDS
constexpr int kPlainWaves = 8;
constexpr int kPayWaves = 8;

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(uint64_t* __restrict__ p, size_t n, uint64_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// exclusive scan of one value per thread over a workgroup of THREADS (a multiple of 64): each
// wavefront scans its 64 values with shuffles, then the wavefront totals are combined through LDS
// (lds: at least THREADS / 64 words). Returns the exclusive prefix and sets *total; lds may be
// reused on return.
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds, uint32_t* total) {
    constexpr int WAVES = THREADS / 64;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = lds[w];
        before += w < wave ? c : 0u;
        all += c;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t* lds, uint32_t* total) {
    return block_exclusive_scan<256>(v, lds, total);
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

// block_off: the scanned block sums (the block's base is block_off[block]); or block_sums: the
// block sums themselves, which the block adds up to its base (few blocks: one kernel less)
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t* in, uint32_t* out, size_t n,
                                                             const uint32_t* __restrict__ n_dev,
                                                             const uint32_t* __restrict__ block_off,
                                                             const uint32_t* __restrict__ block_sums) {
    __shared__ uint32_t lds[256];
    n = count_of(n, n_dev);
    uint32_t off = block_off ? block_off[blockIdx.x] : 0u;
    if (block_sums) {
        uint32_t part = 0;
        for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanThreads) part += block_sums[b];
        (void)block_exclusive_scan_256(part, lds, &off);
    }
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t vals[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        vals[k] = (base + k < n) ? in[base + k] : 0u;
        s += vals[k];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan_256(s, lds, &total) + off;
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
    const size_t stride = (size_t)gridDim.x * 256;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride)   // four independent loads in flight per thread
        s += (unsigned long long)in[i] + in[i + stride] + in[i + 2 * stride] + in[i + 3 * stride];
    for (; i < n; i += stride) s += in[i];
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
    // one 64-bit atomic per workgroup on a single address: few workgroups, each looping over
    // 4,096 or more values (2,048 workgroups had cost 27 us on 1M values, almost all contention)
    const unsigned blocks = (unsigned)std::min<size_t>(div_up(n, 4096), 256);
    hipLaunchKernelGGL(k_reduce64, dim3(blocks), dim3(256), 0, s, in, n, (unsigned long long*)total64);
}

// n is the bound that sizes the grids; n_dev (device, may be null) the count actually scanned.
static void scan_rec(const uint32_t* in, uint32_t* out, size_t n, const uint32_t* n_dev, uint8_t* scratch,
                     hipStream_t s) {
    const size_t blocks = div_up(n, kScanTile);
    if (blocks <= 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                           (const uint32_t*)nullptr, (const uint32_t*)nullptr);
        return;
    }
    uint32_t* sums = (uint32_t*)scratch;
    uint8_t* next = scratch + ((blocks * sizeof(uint32_t) + 255) / 256) * 256;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, in, n, n_dev, sums);
    if (blocks <= 16 * kScanThreads) {   // each block adds up at most 16 sums per thread itself
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                           (const uint32_t*)nullptr, (const uint32_t*)sums);
        return;
    }
    scan_rec(sums, sums, blocks, nullptr, next, s);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                       (const uint32_t*)sums, (const uint32_t*)nullptr);
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

// lanes of this wave holding the same digit of nbits <= 8 bits (among `valid` lanes): per bit, the lane's bit
// spread over a word (0 or ~0) is both the ballot's predicate and the mask that keeps the ballot
// or its complement, so the update is one three-input logic op per half of the peer mask
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid, int nbits) {
    const uint64_t v = ballot64(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        if (b >= nbits) break;   // uniform: one ballot per bit of the pass's digit
        const uint32_t splat = (uint32_t)((int32_t)(d << (31 - b)) >> 31);
        const uint64_t m = ballot64((int32_t)splat < 0);
        lo &= ~((uint32_t)m ^ splat);
        hi &= ~((uint32_t)(m >> 32) ^ splat);
    }
    return ((uint64_t)hi << 32) | lo;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Reduce-then-scan pass, step 1: per-partition digit counts, digit-major (counts[d * parts + p] for
// the mask + 1 digits of the pass), so that one exclusive scan of the whole table gives every
// (digit, partition) its output base. KT: 32- or 16-bit keys.
template <typename KT>
__global__ void __launch_bounds__(256) k_radix_upsweep(const KT* __restrict__ keys, size_t n,
                                                       const uint32_t* __restrict__ n_dev, uint32_t key_base, int shift,
                                                       uint32_t mask, uint32_t parts, uint32_t* __restrict__ counts) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    n = count_of(n, n_dev);
    const size_t base = (size_t)blockIdx.x * kSortTile;
    if (base + kSortTile <= n) {
        // 16 bytes per load: four 32-bit or eight 16-bit keys
        constexpr int kPer = 16 / (int)sizeof(KT);
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base);
        for (int j = threadIdx.x; j < kSortTile / kPer; j += 256) {
            const uint4 k = k4[j];
            const uint32_t w[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (sizeof(KT) == 4) {
                    atomicAdd(&h[((w[e] - key_base) >> shift) & mask], 1u);
                } else {
                    atomicAdd(&h[(((w[e] & 0xffffu) - key_base) >> shift) & mask], 1u);
                    atomicAdd(&h[(((w[e] >> 16) - key_base) >> shift) & mask], 1u);
                }
            }
        }
    } else {
        for (int j = threadIdx.x; j < kSortTile; j += 256) {
            const size_t i = base + j;
            if (i < n) atomicAdd(&h[(((uint32_t)keys[i] - key_base) >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x <= mask) counts[(size_t)threadIdx.x * parts + blockIdx.x] = h[threadIdx.x];
}

// Step 3: rank each partition's items stably with wave64 ballots and scatter them through LDS in
// digit order to the bases the scan gave. PAY: an 8-byte payload per item follows its key, staged
// through the same LDS after the keys and values are out (the digits of the staged order kept
// aside for it). KT: 32- or 16-bit keys (staged as 32 bits).
template <bool PAY, int WAVES, typename KT>
__global__ void __launch_bounds__(WAVES * 64) k_radix_downsweep(
    const KT* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, KT* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const uint2* __restrict__ pay_in, uint2* __restrict__ pay_out, size_t n,
    const uint32_t* __restrict__ n_dev, uint32_t key_base, int shift, uint32_t mask, uint32_t parts,
    const uint32_t* __restrict__ offsets) {
    constexpr int ROUNDS = kSortTile / (WAVES * 64);
    constexpr int THREADS = WAVES * 64;
    // the per-wavefront digit counts; once the items are staged, PAY keeps the digit of every
    // staged position in the same bytes
    __shared__ union {
        uint32_t wcount[WAVES][kRadix];
        uint8_t sdig[kSortTile];
    } cd;
    auto& wcount = cd.wcount;
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t scan_tmp[kRadix];
    __shared__ union {
        struct {
            uint32_t k[kSortTile];
            uint32_t v[kSortTile];
        } kv;
        uint2 p[kSortTile];
    } stg;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nbits = 32 - __builtin_clz(mask | 1u);   // bits of this pass's digit
    for (int d = threadIdx.x; d < WAVES * kRadix; d += THREADS) (&wcount[0][0])[d] = 0;
    const uint32_t part = blockIdx.x;
    n = count_of(n, n_dev);
    if ((size_t)part * kSortTile >= n) return;
    if (threadIdx.x < kRadix) gbase[threadIdx.x] = threadIdx.x <= mask ? offsets[(size_t)threadIdx.x * parts + part] : 0u;
    __syncthreads();
    const size_t base = (size_t)part * kSortTile + (size_t)wave * ROUNDS * 64;
    uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? (uint32_t)keys_in[i] : 0xffffffffu;
        val[r] = valid ? (vals_in ? vals_in[i] : (uint32_t)i) : 0u;
    }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = ((key[r] - key_base) >> shift) & mask;
        const uint64_t peers = digit_peers(d, valid, nbits);
        const uint32_t below = (uint32_t)rank_below(peers);
        const uint32_t before = wcount[wave][d];
        rank[r] = before + below;
        wave_lds_sync();
        if (valid && below == 0) wcount[wave][d] = before + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();
    {
        // digit d = threadIdx.x (threads past the 256 digits join the scan with 0)
        const int d = threadIdx.x;
        uint32_t run = 0;
        if (d < kRadix) {
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint32_t c = wcount[w][d];
                wcount[w][d] = run;
                run += c;
            }
        }
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<THREADS>(run, scan_tmp, &total);
        if (d < kRadix) dstart[d] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const size_t i = base + (size_t)r * 64 + lane;
        if (i < n) {
            const uint32_t d = ((key[r] - key_base) >> shift) & mask;
            const uint32_t pos = dstart[d] + wcount[wave][d] + rank[r];
            stg.kv.k[pos] = key[r];
            stg.kv.v[pos] = val[r];
            rank[r] = pos;
        }
    }
    __syncthreads();   // (the counts are read for the last time above)
    if (PAY) {
#pragma unroll
        for (int r = 0; r < ROUNDS; ++r) {
            const size_t i = base + (size_t)r * 64 + lane;
            if (i < n) cd.sdig[rank[r]] = (uint8_t)(((key[r] - key_base) >> shift) & mask);
        }
    }
    const size_t tile_n = std::min<size_t>((size_t)kSortTile, n - (size_t)part * kSortTile);
    for (int j = threadIdx.x; j < (int)tile_n; j += THREADS) {
        const uint32_t k = stg.kv.k[j];
        const uint32_t d = ((k - key_base) >> shift) & mask;
        const size_t dst = (size_t)gbase[d] + (uint32_t)(j - dstart[d]);
        if (keys_out) keys_out[dst] = (KT)k;   // null: the keys are not needed after this pass
        vals_out[dst] = stg.kv.v[j];
    }
    if (PAY) {
        __syncthreads();   // the keys and values are out of the staging area
        // eight loads in flight at a time (all of them at once would raise the registers the kernel
        // needs and lower its occupancy)
#pragma unroll
        for (int r0 = 0; r0 < ROUNDS; r0 += 8) {
            uint2 pv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const size_t i = base + (size_t)(r0 + q) * 64 + lane;
                pv[q] = i < n ? pay_in[i] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const size_t i = base + (size_t)(r0 + q) * 64 + lane;
                if (i < n) stg.p[rank[r0 + q]] = pv[q];
            }
            asm volatile("" ::: "memory");
        }
        __syncthreads();
        for (int j = threadIdx.x; j < (int)tile_n; j += THREADS) {
            const uint32_t d = cd.sdig[j];
            pay_out[(size_t)gbase[d] + (uint32_t)(j - dstart[d])] = stg.p[j];
        }
    }
}

size_t radix_scratch_bytes(size_t n) {
    const size_t parts = std::max<size_t>(1, div_up(n, kSortTile));
    return align256(parts * kRadix * sizeof(uint32_t)) + scan_scratch_bytes(parts * kRadix);
}

// fewest passes of at most 8 bits, digits spread evenly over them (fewer distinct digits per
// workgroup give longer runs of consecutive stores)
struct PassPlan {
    int passes, dbits;
    uint32_t mask;
};
static PassPlan plan_passes(int bits) {
    PassPlan pl;
    pl.passes = std::max(1, (bits + 7) / 8);
    pl.dbits = (bits + pl.passes - 1) / pl.passes;
    pl.mask = (1u << pl.dbits) - 1u;
    return pl;
}

// The tile sort: the first pass (fused with emission) takes the low tile bits, the passes after
// it the rest, in even digits of at most 8 bits. (Uneven splits of the 14 bits of 9,996 tiles
// were slower: emission + second pass 0.708 ms with 6 + 8 bits and 0.746 ms with 8 + 6, against
// 0.697 ms with 7 + 7.)
static int tile_first_bits(int bits) { return plan_passes(bits).dbits; }

// one reduce-then-scan pass over n items (bound; n_dev the count on the device)
template <typename KT>
static void radix_pass(const KT* keys_in, const uint32_t* vals_in, KT* keys_out, uint32_t* vals_out, size_t n,
                       const uint32_t* n_dev, uint32_t base, int shift, uint32_t mask, void* scratch, hipStream_t s,
                       const uint2* pay_in = nullptr, uint2* pay_out = nullptr) {
    const size_t parts = div_up(n, kSortTile);
    uint8_t* p = (uint8_t*)scratch;
    uint32_t* counts = (uint32_t*)p;
    p += align256(parts * kRadix * sizeof(uint32_t));
    hipLaunchKernelGGL(k_radix_upsweep<KT>, dim3((unsigned)parts), dim3(256), 0, s, keys_in, n, n_dev, base, shift,
                       mask, (uint32_t)parts, counts);
    scan_exclusive_u32(counts, counts, parts * ((size_t)mask + 1), nullptr, p, s, nullptr);
    if (pay_in)
        hipLaunchKernelGGL((k_radix_downsweep<true, kPayWaves, KT>), dim3((unsigned)parts), dim3(kPayWaves * 64), 0,
                           s, keys_in, vals_in, keys_out, vals_out, pay_in, pay_out, n, n_dev, base, shift, mask,
                           (uint32_t)parts, (const uint32_t*)counts);
    else
        hipLaunchKernelGGL((k_radix_downsweep<false, kPlainWaves, KT>), dim3((unsigned)parts), dim3(kPlainWaves * 64),
                           0, s, keys_in, vals_in, keys_out, vals_out, nullptr, nullptr, n, n_dev, base, shift, mask,
                           (uint32_t)parts, (const uint32_t*)counts);
}

int radix_sort_u32(uint32_t* keys[2], uint32_t* vals[2], bool identity_values, size_t n, int bits, void* scratch,
                   hipStream_t s, const uint32_t* n_dev, uint32_t key_base, uint2* pay[2], bool sorted_keys) {
    int cur = 0;
    if (n == 0 || bits <= 0) return cur;
    const PassPlan pl = plan_passes(bits);
    for (int pass = 0; pass < pl.passes; ++pass) {
        const uint32_t* vin = (pass == 0 && identity_values) ? nullptr : vals[cur];
        uint32_t* kout = (pass + 1 == pl.passes && !sorted_keys) ? nullptr : keys[cur ^ 1];
        radix_pass<uint32_t>(keys[cur], vin, kout, vals[cur ^ 1], n, n_dev, key_base, pl.dbits * pass, pl.mask,
                             scratch, s, pay ? pay[cur] : nullptr, pay ? pay[cur ^ 1] : nullptr);
        cur ^= 1;
    }
    return cur;
}

// ---------------------------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t rect_tiles(uint2 r) { return (r.y & 0xffffu) * (r.y >> 16); }


// Pair emission fused with the first pass of the stable sort by global tile id. A workgroup takes
// a chunk of RECS consecutive records of the depth order (512, or 1,024 when records cover fewer
// than four tiles on average, so that a chunk's pairs still fill most of a batch); their pairs, in depth order and
// row-major over each record's tile rectangle, are the chunk's items (the partition of the first
// pass). Both kernels generate them alike: the chunk's rectangles (carried through the depth sort,
// so read in order) and the exclusive prefix of their tile counts are staged in LDS; a lane finds
// the record of the first pair of its run by binary search over that prefix and walks on from
// there (pair t of a record whose rectangle is w tiles wide is tile (tx0 + t mod w, ty0 + t / w)).
// The upsweep counts the digits of the chunk's pairs, a contiguous run per thread; the downsweep,
// in batches of kEmitBatch, lets each lane walk kEmitRounds consecutive pairs, hands them to the wave64
// ballot ranking in round order through LDS, stages the batch in digit order and writes it out in
// runs. The emitted pairs are never stored unsorted.
constexpr int kEmitRecs = 512;        // the smaller chunk (it bounds the count table)
constexpr int kEmitRecsSmall = 1024;  // chunk of records that cover few tiles each
// the downsweep: 4 wavefronts, each ranking 16 rounds of 64 pairs per batch (8 wavefronts of 8
// rounds fit four waves per SIMD instead of three but were slower: 0.423 against 0.407 ms on 54.7M
// pairs, twice the searches per batch)
constexpr int kEmitWaves = 4;
constexpr int kEmitThreads = kEmitWaves * 64;
constexpr int kEmitBatch = 4096;
constexpr int kEmitRounds = kEmitBatch / kEmitThreads;
// per wavefront, its pairs lane-major (lane l walks pairs R l .. R l + R - 1, R = kEmitRounds),
// padded to R + 1 words per lane so that neither the lane-major writes nor the round-major reads
// conflict
constexpr int kEmitPad = kEmitRounds + 1;
constexpr int kEmitStageWords = kEmitWaves * 64 * kEmitPad;   // >= kEmitBatch

// views whose first tile id and tiles per row are staged in LDS for the rectangles' view lookup
// (a batch of more views searches the camera array in global memory). Sized so that the
// downsweep's LDS (allocated in 512-byte granules) still lets three workgroups share a CU: 256
// views made it 2 KB larger and cost a third of its occupancy (317 -> 458 us on the 1M batch).
constexpr int kEmitViews = 128;

template <int RECS>
struct EmitStage {
    uint32_t off[RECS + 1];   // exclusive prefix of the pair counts (+ total)
    uint32_t base[RECS];      // global tile id of the first covered tile
    uint32_t ws[RECS];        // (rectangle width - 1) | (tiles per row of its view - 1) << 16
                              // (both at most 65,536: tiles per view)
    uint32_t rec[RECS];
    uint32_t vbase[kEmitViews];    // the views' first tile ids
    uint32_t vtx[kEmitViews];      // and tiles per row
};

// tiles per row of the view holding global tile id `tile` (vbase, vtx: the LDS table of the first
// kEmitViews views)
__device__ __forceinline__ uint32_t emit_stride(const uint32_t* vbase, const uint32_t* vtx,
                                                const DevCam* __restrict__ cams, int B, uint32_t tile) {
    if (B > kEmitViews) return (uint32_t)cams[find_view(cams, B, tile)].tiles_x;
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (vbase[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return vtx[lo];
}

// Stages records [r0, r0 + cnt) of the depth order (cnt <= RECS); returns the chunk's pairs.
template <int RECS, int THREADS>
__device__ __forceinline__ uint32_t emit_stage(const uint32_t* __restrict__ sorted_rec,
                                               const uint2* __restrict__ sorted_rect,
                                               const DevCam* __restrict__ cams, int B, uint32_t r0, uint32_t cnt,
                                               EmitStage<RECS>& st, uint32_t* scan_tmp) {
    constexpr int kPer = RECS / THREADS;   // consecutive records per thread
    const uint32_t t = threadIdx.x;
    if ((int)t < B && t < (uint32_t)kEmitViews) {
        st.vbase[t] = cams[t].tile_base;
        st.vtx[t] = (uint32_t)cams[t].tiles_x;
    }
    uint2 rc[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t i = kPer * t + (uint32_t)k;
        rc[k] = make_uint2(0u, 0u);
        if (i < cnt) {
            rc[k] = sorted_rect[r0 + i];
            st.rec[i] = sorted_rec[r0 + i];
        }
    }
    __syncthreads();   // the view table
    uint32_t c[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t i = kPer * t + (uint32_t)k;
        c[k] = 0u;
        if (i < cnt) {
            c[k] = rect_tiles(rc[k]);
            st.base[i] = rc[k].x;
            st.ws[i] = ((rc[k].y & 0xffffu) - 1u) | ((emit_stride(st.vbase, st.vtx, cams, B, rc[k].x) - 1u) << 16);
        }
        sum += c[k];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan<THREADS>(sum, scan_tmp, &total);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        st.off[kPer * t + (uint32_t)k] = ex;
        ex += c[k];
    }
    if (t == 0) st.off[RECS] = total;
    __syncthreads();
    return total;
}

// the staged record holding pair j of the chunk: the last one whose prefix is <= j (records
// without pairs are passed over); a fixed number of steps, so that searches of several pairs
// interleave
template <int RECS>
__device__ __forceinline__ uint32_t emit_find(const EmitStage<RECS>& st, uint32_t cnt, uint32_t j) {
    uint32_t k = 0;
#pragma unroll
    for (uint32_t step = RECS / 2; step > 0; step >>= 1)
        if (k + step < cnt && st.off[k + step] <= j) k += step;
    return k;
}


// Walks the pairs of the staged chunk from pair j on, row-major over each rectangle.
template <bool REC, int RECS>
struct EmitWalk {
    uint32_t k, w, stride, left, col, rowkey, rec;
    __device__ __forceinline__ void start(const EmitStage<RECS>& st, uint32_t cnt, uint32_t j) {
        k = emit_find(st, cnt, j);
        if (REC) rec = st.rec[k];
        const uint32_t ws = st.ws[k];
        w = (ws & 0xffffu) + 1u;
        stride = (ws >> 16) + 1u;
        left = st.off[k + 1] - j;
        const uint32_t t = j - st.off[k];
        // t < 65536 (tiles per view), so (t + 0.5) / w in float32 is never within rounding of an integer
        const uint32_t row = (uint32_t)floorf(((float)t + 0.5f) * __builtin_amdgcn_rcpf((float)w));
        col = t - row * w;
        rowkey = st.base[k] + row * stride;
    }
    __device__ __forceinline__ uint32_t key() const { return rowkey + col; }
    // to the next pair; the caller knows there is one
    __device__ __forceinline__ void next(const EmitStage<RECS>& st) {
        if (--left == 0) {
            // the next record: all its fields in one round trip to LDS (records without pairs,
            // which the loop passes over, are rare)
            ++k;
            uint32_t o0 = st.off[k], o1 = st.off[k + 1];
            uint32_t nb = st.base[k], nws = st.ws[k], nr = REC ? st.rec[k] : 0u;
            while (o1 == o0) {
                ++k;
                o1 = st.off[k + 1];
                nb = st.base[k];
                nws = st.ws[k];
                if (REC) nr = st.rec[k];
            }
            rec = nr;
            w = (nws & 0xffffu) + 1u;
            stride = (nws >> 16) + 1u;
            left = o1 - o0;
            rowkey = nb;
            col = 0;
        } else if (++col == w) {
            col = 0;
            rowkey += stride;
        }
    }
};

// The digit counts of the chunk's pairs, without generating them: a row of a record's tile
// rectangle is a run of consecutive tile ids, so its digits (the low bits of the ids) are a cyclic
// run of consecutive digits. Each thread takes whole records and adds each row to a difference
// array over the digits (a run as long as the digit range adds to every digit once); a scan of
// the differences gives the counts.
template <int RECS>
__global__ void __launch_bounds__(kSortThreads) k_emit_upsweep(const uint2* __restrict__ sorted_rect,
                                                               const DevCam* __restrict__ cams, int B, uint32_t n,
                                                               const uint32_t* __restrict__ n_dev, uint32_t mask,
                                                               uint32_t chunks, uint32_t* __restrict__ counts) {
    __shared__ uint32_t vbase[kEmitViews], vtx[kEmitViews];
    __shared__ int diff[kRadix + 1];
    __shared__ uint32_t scan_tmp[kRadix];
    __shared__ uint32_t full;
    const uint32_t t = threadIdx.x;
    diff[t] = 0;
    if (t == 0) {
        diff[kRadix] = 0;
        full = 0u;
    }
    if ((int)t < B && t < (uint32_t)kEmitViews) {
        vbase[t] = cams[t].tile_base;
        vtx[t] = (uint32_t)cams[t].tiles_x;
    }
    n = (uint32_t)count_of(n, n_dev);
    const uint32_t r0 = blockIdx.x * RECS;
    const uint32_t cnt = r0 < n ? min(n - r0, (uint32_t)RECS) : 0u;
    const uint32_t R = mask + 1u;   // digits of the pass (a power of two)
    __syncthreads();
    uint32_t cycles = 0;   // whole runs through all R digits
    for (uint32_t i = t; i < cnt; i += kSortThreads) {
        const uint2 rc = sorted_rect[r0 + i];
        const uint32_t w = rc.y & 0xffffu, h = rc.y >> 16;
        if (w == 0u || h == 0u) continue;
        const uint32_t stride = emit_stride(vbase, vtx, cams, B, rc.x);
        cycles += h * (w / R);
        const uint32_t m = w & mask;   // the partial run of each row
        if (m == 0u) continue;
        for (uint32_t row = 0; row < h; ++row) {
            const uint32_t d0 = (rc.x + row * stride) & mask, e = d0 + m;
            atomicAdd(&diff[d0], 1);
            if (e <= R) {
                atomicAdd(&diff[e], -1);
            } else {
                atomicAdd(&diff[0], 1);
                atomicAdd(&diff[e - R], -1);
            }
        }
    }
    if (cycles) atomicAdd(&full, cycles);
    __syncthreads();
    uint32_t total;
    const uint32_t v = t < R ? (uint32_t)diff[t] : 0u;
    const uint32_t c = block_exclusive_scan_256(v, scan_tmp, &total) + v + full;   // inclusive
    if (t <= mask) counts[(size_t)t * chunks + blockIdx.x] = c;
}

template <int RECS, typename KT>
__global__ void __launch_bounds__(kEmitThreads) k_emit_downsweep(
    const uint32_t* __restrict__ sorted_rec, const uint2* __restrict__ sorted_rect, const DevCam* __restrict__ cams,
    int B, uint32_t n, const uint32_t* __restrict__ n_dev, uint32_t mask, uint32_t chunks,
    const uint32_t* __restrict__ offsets,
    uint32_t K, const uint32_t* __restrict__ K_dev, KT* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
    // 16-bit tile ids: a pair is staged as one word, tile id << 10 | the record's index in the
    // chunk (RECS <= 1024), and its record id looked up at write-out; half the LDS of a key and a
    // value word, so four workgroups share a CU instead of three
    constexpr bool PACK = sizeof(KT) == 2;
    static_assert(!PACK || RECS <= 1024, "packed pairs hold a 10-bit record index");
    __shared__ EmitStage<RECS> st;
    // per wavefront and digit: its items in the batch, then their offset (at most kEmitBatch)
    __shared__ uint16_t wcount[kEmitWaves][kRadix];
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t gbase[kRadix];
    __shared__ uint32_t scan_tmp[kRadix];
    // the lane-major pairs of each wavefront, then (after the ranking) the batch in digit order
    __shared__ uint32_t skey[kEmitStageWords];
    __shared__ uint32_t sval[PACK ? 1 : kEmitStageWords];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nbits = 32 - __builtin_clz(mask | 1u);   // bits of this pass's digit
    const int kshift = PACK ? 10 : 0;   // staged word >> kshift = tile id
    n = (uint32_t)count_of(n, n_dev);
    K = (uint32_t)count_of(K, K_dev);
    const uint32_t r0 = blockIdx.x * RECS;
    if (r0 >= n) return;
    const uint32_t cnt = min(n - r0, (uint32_t)RECS);
    if (threadIdx.x < kRadix)
        gbase[threadIdx.x] = threadIdx.x <= mask ? offsets[(size_t)threadIdx.x * chunks + blockIdx.x] : 0u;
    const uint32_t total = emit_stage<RECS, kEmitThreads>(sorted_rec, sorted_rect, cams, B, r0, cnt, st, scan_tmp);
    for (uint32_t b0 = 0; b0 < total; b0 += kEmitBatch) {
        const uint32_t bn = min(total - b0, (uint32_t)kEmitBatch);
        for (int i = threadIdx.x; i < kEmitWaves * kRadix; i += kEmitThreads) (&wcount[0][0])[i] = 0u;
        __syncthreads();
        const uint32_t wbase = (uint32_t)wave * kEmitRounds * 64u;
        uint32_t key[kEmitRounds], val[kEmitRounds], rank[kEmitRounds];
        {
            // lane l walks this wavefront's pairs R l .. R l + R - 1 (R = kEmitRounds; one search per lane) ...
            uint32_t* tk = skey + wave * 64 * kEmitPad + lane * kEmitPad;
            uint32_t* tv = sval + (PACK ? 0 : wave * 64 * kEmitPad + lane * kEmitPad);
            const uint32_t j0 = wbase + (uint32_t)lane * kEmitRounds;
            if (j0 < bn) {
                EmitWalk<!PACK, RECS> wk;
                wk.start(st, cnt, b0 + j0);
                const uint32_t m = min((uint32_t)kEmitRounds, bn - j0);
                for (uint32_t i = 0;;) {
                    if (PACK) {
                        tk[i] = (wk.key() << 10) | wk.k;
                    } else {
                        tk[i] = wk.key();
                        tv[i] = wk.rec;
                    }
                    if (++i == m) break;
                    wk.next(st);
                }
            }
            wave_lds_sync();
            // ... and round r takes pairs 64 r .. 64 r + 63 of the wavefront
#pragma unroll
            for (int r = 0; r < kEmitRounds; ++r) {
                const uint32_t p = (uint32_t)r * 64u + (uint32_t)lane;
                const uint32_t at = (uint32_t)wave * 64u * kEmitPad + (p / kEmitRounds) * kEmitPad + p % kEmitRounds;
                key[r] = skey[at];
                val[r] = PACK ? 0u : sval[at];
            }
        }
        // (the staging below reuses skey and sval after the barrier that follows the ranking)
#pragma unroll
        for (int r = 0; r < kEmitRounds; ++r) {
            rank[r] = 0u;
            if (wbase + (uint32_t)r * 64u >= bn) continue;   // uniform over the wavefront
            const uint32_t j = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            const bool valid = j < bn;
            const uint32_t d = (key[r] >> kshift) & mask;
            const uint64_t peers = digit_peers(d, valid, nbits);
            const uint32_t below = (uint32_t)rank_below(peers);
            const uint32_t before = wcount[wave][d];
            rank[r] = before + below;
            wave_lds_sync();
            if (valid && below == 0) wcount[wave][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
            wave_lds_sync();
        }
        __syncthreads();
        uint32_t run = 0;   // this batch's items of digit threadIdx.x (threads past the digits: 0)
        {
            const int d = threadIdx.x;
            if (d < kRadix) {
#pragma unroll
                for (int w = 0; w < kEmitWaves; ++w) {
                    const uint32_t c = wcount[w][d];
                    wcount[w][d] = (uint16_t)run;
                    run += c;
                }
            }
            uint32_t tot;
            const uint32_t ex = block_exclusive_scan<kEmitThreads>(run, scan_tmp, &tot);
            if (d < kRadix) dstart[d] = ex;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kEmitRounds; ++r) {
            const uint32_t j = wbase + (uint32_t)r * 64u + (uint32_t)lane;
            if (j < bn) {
                const uint32_t d = (key[r] >> kshift) & mask;
                const uint32_t pos = dstart[d] + wcount[wave][d] + rank[r];
                skey[pos] = key[r];
                if (!PACK) sval[pos] = val[r];
            }
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < bn; j += kEmitThreads) {
            const uint32_t w = skey[j];
            const uint32_t k = w >> kshift;
            const uint32_t d = k & mask;
            const uint32_t dst = gbase[d] + (j - dstart[d]);
            if (dst < K) {   // the pair count the buffers were sized by
                keys_out[dst] = (KT)k;
                vals_out[dst] = PACK ? st.rec[w & 1023u] : sval[j];
            }
        }
        __syncthreads();
        if (threadIdx.x < kRadix) gbase[threadIdx.x] += run;
    }
}

// [start, end) of each global tile's run in the sorted pair keys, by binary search: a wavefront
// finds where tiles t0 .. t0 + 63 start (one search per lane) and writes the ranges of the first
// 63, the end of a run being the start of the next tile's
template <typename KT>
__global__ void __launch_bounds__(256) k_ranges_search(const KT* __restrict__ keys, uint32_t K,
                                                       const uint32_t* __restrict__ K_dev, uint32_t n_tiles,
                                                       uint2* __restrict__ ranges) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t t = (blockIdx.x * 4u + (threadIdx.x >> 6)) * 63u + lane;
    K = (uint32_t)count_of(K, K_dev);
    uint32_t lo = 0, hi = K;   // first index with keys[i] >= t
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if ((uint32_t)keys[mid] < t) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t next = (uint32_t)__shfl_down((int)lo, 1, 64);
    if (lane < 63u && t < n_tiles) ranges[t] = next > lo ? make_uint2(lo, next) : make_uint2(0u, 0u);
}

template <typename KT>
__global__ void k_export_keys(const KT* __restrict__ tile_keys, const uint32_t* __restrict__ vals,
                              const BlendRec* __restrict__ recs, const DevCam* __restrict__ cams, uint32_t K,
                              uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    const uint32_t r = vals[i];
    const BlendRec& rec = recs[r];
    const uint32_t local = (uint32_t)tile_keys[i] - cams[rec.view].tile_base;
    if (keys_out) keys_out[i] = ((uint64_t)rec.view << 48) | ((uint64_t)local << 32) | (uint64_t)rec.depth_bits;
    if (vals_out) vals_out[i] = rec.gid;
}

size_t emit_sort_scratch_bytes(size_t n_rec, size_t K) {
    const size_t chunks = std::max<size_t>(1, div_up(n_rec, kEmitRecs));
    return std::max(radix_scratch_bytes(K), align256(chunks * kRadix * sizeof(uint32_t)) +
                                                scan_scratch_bytes(chunks * kRadix));
}

void emit_pairs_first_pass(const uint32_t* sorted_rec, const uint2* sorted_rect, const DevCam* cams, int B,
                           size_t n_rec, const uint32_t* n_rec_dev, void* keys, bool key16, uint32_t* vals, size_t K,
                           const uint32_t* K_dev, int bits, void* scratch, hipStream_t s) {
    if (n_rec == 0 || K == 0) return;
    // records covering fewer than four tiles on average: chunks of twice the records
    const bool small_rects = K < 4 * (size_t)n_rec;
    const uint32_t first_mask = (1u << tile_first_bits(bits)) - 1u;
    const int recs = small_rects ? kEmitRecsSmall : kEmitRecs;
    const size_t chunks = div_up(n_rec, (size_t)recs);
    uint8_t* p = (uint8_t*)scratch;
    uint32_t* counts = (uint32_t*)p;
    p += align256(chunks * kRadix * sizeof(uint32_t));
    hipLaunchKernelGGL(small_rects ? k_emit_upsweep<kEmitRecsSmall> : k_emit_upsweep<kEmitRecs>,
                       dim3((unsigned)chunks), dim3(kSortThreads), 0, s, sorted_rect, cams, B, (uint32_t)n_rec,
                       n_rec_dev, first_mask, (uint32_t)chunks, counts);
    scan_exclusive_u32(counts, counts, chunks * ((size_t)first_mask + 1), nullptr, p, s, nullptr);
    if (key16)
        hipLaunchKernelGGL(
            (small_rects ? k_emit_downsweep<kEmitRecsSmall, uint16_t> : k_emit_downsweep<kEmitRecs, uint16_t>),
            dim3((unsigned)chunks), dim3(kEmitThreads), 0, s, sorted_rec, sorted_rect, cams, B, (uint32_t)n_rec,
            n_rec_dev, first_mask, (uint32_t)chunks, (const uint32_t*)counts, (uint32_t)K, K_dev, (uint16_t*)keys, vals);
    else
        hipLaunchKernelGGL(
            (small_rects ? k_emit_downsweep<kEmitRecsSmall, uint32_t> : k_emit_downsweep<kEmitRecs, uint32_t>),
            dim3((unsigned)chunks), dim3(kEmitThreads), 0, s, sorted_rec, sorted_rect, cams, B, (uint32_t)n_rec,
            n_rec_dev, first_mask, (uint32_t)chunks, (const uint32_t*)counts, (uint32_t)K, K_dev, (uint32_t*)keys, vals);
}

template <typename KT>
static int sort_pairs_rest_t(KT* keys[2], uint32_t* vals[2], size_t K, const uint32_t* K_dev, int bits, void* scratch,
                             hipStream_t s) {
    int cur = 0;
    if (K == 0) return cur;
    const int first = tile_first_bits(bits);
    if (first >= bits) return cur;
    const PassPlan pl = plan_passes(bits - first);
    for (int pass = 0; pass < pl.passes; ++pass) {
        radix_pass<KT>(keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1], K, K_dev, 0u, first + pl.dbits * pass,
                       pl.mask, scratch, s);
        cur ^= 1;
    }
    return cur;
}

int sort_pairs_rest(void* keys[2], bool key16, uint32_t* vals[2], size_t K, const uint32_t* K_dev, int bits,
                    void* scratch, hipStream_t s) {
    if (key16) {
        uint16_t* k[2] = {(uint16_t*)keys[0], (uint16_t*)keys[1]};
        return sort_pairs_rest_t<uint16_t>(k, vals, K, K_dev, bits, scratch, s);
    }
    uint32_t* k[2] = {(uint32_t*)keys[0], (uint32_t*)keys[1]};
    return sort_pairs_rest_t<uint32_t>(k, vals, K, K_dev, bits, scratch, s);
}

void launch_ranges(const void* keys, bool key16, uint32_t K, uint32_t n_tiles, uint2* ranges, hipStream_t s,
                   const uint32_t* K_dev) {
    if (!n_tiles) return;
    if (key16)
        hipLaunchKernelGGL(k_ranges_search<uint16_t>, dim3((n_tiles + 251) / 252), dim3(256), 0, s,
                           (const uint16_t*)keys, K, K_dev, n_tiles, ranges);
    else
        hipLaunchKernelGGL(k_ranges_search<uint32_t>, dim3((n_tiles + 251) / 252), dim3(256), 0, s,
                           (const uint32_t*)keys, K, K_dev, n_tiles, ranges);
}

void launch_export_keys(const void* tile_keys, bool key16, const uint32_t* vals, const BlendRec* recs,
                        const DevCam* cams, int B, uint32_t K, uint64_t* keys_out, uint32_t* vals_out,
                        hipStream_t s) {
    (void)B;
    if (!K) return;
    if (key16)
        hipLaunchKernelGGL(k_export_keys<uint16_t>, dim3((K + 255) / 256), dim3(256), 0, s,
                           (const uint16_t*)tile_keys, vals, recs, cams, K, keys_out, vals_out);
    else
        hipLaunchKernelGGL(k_export_keys<uint32_t>, dim3((K + 255) / 256), dim3(256), 0, s,
                           (const uint32_t*)tile_keys, vals, recs, cams, K, keys_out, vals_out);
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

// the same with 16-byte stores (p 16-byte aligned): four values per thread
__global__ void k_fill_u32x4_count(uint32_t* __restrict__ p, size_t n, const uint32_t* __restrict__ n_dev,
                                   uint32_t per, uint32_t v) {
    const size_t i = 4 * ((size_t)blockIdx.x * blockDim.x + threadIdx.x);
    const size_t total = (size_t)per * count_of(n, n_dev);
    if (i + 3 < total) {
        *reinterpret_cast<uint4*>(p + i) = make_uint4(v, v, v, v);
    } else {
        for (size_t j = i; j < total; ++j) p[j] = v;
    }
}

void fill_u32_count(uint32_t* p, size_t n, const uint32_t* n_dev, uint32_t per, uint32_t v, hipStream_t s) {
    if (!n || !per) return;
    if (((uintptr_t)p & 15u) == 0)
        hipLaunchKernelGGL(k_fill_u32x4_count, dim3((unsigned)div_up(n * per, 1024)), dim3(256), 0, s, p, n, n_dev,
                           per, v);
    else
        hipLaunchKernelGGL(k_fill_u32_count, dim3((unsigned)div_up(n * per, 256)), dim3(256), 0, s, p, n, n_dev, per,
                           v);
}

// Capacity mode: the records and pairs of this call against the buffers' capacities. Within them,
// eff = (V, K); beyond either, eff = (0, 0) and the overflow word is set, so every later kernel
// does no work and stays inside its buffers.
// Also: the depth keys of the records (key_range: min, ~max) must lie in the window
// [key_base, key_base + 2^key_bits) the depth sort of this call orders (bit 3 otherwise); the
// range is kept in range_out for the host.
__global__ void k_capacity_clamp(const unsigned long long* __restrict__ totals, uint64_t cap_v, uint64_t cap_k,
                                 uint32_t* __restrict__ eff, uint32_t* __restrict__ overflow,
                                 const uint32_t* __restrict__ key_range, uint32_t key_base, int key_bits,
                                 uint32_t* __restrict__ range_out) {
    const uint64_t V = totals[0], K = totals[1];
    uint32_t bits = V > cap_v || K > cap_k ? 1u : 0u;
    if (key_range) {
        const uint32_t kmin = key_range[0], kmax = ~key_range[1];
        range_out[0] = kmin;
        range_out[1] = key_range[1];
        if (V > 0 && key_bits < 32 && (kmin < key_base || ((kmax - key_base) >> key_bits) != 0u)) bits |= 8u;
    }
    eff[0] = bits ? 0u : (uint32_t)V;
    eff[1] = bits ? 0u : (uint32_t)K;
    overflow[0] = bits;
}

void launch_capacity_clamp(const uint64_t* totals, uint64_t cap_v, uint64_t cap_k, uint32_t* eff, uint32_t* overflow,
                           hipStream_t s, const uint32_t* key_range, uint32_t key_base, int key_bits,
                           uint32_t* range_out) {
    hipLaunchKernelGGL(k_capacity_clamp, dim3(1), dim3(1), 0, s, (const unsigned long long*)totals, cap_v, cap_k, eff,
                       overflow, key_range, key_base, key_bits, range_out);
}

}  // namespace mvgs
