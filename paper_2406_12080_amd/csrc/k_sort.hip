// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits,
// LDS-staged.  A fixed grid of G blocks each owns one contiguous chunk of the
// input (so the element count may be a device value and the launches can be
// captured in a graph):
//   hist    : per-block digit histogram -> hist[digit * G + block]
//   scan    : exclusive scan of hist (digit-major) = first output slot of
//             every (digit, block)
//   scatter : each block walks its chunk in tiles of 2048 keys, ranks keys
//             stably inside the tile (64-lane digit match from 8 ballots,
//             per-wave running counts in LDS), regroups the tile by digit in
//             LDS, and writes runs of equal digits contiguously.
// Ranking order inside a tile is (wave, item, lane) = input order, so equal
// keys keep their input order.
// Segmented mode (one segment per view): k_seg_plan gives every segment its
// own blocks, and lays the histogram out as (segment, digit, block), so that
// the one exclusive scan over it places each segment's output exactly over
// its input range.
#include <algorithm>

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;
constexpr int kWaves = kT / 64;
constexpr int kItems = 8;
constexpr int kTile = kT * kItems;
constexpr int kRadix = 256;

__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ void chunk_of(uint32_t n, int G, uint32_t &b0, uint32_t &b1)
{
    const uint32_t chunk = (n + G - 1) / G;
    b0 = min(n, blockIdx.x * chunk);
    b1 = min(n, b0 + chunk);
}

// The work of this block: its element range, histogram slots and key base
// (uniform chunks of [0, n) without a plan).  False: no work.
__device__ __forceinline__ bool block_work(const SortBlock *plan, uint32_t n, int G, uint32_t &b0, uint32_t &b1,
                                           uint32_t &hbase, uint32_t &hstride, uint32_t &kbase)
{
    if (plan) {
        const SortBlock p = plan[blockIdx.x];
        b0 = p.b0;
        b1 = p.b1;
        hbase = p.hbase;
        hstride = p.hstride;
        kbase = p.kbase;
        return hstride != 0;
    }
    chunk_of(n, G, b0, b1);
    hbase = blockIdx.x;
    hstride = (uint32_t)G;
    kbase = 0;
    return true;
}

// Plan of a segmented sort over G blocks: segment i of [bounds[i],
// bounds[i + 1]) (clamped to n) gets ceil(size / C) blocks for one chunk size
// C chosen so that the blocks of all segments fit in G.  One thread per
// segment; *hist_n receives the histogram length 256 x (blocks used).
__global__ __launch_bounds__(kMaxViews) void k_seg_plan(const uint32_t *__restrict__ bounds, int nseg,
                                                        const uint32_t *__restrict__ kbase, uint32_t cap,
                                                        const uint32_t *__restrict__ n_dev, int G,
                                                        SortBlock *__restrict__ plan, uint32_t *__restrict__ hist_n)
{
    __shared__ uint32_t s_w[kMaxViews / 64];
    const uint32_t n = min(*n_dev, cap);
    const int i = threadIdx.x;
    uint32_t lo = 0, hi = 0;
    if (i < nseg) {
        lo = min(bounds[i], n);
        hi = min(max(bounds[i + 1], lo), n);
    }
    const uint32_t chunk = max((uint32_t)kTile, (n + (uint32_t)(G - nseg) - 1) / (uint32_t)(G - nseg));
    const uint32_t nb = (hi - lo + chunk - 1) / chunk;
    // exclusive scan of the block counts over the segments
    const int lane = i & 63, w = i >> 6;
    uint32_t inc = nb;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t first = inc - nb, used = 0;
    for (int k = 0; k < kMaxViews / 64; ++k) {
        first += k < w ? s_w[k] : 0u;
        used += s_w[k];
    }
    if (used > (uint32_t)G) {  // cannot happen for ascending bounds; never write past the plan
        for (uint32_t b = (uint32_t)i; b < (uint32_t)G; b += kMaxViews) {
            SortBlock p = {};
            plan[b] = p;
        }
        if (i == 0) *hist_n = 0u;
        return;
    }
    for (uint32_t j = 0; j < nb; ++j) {
        SortBlock p;
        p.b0 = lo + j * chunk;
        p.b1 = min(hi, p.b0 + chunk);
        p.hbase = 256u * first + j;
        p.hstride = nb;
        p.kbase = kbase ? kbase[i] : 0u;
        p.pad[0] = p.pad[1] = p.pad[2] = 0u;
        plan[first + j] = p;
    }
    __syncthreads();
    for (uint32_t b = used + (uint32_t)i; b < (uint32_t)G; b += kMaxViews) {
        SortBlock p = {};
        plan[b] = p;  // no work
    }
    if (i == 0) *hist_n = 256u * used;
}

__global__ __launch_bounds__(kT) void k_rs_hist(const uint32_t *__restrict__ keys, uint32_t cap,
                                                const uint32_t *__restrict__ n_dev, int shift,
                                                uint32_t *__restrict__ hist, int G,
                                                const SortBlock *__restrict__ plan)
{
    __shared__ uint32_t s_h[kRadix];
    const uint32_t n = min(*n_dev, cap);
    uint32_t b0, b1, hbase, hstride, kbase;
    if (!block_work(plan, n, G, b0, b1, hbase, hstride, kbase)) return;
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (uint32_t base = b0; base < b1; base += kTile) {
        uint32_t d[kItems];
#pragma unroll
        for (int it = 0; it < kItems; ++it) {  // all loads of the tile in flight at once
            const uint32_t i = base + (uint32_t)(w * 64 * kItems + it * 64 + lane);
            d[it] = i < b1 ? ((keys[i] - kbase) >> shift) & 0xFFu : 0x100u;
        }
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const bool valid = d[it] < 0x100u;
            const uint64_t peers = match_digit(d[it] & 0xFFu, valid);
            if (valid && (peers & lt) == 0) atomicAdd(&s_h[d[it]], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    hist[hbase + threadIdx.x * hstride] = s_h[threadIdx.x];
}

__global__ __launch_bounds__(kT) void k_rs_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                   uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                   uint32_t cap, const uint32_t *__restrict__ n_dev, int shift,
                                                   const uint32_t *__restrict__ offsets, int G,
                                                   const SortBlock *__restrict__ plan)
{
    __shared__ uint32_t s_keys[kTile];
    __shared__ uint32_t s_vals[kTile];
    __shared__ uint32_t s_wcnt[kWaves][kRadix];
    __shared__ uint32_t s_run[kRadix];
    __shared__ uint32_t s_start[kRadix];
    __shared__ uint32_t s_tot[kRadix];
    __shared__ uint32_t s_w[kWaves];

    const uint32_t n = min(*n_dev, cap);
    uint32_t b0, b1, hbase, hstride, kbase;
    if (!block_work(plan, n, G, b0, b1, hbase, hstride, kbase)) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t lt = lanemask_lt();
    s_run[threadIdx.x] = offsets[hbase + threadIdx.x * hstride];

    for (uint32_t base = b0; base < b1; base += kTile) {
#pragma unroll
        for (int k = 0; k < kWaves; ++k) s_wcnt[k][threadIdx.x] = 0;
        __syncthreads();
        uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            const uint32_t i = base + (uint32_t)(w * 64 * kItems + it * 64 + lane);
            const bool valid = i < b1;
            key[it] = valid ? kin[i] : 0u;
            val[it] = valid ? vin[i] : 0u;
            const uint32_t d = ((key[it] - kbase) >> shift) & 0xFFu;
            const uint64_t peers = match_digit(d, valid);
            const uint32_t before = s_wcnt[w][d];
            rank[it] = before + (uint32_t)__popcll(peers & lt);
            if (valid && (peers & lt) == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
            if (!valid) rank[it] = 0xFFFFFFFFu;
        }
        __syncthreads();
        // per digit: wave offsets and tile total
        {
            const int d = threadIdx.x;
            uint32_t acc = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) {
                const uint32_t c = s_wcnt[k][d];
                s_wcnt[k][d] = acc;
                acc += c;
            }
            s_tot[d] = acc;
            // exclusive scan of tile totals over digits (one digit per thread)
            uint32_t x = acc;
            uint32_t inc = x;
#pragma unroll
            for (int dd = 1; dd < 64; dd <<= 1) {
                const uint32_t y = __shfl_up(inc, dd, 64);
                if (lane >= dd) inc += y;
            }
            if (lane == 63) s_w[w] = inc;
            __syncthreads();
            uint32_t wb = 0;
#pragma unroll
            for (int k = 0; k < kWaves; ++k) wb += k < w ? s_w[k] : 0u;
            s_start[d] = wb + inc - x;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kItems; ++it) {
            if (rank[it] == 0xFFFFFFFFu) continue;
            const uint32_t d = ((key[it] - kbase) >> shift) & 0xFFu;
            const uint32_t lp = s_start[d] + s_wcnt[w][d] + rank[it];
            s_keys[lp] = key[it];
            s_vals[lp] = val[it];
        }
        __syncthreads();
        const uint32_t cnt = min((uint32_t)kTile, b1 - base);
        for (uint32_t j = threadIdx.x; j < cnt; j += kT) {
            const uint32_t k2 = s_keys[j];
            const uint32_t d = ((k2 - kbase) >> shift) & 0xFFu;
            const uint32_t g = s_run[d] + (j - s_start[d]);
            kout[g] = k2;
            vout[g] = s_vals[j];
        }
        __syncthreads();
        s_run[threadIdx.x] += s_tot[threadIdx.x];
        __syncthreads();
    }
}

}  // namespace

// Sorts (keys, vals) over bits [0, bits) with ceil(bits / 8) passes that
// ping-pong between (keys, vals) and the scratch pair.  Returns true when the
// pass count is odd, i.e. the sorted result is in (s.k2, s.v2).
bool launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t cap, const uint32_t *n_dev, int bits,
                       const SortScratch &s, hipStream_t st, const uint32_t *seg_bounds, int nseg,
                       const uint32_t *seg_kbase)
{
    if (cap == 0 || bits <= 0) return false;
    const int passes = (bits + 7) / 8;
    // blocks of >= 4 tiles each, up to kSortBlocksMax: enough waves in flight
    // to cover the memory latency of the digit passes
    const uint32_t want = std::max<uint32_t>(1u, (cap + 4 * kTile - 1) / (4 * kTile));
    int G = (int)std::min<uint32_t>(kSortBlocksMax, want);
    const SortBlock *plan = nullptr;
    const uint32_t *hist_n = nullptr;
    if (seg_bounds) {
        G = std::min(kSortBlocksMax, std::max(G, 2 * nseg + 1));
        hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(kMaxViews), 0, st, seg_bounds, nseg, seg_kbase, cap, n_dev, G,
                           s.plan, s.total + 1);
        plan = s.plan;
        hist_n = s.total + 1;
    }
    uint32_t *ki = keys, *vi = vals, *ko = s.k2, *vo = s.v2;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * 8;
        hipLaunchKernelGGL(k_rs_hist, dim3(G), dim3(kT), 0, st, ki, cap, n_dev, shift, s.hist, G, plan);
        launch_scan(s.hist, nullptr, (uint32_t)(kRadix * G), hist_n, s.hist_scan, s.total, s.partial, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3(G), dim3(kT), 0, st, ki, vi, ko, vo, cap, n_dev, shift, s.hist_scan,
                           G, plan);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    return (passes & 1) != 0;
}

}  // namespace hgs
