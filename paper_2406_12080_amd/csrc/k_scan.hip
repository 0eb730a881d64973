// Device-wide exclusive scan of uint32 counts with a fixed grid (reduce, scan
// of the per-block partials, down-sweep), so that the element count may live
// in device memory and the launch sequence can be captured in a graph.
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;
constexpr int kItems = 4;

__device__ __forceinline__ uint32_t wave_inclusive(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan across a block of kT threads; *total receives the sum.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t x, uint32_t &total, uint32_t *s_w)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_inclusive(x);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kT / 64; ++k) {
        const uint32_t c = s_w[k];
        base += k < w ? c : 0u;
        tot += c;
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

__device__ __forceinline__ uint32_t count_of(uint32_t n_host, const uint32_t *n_dev)
{
    return n_dev ? min(*n_dev, n_host) : n_host;
}

__device__ __forceinline__ uint32_t load_in(const uint32_t *in, const uint32_t *idx, uint32_t i)
{
    return in[idx ? idx[i] : i];
}

// With idx, the gathered values in[idx[i]] are also stored to dense[i], so
// that the down-sweep reads them in order (one gather instead of two).
__global__ __launch_bounds__(kT) void k_scan_reduce(const uint32_t *__restrict__ in, const uint32_t *__restrict__ idx,
                                                    uint32_t n_host, const uint32_t *__restrict__ n_dev,
                                                    uint32_t *__restrict__ partial, uint32_t *__restrict__ dense)
{
    __shared__ uint32_t s_w[kT / 64];
    const uint32_t n = count_of(n_host, n_dev);
    const uint32_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const uint32_t b0 = min(n, blockIdx.x * chunk), b1 = min(n, b0 + chunk);
    uint32_t s = 0;
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += kT) {
        const uint32_t x = load_in(in, idx, i);
        if (dense) dense[i] = x;
        s += x;
    }
    uint32_t tot;
    block_exclusive(s, tot, s_w);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlocks) void k_scan_partials(uint32_t *__restrict__ partial,
                                                               uint32_t *__restrict__ total)
{
    __shared__ uint32_t s_w[kScanBlocks / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t x = partial[threadIdx.x];
    const uint32_t inc = wave_inclusive(x);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int k = 0; k < kScanBlocks / 64; ++k) {
        base += k < w ? s_w[k] : 0u;
        tot += s_w[k];
    }
    partial[threadIdx.x] = base + inc - x;
    if (threadIdx.x == 0 && total) *total = tot;
}

// May run in place (in == out): each thread reads its elements before it
// writes them, and no other thread touches them.
__global__ __launch_bounds__(kT) void k_scan_down(const uint32_t *in, const uint32_t *__restrict__ idx,
                                                  uint32_t n_host, const uint32_t *__restrict__ n_dev,
                                                  const uint32_t *__restrict__ partial, uint32_t *out)
{
    __shared__ uint32_t s_w[kT / 64];
    const uint32_t n = count_of(n_host, n_dev);
    const uint32_t chunk = (n + kScanBlocks - 1) / kScanBlocks;
    const uint32_t b0 = min(n, blockIdx.x * chunk), b1 = min(n, b0 + chunk);
    uint32_t run = partial[blockIdx.x];
    for (uint32_t base = b0; base < b1; base += kT * kItems) {
        uint32_t v[kItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t i = base + threadIdx.x * kItems + k;
            v[k] = i < b1 ? load_in(in, idx, i) : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t ex = block_exclusive(s, tot, s_w) + run;
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            const uint32_t i = base + threadIdx.x * kItems + k;
            if (i < b1) out[i] = ex;
            ex += v[k];
        }
        run += tot;
    }
}

}  // namespace

void launch_scan(const uint32_t *in, const uint32_t *idx, uint32_t n_host, const uint32_t *n_dev, uint32_t *out,
                 uint32_t *total, uint32_t *partial, hipStream_t st)
{
    // a gathered input is made dense in `out` by the first pass; the
    // down-sweep then scans `out` in place
    hipLaunchKernelGGL(k_scan_reduce, dim3(kScanBlocks), dim3(kT), 0, st, in, idx, n_host, n_dev, partial,
                       idx ? out : nullptr);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanBlocks), 0, st, partial, total);
    hipLaunchKernelGGL(k_scan_down, dim3(kScanBlocks), dim3(kT), 0, st, idx ? out : in, nullptr, n_host, n_dev,
                       partial, out);
}

}  // namespace hgs
