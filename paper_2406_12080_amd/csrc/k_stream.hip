// Out-of-core rendering (Sec. 6.3: the cut is updated as the camera moves,
// nodes are transferred to the GPU from CPU RAM as it needs them, and a
// cleanup runs every so many frames).  The topology and boxes stay on the
// device (the cut reads every node); the Gaussians' 59 parameters stay in
// pinned host memory, and a device cache of fixed capacity holds those of
// the nodes the recent cuts used.  slot[node] is the node's cache slot (-1:
// not resident, -2: claimed by this frame's transfer).  Per render:
//   tick  : the frame counter advances;
//   claim : every cut entry's node and its parent (the interpolation reads
//           both) are stamped with the frame when resident, else claimed by
//           one compare-and-swap and appended to the frame's request list;
//   fetch : each request takes a free slot from the top of the free stack
//           and one wave copies the node's record from host memory (59
//           floats over PCIe/xGMI) into it; requests beyond the free slots
//           are released and flag an overflow (those splats are skipped);
//   pop   : the free stack shrinks by the slots taken.
// cleanup (on request): slots unused for more than max_age frames are freed.
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;

__global__ void k_stream_tick(StreamDev s)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *s.frame += 1;
        *s.req_count = 0;
        *s.overflow = 0;
    }
}

__device__ __forceinline__ void claim_one(const StreamDev &s, uint32_t x, uint32_t frame)
{
    const int32_t cur = s.slot[x];
    if (cur >= 0) {
        s.last_used[cur] = frame;
        return;
    }
    if (cur == -1 && atomicCAS(&s.slot[x], -1, -2) == -1) {
        const uint32_t r = atomicAdd(s.req_count, 1u);
        if (r < s.req_cap) {
            s.req[r] = x;
        } else {
            s.slot[x] = -1;  // no room to record it: released, and the frame overflows
            atomicOr(s.overflow, 1u);
        }
    }
}

__global__ __launch_bounds__(kT) void k_stream_claim(const uint32_t *__restrict__ pinfo,
                                                     const int32_t *__restrict__ cut_ids,
                                                     const uint32_t *__restrict__ cut_total, uint32_t cap,
                                                     StreamDev s)
{
    const uint32_t n = min(*cut_total, cap);
    const uint32_t frame = *s.frame;
    for (uint32_t k = blockIdx.x * kT + threadIdx.x; k < n; k += gridDim.x * kT) {
        const uint32_t node = (uint32_t)cut_ids[k];
        claim_one(s, node, frame);
        const uint32_t par = pinfo[node] & ~kLeafBit;
        if (par != kRootParent) claim_one(s, par, frame);
    }
}

// One wave per request: lanes 0..58 copy the record's floats (mean 3, scale
// 3, rotation 4, opacity 1, SH 48).
__global__ __launch_bounds__(kT) void k_stream_fetch(StreamDev s, StreamParams host, StreamParams cache)
{
    const uint32_t nreq = min(*s.req_count, s.req_cap);
    const uint32_t nfree = *s.free_top;
    const uint32_t frame = *s.frame;
    const int lane = threadIdx.x & 63;
    for (uint32_t r = (blockIdx.x * kT + threadIdx.x) >> 6; r < nreq; r += (gridDim.x * kT) >> 6) {
        const uint32_t x = s.req[r];
        if (r >= nfree) {
            if (lane == 0) {
                s.slot[x] = -1;
                atomicOr(s.overflow, 1u);
            }
            continue;
        }
        const uint32_t d = s.free_stack[nfree - 1 - r];
        const size_t X = x, D = d;
        if (lane < 3) cache.mean[3 * D + lane] = host.mean[3 * X + lane];
        else if (lane < 6) cache.scale[3 * D + lane - 3] = host.scale[3 * X + lane - 3];
        else if (lane < 10) cache.rot[4 * D + lane - 6] = host.rot[4 * X + lane - 6];
        else if (lane == 10) cache.opacity[D] = host.opacity[X];
        else if (lane < 59) cache.sh[48 * D + lane - 11] = host.sh[48 * X + lane - 11];
        // the copy is read by later kernels only (preprocess), after this one ends
        if (lane == 0) {
            s.node_in_slot[d] = (int32_t)x;
            s.last_used[d] = frame;
            s.slot[x] = (int32_t)d;
        }
    }
}

__global__ void k_stream_pop(StreamDev s)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const uint32_t nreq = min(*s.req_count, s.req_cap);
        const uint32_t nfree = *s.free_top;
        const uint32_t taken = nreq < nfree ? nreq : nfree;
        *s.free_top = nfree - taken;
        *s.transferred += taken;
    }
}

__global__ __launch_bounds__(kT) void k_stream_cleanup(StreamDev s, uint32_t max_age)
{
    const uint32_t frame = *s.frame;
    for (uint32_t d = blockIdx.x * kT + threadIdx.x; d < s.cap; d += gridDim.x * kT) {
        const int32_t x = s.node_in_slot[d];
        if (x < 0 || frame - s.last_used[d] <= max_age) continue;
        s.slot[x] = -1;
        s.node_in_slot[d] = -1;
        const uint32_t i = atomicAdd(s.free_top, 1u);
        s.free_stack[i] = d;
    }
}

__global__ __launch_bounds__(kT) void k_stream_init(StreamDev s, int64_t n_nodes)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n_nodes; i += (int64_t)gridDim.x * kT)
        s.slot[i] = -1;
    for (uint32_t d = blockIdx.x * kT + threadIdx.x; d < s.cap; d += gridDim.x * kT) {
        s.node_in_slot[d] = -1;
        s.last_used[d] = 0;
        s.free_stack[d] = s.cap - 1 - d;  // pops hand out slots 0, 1, 2, ...
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *s.free_top = s.cap;
        *s.frame = 0;
        *s.req_count = 0;
        *s.overflow = 0;
        *s.transferred = 0;
    }
}

}  // namespace

void launch_stream_init(const StreamDev &s, int64_t n_nodes, hipStream_t st)
{
    hipLaunchKernelGGL(k_stream_init, dim3(2048), dim3(kT), 0, st, s, n_nodes);
}

void launch_stream_frame(const StreamDev &s, const uint32_t *pinfo, const int32_t *cut_ids,
                         const uint32_t *cut_total, uint32_t cap, const StreamParams &host,
                         const StreamParams &cache, hipStream_t st)
{
    hipLaunchKernelGGL(k_stream_tick, dim3(1), dim3(64), 0, st, s);
    hipLaunchKernelGGL(k_stream_claim, dim3(2048), dim3(kT), 0, st, pinfo, cut_ids, cut_total, cap, s);
    hipLaunchKernelGGL(k_stream_fetch, dim3(2048), dim3(kT), 0, st, s, host, cache);
    hipLaunchKernelGGL(k_stream_pop, dim3(1), dim3(64), 0, st, s);
}

void launch_stream_cleanup(const StreamDev &s, uint32_t max_age, hipStream_t st)
{
    hipLaunchKernelGGL(k_stream_cleanup, dim3(1024), dim3(kT), 0, st, s, max_age);
}

}  // namespace hgs
