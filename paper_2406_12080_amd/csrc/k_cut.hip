// Level-of-detail cut (Sec. 4.2, "Hierarchy Cut Selection and Level
// Switching") and the interpolation weight of Eq. (t_interp).
//
// A node n meets the target granularity tau when it is a leaf or when the
// projected size of the largest dimension of its leaf bounding box,
// eps(n) = f L(n) / d(n) (d = distance from the eye to the box), is at most
// tau.  The cut is every node that meets it while its parent does not: a
// constant-time test per node, run here as a coalesced sweep over the
// structure-of-arrays boxes with one thread per node and every view handled
// by the thread that holds the node (the node's box is read once per batch
// of views).  Selected nodes are compacted in ascending id order with a
// 64-lane ballot bitmask per wave, a per-block count, one exclusive scan over
// (view, block), and an emit pass that writes ids and weights.  Each lane
// evaluates F(n) = leaf or eps(n) <= tau for its node and for its node's
// parent (parents of neighbouring nodes are neighbours: cached boxes).
//
// The selection is defined by eps evaluated in FP64 with contraction
// disabled, from the FP32 stored boxes, so that it does not depend on FP32
// rounding; t is evaluated the same way.  The sweep first decides each test
// in FP32 as L^2 against (tau / f)^2 d^2 and falls back to the FP64
// evaluation only when the two sides are within a relative kCutMargin, far
// wider than the FP32 rounding error of either side (a few units in the last
// place), so both evaluations always agree.
#include "hgs_internal.h"

namespace hgs {

__device__ __forceinline__ double granularity(const float b[6], const DevView &V)
{
#pragma clang fp contract(off)
    double L = 0.0;
    double dd[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double lo = b[k], hi = b[3 + k];
        const double ext = hi - lo;
        if (ext > L) L = ext;
        const double e = V.eye[k];
        const double c = e < lo ? lo : (e > hi ? hi : e);
        dd[k] = e - c;
    }
    const double d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
    const double d = sqrt(d2);
    if (d == 0.0) return __builtin_inf();
    const double f = V.fx > V.fy ? (double)V.fx : (double)V.fy;
    return (f * L) / d;
}

// The FP32 prefilter of eps(box) <= tau, written L^2 <= k d^2 with the
// per-view constant k = (tau / f)^2, as lane masks of one wave: `yes` where
// L^2 < k (1 - kCutMargin) d^2, `no` where L^2 > k (1 + kCutMargin) d^2, and
// neither inside that band or where a square is too small to be accurate in
// FP32 (d^2 < 1e-18, which includes the eye inside the box, or a non-zero
// L^2 < 1e-30).  Either side carries at most a few units in the last place
// of rounding, far inside the band, so a decision taken here is the FP64
// one.  Lok: the lanes whose L^2 is usable.
struct CutTest {
    uint64_t yes, no;
};

// (wave-wide float compares straight to lane masks)
constexpr int kFcmpOgt = 2, kFcmpOge = 3, kFcmpOlt = 4;

__device__ __forceinline__ CutTest meets_tau_f32(const float b[6], float L2, uint64_t Lok, const DevView &V)
{
    const float ex = V.eye[0], ey = V.eye[1], ez = V.eye[2];
    const float dx = ex - __builtin_amdgcn_fmed3f(ex, b[0], b[3]);  // eye minus its clamp to the box
    const float dy = ey - __builtin_amdgcn_fmed3f(ey, b[1], b[4]);
    const float dz = ez - __builtin_amdgcn_fmed3f(ez, b[2], b[5]);
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const uint64_t ok = Lok & __builtin_amdgcn_fcmpf(d2, 1e-18f, kFcmpOge);
    CutTest r;
    r.yes = ok & __builtin_amdgcn_fcmpf(L2, V.cut_klo * d2, kFcmpOlt);
    r.no = ok & __builtin_amdgcn_fcmpf(L2, V.cut_khi * d2, kFcmpOgt);
    return r;
}

__device__ __forceinline__ void load_box(const DevHier &h, int64_t i, float b[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) b[k] = h.box[k * h.n + i];
}

// The cut in one sweep: each lane tests its node and its node's parent for
// every view (the FP32 prefilter is a few instructions per test, so testing a
// parent once per child costs less than a second sweep over stored bits) and
// keeps F(n) and not F(parent).  Writes the cut bit masks and per-block
// counts.
__global__ __launch_bounds__(kCutThreads) void k_cut_onepass(DevHier h, const DevView *__restrict__ views, int nv,
                                                             uint64_t *__restrict__ masks,
                                                             uint32_t *__restrict__ block_counts, int nblocks)
{
    __shared__ uint32_t s_cnt[kMaxViews];
    for (int v = threadIdx.x; v < nv; v += kCutThreads) s_cnt[v] = 0;
    __syncthreads();
    const int64_t n = h.n;
    const int64_t words = (n + 63) >> 6;
    const int lane = threadIdx.x & 63;
#pragma unroll 1
    for (int it = 0; it < kCutItems; ++it) {
        const int64_t i0 = (int64_t)blockIdx.x * kCutBlock + it * kCutThreads + (threadIdx.x & ~63);
        const int64_t i = i0 + lane;
        const bool valid = i < n;
        if (i0 >= n) break;
        float b[6] = {0, 0, 0, 0, 0, 0}, pb[6] = {0, 0, 0, 0, 0, 0};
        bool leaf = true, root = true;
        if (valid) {
            const uint32_t pi = h.pinfo[i];
            leaf = (pi & kLeafBit) != 0;
            const uint32_t par = pi & ~kLeafBit;
            root = par == kRootParent;
            load_box(h, i, b);
            if (!root) load_box(h, par, pb);
        }
        // leaves (and the padding past n) always meet tau; the root and the
        // padding have no parent that meets it
        const uint64_t leaves = __ballot(leaf), no_parent = __ballot(root), live = __ballot(valid);
        float L = 0.0f, Lp = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            L = fmaxf(L, b[3 + k] - b[k]);
            Lp = fmaxf(Lp, pb[3 + k] - pb[k]);
        }
        const float L2 = L * L, Lp2 = Lp * Lp;
        const uint64_t Lok = __ballot(L2 == 0.0f || L2 >= 1e-30f), Lpok = __ballot(Lp2 == 0.0f || Lp2 >= 1e-30f);
#pragma unroll 1
        for (int v0 = 0; v0 < nv; v0 += 64) {  // up to 64 views gathered on lanes
            uint64_t word = 0;
            const int nvc = min(64, nv - v0);
#pragma unroll 1
            for (int u = 0; u < nvc; ++u) {
                const DevView &V = views[v0 + u];
                const CutTest c = meets_tau_f32(b, L2, Lok, V);
                uint64_t F = leaves | c.yes;
                const uint64_t open = ~(F | c.no) & live;
                if (open) {  // rare: decide by the FP64 evaluation that defines the cut
                    const bool m = ((open >> lane) & 1ull) && granularity(b, V) <= (double)V.tau;
                    F |= __ballot(m);
                }
                uint64_t sel = F & live & ~no_parent;  // nodes whose parent must fail the test
                uint64_t Fp = 0;
                if (sel) {
                    const CutTest cp = meets_tau_f32(pb, Lp2, Lpok, V);
                    Fp = cp.yes;
                    const uint64_t openp = ~(cp.yes | cp.no) & sel;
                    if (openp) {
                        const bool m = ((openp >> lane) & 1ull) && granularity(pb, V) <= (double)V.tau;
                        Fp |= __ballot(m);
                    }
                }
                const uint64_t cut = F & live & (no_parent | ~Fp);
                word = lane == u ? cut : word;
            }
            if (lane < nvc) {
                masks[(int64_t)(v0 + lane) * words + (i0 >> 6)] = word;
                if (word) atomicAdd(&s_cnt[v0 + lane], (uint32_t)__popcll(word));
            }
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < nv; v += kCutThreads) block_counts[(int64_t)v * nblocks + blockIdx.x] = s_cnt[v];
}

__device__ __forceinline__ double cut_weight(const DevHier &h, const DevView &V, int64_t i)
{
#pragma clang fp contract(off)
    const uint32_t par = h.pinfo[i] & ~kLeafBit;
    if (par == kRootParent) return 0.0;
    float b[6], pb[6];
    load_box(h, i, b);
    load_box(h, par, pb);
    const double en = granularity(b, V);
    const double ep = granularity(pb, V);
    if (__builtin_isinf(ep) || !(ep > en)) return 0.0;
    double t = ((double)V.tau - en) / (ep - en);
    return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}

// Index of the r-th set bit of m (r < popcount(m)), by halving.
__device__ __forceinline__ int nth_set_bit(uint64_t m, uint32_t r)
{
    int b = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const uint64_t low = m & ((1ull << width) - 1ull);
        const uint32_t c = (uint32_t)__popcll(low);
        if (r >= c) {
            r -= c;
            m >>= width;
            b += width;
        } else {
            m = low;
        }
    }
    return b;
}

// Emits the cut of kEmitViews views over one block of kCutBlock nodes: ids
// in node order at the positions the scan gave, the weight t, and the
// position of the first selected node of every mask word (word_off).  The
// selected nodes of the block are spread densely over its threads, so that
// every lane works on one of them.
constexpr int kEmitViews = 8;

__global__ __launch_bounds__(kCutThreads) void k_cut_emit(DevHier h, const DevView *__restrict__ views, int nv,
                                                          const uint64_t *__restrict__ masks,
                                                          const uint32_t *__restrict__ block_offsets, int nblocks,
                                                          uint32_t *__restrict__ word_off,
                                                          int32_t *__restrict__ out_ids, float *__restrict__ out_t,
                                                          double *__restrict__ out_t64, uint32_t cap)
{
    constexpr int W = kCutBlock / 64;  // mask words per block and view
    constexpr int VB = kEmitViews;
    __shared__ uint64_t s_word[VB][W];
    __shared__ uint32_t s_pre[VB][W + 1];  // selected nodes of the view before word k; [W]: the view's count
    __shared__ uint32_t s_vpre[VB + 1];    // selected nodes of the block before view u
    __shared__ uint32_t s_off[VB];         // cut position of the view's first selected node here
    const int64_t n = h.n;
    const int64_t words = (n + 63) >> 6;
    const int v0 = blockIdx.y * VB, nvb = min(VB, nv - v0);
    const int64_t w0 = (int64_t)blockIdx.x * W;
    if (threadIdx.x < VB * W) {
        const int u = threadIdx.x / W, k = threadIdx.x % W;
        const int64_t w = w0 + k;
        s_word[u][k] = u < nvb && w < words ? masks[(int64_t)(v0 + u) * words + w] : 0ull;
    }
    __syncthreads();
    if (threadIdx.x < VB) {
        const int u = threadIdx.x;
        uint32_t acc = 0;
        for (int k = 0; k < W; ++k) {
            s_pre[u][k] = acc;
            acc += (uint32_t)__popcll(s_word[u][k]);
        }
        s_pre[u][W] = acc;
        s_off[u] = acc ? block_offsets[(int64_t)(v0 + u) * nblocks + blockIdx.x] : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int u = 0; u < VB; ++u) {
            s_vpre[u] = acc;
            acc += s_pre[u][W];
        }
        s_vpre[VB] = acc;
    }
    __syncthreads();
    const uint32_t S = s_vpre[VB];
    if (S == 0) return;
    if (threadIdx.x < VB * W) {
        const int u = threadIdx.x / W, k = threadIdx.x % W;
        if (s_pre[u][W] && w0 + k < words) word_off[(int64_t)(v0 + u) * words + w0 + k] = s_off[u] + s_pre[u][k];
    }
    for (uint32_t j = threadIdx.x; j < S; j += kCutThreads) {
        int u = 0;  // view of the j-th selected node
        while (u + 1 < VB && s_vpre[u + 1] <= j) ++u;
        const uint32_t r = j - s_vpre[u];  // its rank among the view's selected nodes here
        int lo = 0, hi = W - 1;            // its word: the last k with s_pre[u][k] <= r (never empty)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[u][mid] <= r) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t pos = s_off[u] + r;
        if (pos >= cap) continue;
        const int bit = nth_set_bit(s_word[u][lo], r - s_pre[u][lo]);
        const int64_t i = (int64_t)blockIdx.x * kCutBlock + lo * 64 + bit;
        out_ids[pos] = (int32_t)i;
        if (out_t || out_t64) {
            const double t = cut_weight(h, views[v0 + u], i);
            if (out_t) out_t[pos] = (float)t;
            if (out_t64) out_t64[pos] = t;
        }
    }
}

__global__ void k_cut_finish(const uint32_t *__restrict__ block_offsets, int nblocks, int nv,
                             uint32_t *__restrict__ cut_base, const uint32_t *__restrict__ total)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < nv) cut_base[v] = block_offsets[(int64_t)v * nblocks];
    if (v == nv) cut_base[nv] = *total;
}

// Hierarchy compaction (Sec. 5.2, "Compacting the Hierarchy").  For a set
// of views and the granularity ladder tau_i = tau_min 2^i <= tau_max, the
// nodes that the paper keeps are the leaves, the bottom-most nodes of the
// union of the views' cuts at every tau_i, and the nodes above the last of
// these.  A node of the union has a descendant in it exactly when some view
// finds the node too coarse (that view's cut then lies below it), so the
// bottom-most nodes at tau are the cut of G(n) = "every view meets tau at n":
// n with G(n) and not G(parent).  With e(n) = max over the views of eps(n)
// (the same FP64 evaluation as the cut), G(n) is e(n) <= tau for an interior
// node, so one sweep over the views gives every level.
//
// k_node_emax: e(n) over one batch of views, folded into emax (first batch:
// written).  Leaves are not evaluated (they always meet tau).  L is the
// node's own, so the view of largest eps is the one of largest (f / d)^2: a
// first pass finds that ratio in FP32, and only views within a relative
// kEmaxBand of it (or with d^2 too small for FP32, where eps may be +inf)
// get the FP64 evaluation, whose maximum is therefore the exact one: the
// FP32 ratio is off by a few units in the last place, far inside the band.
constexpr float kEmaxBand = 2e-5f;

__device__ __forceinline__ float view_ratio(const float b[6], const DevView &V, float &d2)
{
    const float ex = V.eye[0], ey = V.eye[1], ez = V.eye[2];
    const float dx = ex - __builtin_amdgcn_fmed3f(ex, b[0], b[3]);
    const float dy = ey - __builtin_amdgcn_fmed3f(ey, b[1], b[4]);
    const float dz = ez - __builtin_amdgcn_fmed3f(ez, b[2], b[5]);
    d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float f = fmaxf(V.fx, V.fy);
    return f * f * __builtin_amdgcn_rcpf(d2);
}

__global__ __launch_bounds__(kCutThreads) void k_node_emax(DevHier h, const DevView *__restrict__ views, int nv,
                                                           int first, double *__restrict__ emax)
{
    const int64_t i = (int64_t)blockIdx.x * kCutThreads + threadIdx.x;
    if (i >= h.n) return;
    if (h.pinfo[i] & kLeafBit) {
        emax[i] = 0.0;
        return;
    }
    float b[6];
    load_box(h, i, b);
    float best = 0.0f;
    for (int v = 0; v < nv; ++v) {
        float d2;
        const float r = view_ratio(b, views[v], d2);
        if (d2 >= 1e-18f) best = fmaxf(best, r);
    }
    const float thr = best * (1.0f - kEmaxBand);
    double e = first ? 0.0 : emax[i];
    for (int v = 0; v < nv; ++v) {
        float d2;
        const float r = view_ratio(b, views[v], d2);
        if (d2 < 1e-18f || r >= thr) {
            const double g = granularity(b, views[v]);
            e = g > e ? g : e;
        }
    }
    emax[i] = e;
}

// keep[n] = 1 for a leaf, a node with e(n) <= tau_i < e(parent) for some
// level i (the root: e(n) <= tau_i), or a node with e(n) > tau_last; with no
// level at all (tau_min > tau_max) every node is kept.
__global__ __launch_bounds__(kCutThreads) void k_compact_keep(DevHier h, const double *__restrict__ emax,
                                                              double tau_min, int levels, uint8_t *__restrict__ keep)
{
    const int64_t i = (int64_t)blockIdx.x * kCutThreads + threadIdx.x;
    if (i >= h.n) return;
    const uint32_t pi = h.pinfo[i];
    if ((pi & kLeafBit) || levels == 0) {
        keep[i] = 1;
        return;
    }
    const uint32_t par = pi & ~kLeafBit;
    const bool root = par == kRootParent;
    const double en = emax[i], ep = root ? 0.0 : emax[par];
    bool k = false;
    double tau = tau_min;
    for (int l = 0; l < levels; ++l) {
        k |= en <= tau && (root || !(ep <= tau));
        if (l + 1 < levels) tau *= 2.0;
    }
    k |= !(en <= tau);
    keep[i] = k ? 1 : 0;
}

void launch_compact_emax(const DevHier &h, const DevView *views, int nv, bool first, double *emax, hipStream_t st)
{
    hipLaunchKernelGGL(k_node_emax, dim3((uint32_t)((h.n + kCutThreads - 1) / kCutThreads)), dim3(kCutThreads), 0,
                       st, h, views, nv, first ? 1 : 0, emax);
}

void launch_compact_keep(const DevHier &h, const double *emax, double tau_min, int levels, uint8_t *keep,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_compact_keep, dim3((uint32_t)((h.n + kCutThreads - 1) / kCutThreads)), dim3(kCutThreads),
                       0, st, h, emax, tau_min, levels, keep);
}

void launch_cut_flags(const DevHier &h, const DevView *views, int nv, uint64_t *masks, uint32_t *block_counts,
                      int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_cut_onepass, dim3(nblocks), dim3(kCutThreads), 0, st, h, views, nv, masks, block_counts,
                       nblocks);
}

void launch_cut_emit(const DevHier &h, const DevView *views, int nv, const uint64_t *masks,
                     const uint32_t *block_offsets, int nblocks, uint32_t *word_off, int32_t *out_ids, float *out_t,
                     double *out_t64, uint32_t cap, hipStream_t st)
{
    hipLaunchKernelGGL(k_cut_emit, dim3(nblocks, (nv + kEmitViews - 1) / kEmitViews), dim3(kCutThreads), 0, st, h,
                       views, nv, masks, block_offsets, nblocks, word_off, out_ids, out_t, out_t64, cap);
}

void launch_cut_finish(const uint32_t *block_offsets, const uint32_t *, int nblocks, int nv, uint32_t *cut_base,
                       Counters *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_cut_finish, dim3((nv + 1 + 255) / 256), dim3(256), 0, st, block_offsets, nblocks, nv,
                       cut_base, &ctr->cut_total);
}

}  // namespace hgs
