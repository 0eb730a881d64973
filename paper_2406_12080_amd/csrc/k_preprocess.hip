// Preprocess (one thread per cut entry): interpolation and EWA projection in
// FP64, footprint and tile rectangle, then SH colour (FP32) of the visible
// splats only; then visibility compaction, tile
// counts, pair emission and per-tile ranges.  Also the preprocess backward.
#include <algorithm>

#include "hgs_internal.h"
#include "project.h"

namespace hgs {

namespace {

constexpr int kT = 256;
constexpr double kAlphaMinD = 1.0 / 255.0;
// per cut entry, gradient w.r.t. the interpolated attributes: mean 0..2,
// scale 3..5, raw quaternion 6..9, node opacity 10, parent opacity 11,
// colour cotangent 12..14, view direction 15..17 (the SH basis follows from
// it in the gather, as the forward evaluated it), 18 unused, live flag 19
constexpr int kPG = kPGradFloats;
static_assert(kPG == 20, "row layout");

__device__ __forceinline__ int view_of(const uint32_t *cut_base, int nv, uint32_t k)
{
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cut_base[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// view_of for the lanes of a wave whose entries are close together: one
// search with the first active lane's entry (a wave-uniform value, so its
// loads go through the scalar cache), and a search of its own only for a
// lane whose entry lies outside that view
__device__ __forceinline__ int view_of_wave(const uint32_t *cut_base, int nv, uint32_t k)
{
    const uint32_t kf = __builtin_amdgcn_readfirstlane(k);
    const int vf = view_of(cut_base, nv, kf);
    const uint32_t b0 = cut_base[vf], b1 = vf + 1 < nv ? cut_base[vf + 1] : 0xFFFFFFFFu;
    return k >= b0 && k < b1 ? vf : view_of(cut_base, nv, k);
}

__global__ __launch_bounds__(kT, 5) void k_preprocess(DevHier h, const DevView *__restrict__ views, int nv,
                                                   const uint32_t *__restrict__ cut_base,
                                                   const int32_t *__restrict__ cut_ids,
                                                   const double *__restrict__ cut_t,
                                                   const uint32_t *__restrict__ cut_total, uint32_t cap,
                                                   SplatRec *__restrict__ recs, double4 *__restrict__ axes,
                                                   uint32_t *__restrict__ depth_key,
                                                   uint4 *__restrict__ trec, uint32_t *__restrict__ ntiles,
                                                   float *__restrict__ cjac, uint64_t *__restrict__ vis_mask,
                                                   uint32_t *__restrict__ vis_block_counts, int tile_w, int tile_h)
{
    __shared__ uint32_t s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const uint32_t total = min(*cut_total, cap);
    const uint32_t k = blockIdx.x * kT + threadIdx.x;
    bool vis = false;
    uint32_t nt = 0;
    if (k < total) {
        const int vi = view_of_wave(cut_base, nv, k);
        const DevView &V = views[vi];
        Proj P;
        project_splat(h, V, (uint32_t)cut_ids[k], cut_t[k], P);
        if (P.ok) {
            // footprint: alpha <= min(0.99, A G) with A = kappa((1-t)o_n + t o_p);
            // alpha_min can only be reached inside d^T Sigma2'^-1 d <= 2 ln(A/alpha_min)
            const double A = P.kappa * ((1.0 - P.t) * P.o_n + P.t * P.o_p);
            if (A >= kAlphaMinD && fabs(P.u) < 1e9 && fabs(P.v) < 1e9) {
                const double r2 = 2.0 * log(A / kAlphaMinD);
                const double hx = sqrt(r2 * (P.a + kDilation)), hy = sqrt(r2 * (P.c + kDilation));
                double x0 = ceil(P.u - hx - 0.5), x1 = floor(P.u + hx - 0.5);
                double y0 = ceil(P.v - hy - 0.5), y1 = floor(P.v + hy - 0.5);
                x0 = fmax(x0, 0.0);
                y0 = fmax(y0, 0.0);
                x1 = fmin(x1, (double)(V.W - 1));
                y1 = fmin(y1, (double)(V.H - 1));
                if (x1 >= x0 && y1 >= y0) {
                    vis = true;
                    const uint32_t tx0 = (uint32_t)x0 / tile_w, tx1 = (uint32_t)x1 / tile_w;
                    const uint32_t ty0 = (uint32_t)y0 / tile_h, ty1 = (uint32_t)y1 / tile_h;
                    nt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                    trec[k] = make_uint4(tx0 | (tx1 << 16), ty0 | (ty1 << 16), nt, 0u);
                    SplatRec r;
                    const double fu = floor(P.u), fv = floor(P.v);
                    r.ax = (int32_t)fu;
                    r.ay = (int32_t)fv;
                    r.fx = (float)(P.u - fu);
                    r.fy = (float)(P.v - fv);
                    // eigen-axes of the conic [[ca, cb], [cb, cc]]: the major axis at
                    // angle th with (cos 2th, sin 2th) = (ca - cc, 2 cb) / r, its cosine
                    // and sine by the half-angle formulas (each from the better
                    // conditioned one), th in (-pi/2, pi/2]; any direction for a circle
                    const double ca = P.conic[0], cb = P.conic[1], cc = P.conic[2];
                    const double dx = ca - cc, dy = 2.0 * cb, rr = sqrt(dx * dx + dy * dy);
                    double cs = 1.0, sn = 0.0;
                    if (rr > 0.0) {
                        const double c2 = dx / rr, s2 = dy / rr;
                        if (c2 >= 0.0) {
                            cs = sqrt(0.5 * (1.0 + c2));
                            sn = s2 / (2.0 * cs);
                        } else {
                            sn = copysign(sqrt(0.5 * (1.0 - c2)), s2);
                            cs = s2 / (2.0 * sn);
                        }
                    }
                    const double l1 = ca * cs * cs + 2.0 * cb * sn * cs + cc * sn * sn;
                    const double l2 = ca * sn * sn - 2.0 * cb * sn * cs + cc * cs * cs;
                    const double s1 = sqrt(fmax(l1, 0.0) * kHalfLog2e), s2 = sqrt(fmax(l2, 0.0) * kHalfLog2e);
                    const double4 ax4 = make_double4(s1 * cs, s1 * sn, -s2 * sn, s2 * cs);
                    axes[k] = ax4;
                    r.An = (float)(P.kappa * P.o_n);
                    r.Ap = (float)(P.kappa * P.o_p);
                    r.t = (float)P.t;
                    r.invK = (float)(1.0 / (double)P.K);
                    float raw[3], dcol[3][3], dpn[3];
                    splat_colour(h, P, raw, dcol, dpn);  // visible splats only
                    r.r = fmaxf(raw[0], 0.0f);
                    r.g = fmaxf(raw[1], 0.0f);
                    r.b = fmaxf(raw[2], 0.0f);
                    r.unused = 0.0f;
                    recs[k] = r;
                    depth_key[k] = __float_as_uint((float)P.pc[2]);
                    float *cj = cjac + (size_t)k * 12;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) {
                        cj[3 * ch] = dcol[ch][0];
                        cj[3 * ch + 1] = dcol[ch][1];
                        cj[3 * ch + 2] = dcol[ch][2];
                        cj[9 + ch] = dpn[ch];
                    }
                }
            }
        }
        ntiles[k] = nt;
    }
    const uint64_t m = __ballot(vis);
    const uint32_t k0 = blockIdx.x * kT + (threadIdx.x & ~63u);
    if ((threadIdx.x & 63) == 0) {
        if (k0 < cap) vis_mask[k0 >> 6] = m;
        if (m) atomicAdd(&s_cnt, (uint32_t)__popcll(m));
    }
    __syncthreads();
    if (threadIdx.x == 0) vis_block_counts[blockIdx.x] = s_cnt;
}

__global__ __launch_bounds__(kT) void k_compact_visible(const uint64_t *__restrict__ vis_mask,
                                                        const uint32_t *__restrict__ offsets,
                                                        const uint32_t *__restrict__ cut_total, uint32_t cap,
                                                        const uint32_t *__restrict__ depth_key,
                                                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                        uint32_t *__restrict__ vis_rank,
                                                        uint32_t *__restrict__ vis_entry)
{
    const uint32_t total = min(*cut_total, cap);
    const uint32_t k = blockIdx.x * kT + threadIdx.x;
    if (blockIdx.x * kT >= total) return;
    __shared__ uint32_t s_pre[kT / 64];
    __shared__ uint64_t s_m[kT / 64];
    if (threadIdx.x < kT / 64) s_m[threadIdx.x] = vis_mask[blockIdx.x * (kT / 64) + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int w = 0; w < kT / 64; ++w) {
            s_pre[w] = acc;
            acc += (uint32_t)__popcll(s_m[w]);
        }
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, bit = threadIdx.x & 63;
    const uint64_t m = s_m[w];
    if (k < total && ((m >> bit) & 1ull)) {
        const uint32_t pos = offsets[blockIdx.x] + s_pre[w] + (uint32_t)__popcll(m & ((1ull << bit) - 1ull));
        keys[pos] = depth_key[k];
        vals[pos] = k;
        vis_rank[k] = pos;
        vis_entry[pos] = k;
    }
}

// Per view, the slot of its first visible splat: visible entries before cut
// position cut_base[v] (the visible list keeps the cut's view-major order).
__global__ void k_vis_bounds(const uint32_t *__restrict__ cut_base, int nv, const uint64_t *__restrict__ vis_mask,
                             const uint32_t *__restrict__ vis_offsets, const uint32_t *__restrict__ cut_total,
                             uint32_t cap, const uint32_t *__restrict__ vis_total, uint32_t *__restrict__ bounds)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > nv) return;
    const uint32_t total = min(*cut_total, cap);
    const uint32_t k = v < nv ? cut_base[v] : total;
    if (k >= total) {
        bounds[v] = min(*vis_total, cap);
        return;
    }
    uint32_t c = vis_offsets[k / kT];  // visible entries of the preprocess blocks before k's
    for (uint32_t w = (k / kT) * (kT / 64); w < (k >> 6); ++w) c += (uint32_t)__popcll(vis_mask[w]);
    if (k & 63u) c += (uint32_t)__popcll(vis_mask[k >> 6] & ((1ull << (k & 63u)) - 1ull));
    bounds[v] = c;
}

// Per view, the position of its first pair and its first global tile id.
__global__ void k_pair_bounds(const uint32_t *__restrict__ vis_bounds, const DevView *__restrict__ views, int nv,
                              const uint32_t *__restrict__ pair_offsets, const uint32_t *__restrict__ vis_total,
                              uint32_t vis_cap, const uint32_t *__restrict__ pair_total, uint32_t pair_cap,
                              uint32_t *__restrict__ bounds, uint32_t *__restrict__ tile_base)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v > nv) return;
    const uint32_t nvis = min(*vis_total, vis_cap), npairs = min(*pair_total, pair_cap);
    const uint32_t j = vis_bounds[v];
    bounds[v] = j < nvis ? min(pair_offsets[j], npairs) : npairs;
    if (v < nv) tile_base[v] = views[v].tile_base;
}

// The tile records of the visible splats in depth order: the one random
// gather of per-splat data between the depth sort and the pair emission;
// also each cut entry's depth-order slot (jrank), which the deterministic
// backward uses to find a pair's position in the emitted list.
__global__ __launch_bounds__(kT) void k_gather_tiles(const uint4 *__restrict__ trec,
                                                     const uint32_t *__restrict__ sorted_vals,
                                                     const uint32_t *__restrict__ vis_total, uint32_t vis_cap,
                                                     uint32_t *__restrict__ counts, uint2 *__restrict__ rect,
                                                     uint32_t *__restrict__ jrank)
{
    const uint32_t n = min(*vis_total, vis_cap);
    const uint32_t i = blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = sorted_vals[i];
    const uint4 r = trec[s];
    counts[i] = r.z;
    rect[i] = make_uint2(r.x, r.y);
    jrank[s] = i;
}

// Deterministic mode: the screen gradient of depth-sorted visible splat j is
// the sum, in emission order, of the rows its pairs' tiles stored (every row
// of the emitted list is written by the backward or zeroed before it).
__global__ __launch_bounds__(kT) void k_det_sum(const double *__restrict__ part,
                                                const uint32_t *__restrict__ pair_offsets,
                                                const uint32_t *__restrict__ sorted_vals,
                                                const uint32_t *__restrict__ vis_rank,
                                                const uint32_t *__restrict__ vis_total, uint32_t vis_cap,
                                                const uint32_t *__restrict__ pair_total, uint32_t pair_cap,
                                                double *__restrict__ sgrad)
{
    const uint32_t n = min(*vis_total, vis_cap);
    const uint32_t j = blockIdx.x * kT + threadIdx.x;
    if (j >= n) return;
    const uint32_t p0 = min(pair_offsets[j], pair_cap);
    const uint32_t p1 = min(j + 1 < n ? pair_offsets[j + 1] : *pair_total, pair_cap);
    double acc[11];
#pragma unroll
    for (int k = 0; k < 11; ++k) acc[k] = 0.0;
    for (uint32_t p = p0; p < p1; ++p) {
        const double *row = part + (size_t)p * 11;
#pragma unroll
        for (int k = 0; k < 11; ++k) acc[k] += row[k];
    }
    double *o = sgrad + (size_t)vis_rank[sorted_vals[j]] * 12;
#pragma unroll
    for (int k = 0; k < 11; ++k) o[k] = acc[k];
    o[11] = 0.0;
}

// Pair emission, balanced by pairs: block b writes pairs [b P, (b + 1) P)
// of the depth-ordered list, whatever the footprints of the splats they come
// from (the nearest splats of every view sort first and may cover thousands
// of tiles each).  k_dup_starts records the splat holding each block's first
// pair; k_duplicate stages the block's slice of the pair offsets in LDS.
// Each thread writes kDupPer consecutive pairs (one vector store per array
// and thread, contiguous across the wave): a binary search finds the splat
// of its first pair, then it walks forward tile by tile.
constexpr int kDupPer = 8;
constexpr uint32_t kDupPairs = kT * kDupPer;

__global__ __launch_bounds__(kT) void k_dup_starts(const uint32_t *__restrict__ offsets,
                                                   const uint32_t *__restrict__ vis_total, uint32_t vis_cap,
                                                   const uint32_t *__restrict__ pair_total, uint32_t pair_cap,
                                                   uint32_t *__restrict__ block_first)
{
    const uint32_t nvis = min(*vis_total, vis_cap);
    const uint32_t npairs = min(*pair_total, pair_cap);
    const uint32_t j = blockIdx.x * kT + threadIdx.x;
    if (j >= nvis) return;
    const uint32_t o = offsets[j];
    const uint32_t e = j + 1 < nvis ? offsets[j + 1] : *pair_total;  // end of splat j's pairs
    for (uint32_t b = (o + kDupPairs - 1) / kDupPairs; b * kDupPairs < min(e, npairs); ++b) block_first[b] = j;
}

__global__ __launch_bounds__(kT) void k_duplicate(const uint2 *__restrict__ rect, const DevView *__restrict__ views,
                                                  int nv, const uint32_t *__restrict__ cut_base,
                                                  const uint32_t *__restrict__ sorted_vals,
                                                  const uint32_t *__restrict__ offsets,
                                                  const uint32_t *__restrict__ block_first,
                                                  const uint32_t *__restrict__ vis_total, uint32_t vis_cap,
                                                  const uint32_t *__restrict__ pair_total, uint32_t pair_cap,
                                                  uint32_t *__restrict__ pair_keys, uint32_t *__restrict__ pair_vals,
                                                  Counters *__restrict__ ctr)
{
    __shared__ uint32_t s_off[kDupPairs + 1];
    __shared__ uint32_t s_cb[kMaxViews + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0 && *pair_total > pair_cap) atomicOr(&ctr->overflow, 4u);
    const uint32_t nvis = min(*vis_total, vis_cap);
    const uint32_t npairs = min(*pair_total, pair_cap);
    const uint32_t o0 = blockIdx.x * kDupPairs;
    if (o0 >= npairs || nvis == 0) return;
    const uint32_t o1 = min(o0 + kDupPairs, npairs);
    const uint32_t j0 = block_first[blockIdx.x];
    // last splat that can hold one of the block's pairs: the one holding pair
    // o1 (or the last splat); never more than kDupPairs past j0, since every
    // splat has at least one pair (this also bounds the LDS slice when the
    // pair count exceeded the capacity)
    uint32_t j1 = o1 < npairs ? block_first[blockIdx.x + 1] : nvis - 1;
    j1 = min(j1, j0 + kDupPairs);
    const uint32_t cnt = j1 - j0 + 1;
    for (uint32_t k = threadIdx.x; k < cnt; k += kT) s_off[k] = offsets[j0 + k];
    for (int k = threadIdx.x; k <= nv; k += kT) s_cb[k] = cut_base[k];
    __syncthreads();
    const uint32_t ob = o0 + threadIdx.x * kDupPer;
    if (ob >= o1) return;
    uint32_t lo = 0, hi = cnt - 1;  // the last slot with s_off <= ob
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1u) >> 1;
        if (s_off[mid] <= ob) lo = mid;
        else hi = mid - 1u;
    }
    uint32_t key[kDupPer], val[kDupPer];
    uint32_t cur = ~0u, s = 0, tx = 0, ty = 0, tx0 = 0, tx1 = 0, base = 0, tiles_x = 0;
#pragma unroll
    for (int k = 0; k < kDupPer; ++k) {
        const uint32_t o = ob + k;
        if (o < o1) {
            while (lo + 1u < cnt && s_off[lo + 1u] <= o) ++lo;
            if (lo != cur) {  // first pair of this thread from splat slot lo
                cur = lo;
                s = sorted_vals[j0 + lo];
                int vlo = 0, vhi = nv - 1;  // view of cut entry s
                while (vlo < vhi) {
                    const int mid = (vlo + vhi + 1) >> 1;
                    if (s_cb[mid] <= s) vlo = mid;
                    else vhi = mid - 1;
                }
                const DevView &V = views[vlo];
                base = V.tile_base;
                tiles_x = (uint32_t)V.tiles_x;
                const uint2 r = rect[j0 + lo];
                tx0 = r.x & 0xFFFFu;
                tx1 = r.x >> 16;
                const uint32_t w = tx1 - tx0 + 1u, q = o - s_off[lo];
                ty = (r.y & 0xFFFFu) + q / w;
                tx = tx0 + q % w;
            } else if (++tx > tx1) {  // next tile of the same splat, row by row
                tx = tx0;
                ++ty;
            }
        }
        key[k] = base + ty * tiles_x + tx;
        val[k] = s;
    }
    if (ob + kDupPer <= o1) {
        uint4 *kd = reinterpret_cast<uint4 *>(pair_keys + ob), *vd = reinterpret_cast<uint4 *>(pair_vals + ob);
#pragma unroll
        for (int k = 0; k < kDupPer / 4; ++k) {
            kd[k] = make_uint4(key[4 * k], key[4 * k + 1], key[4 * k + 2], key[4 * k + 3]);
            vd[k] = make_uint4(val[4 * k], val[4 * k + 1], val[4 * k + 2], val[4 * k + 3]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kDupPer; ++k)
            if (ob + k < o1) {
                pair_keys[ob + k] = key[k];
                pair_vals[ob + k] = val[k];
            }
    }
}

// Zeroes the first (visible count) x width doubles of `rows` (the screen
// gradients, one row per visible splat by visible rank).
__global__ __launch_bounds__(kT) void k_zero_rows(double *__restrict__ rows, int width,
                                                  const uint32_t *__restrict__ vis_total, uint32_t vis_cap)
{
    const size_t n = (size_t)min(*vis_total, vis_cap) * (size_t)width;
    for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < n; e += (size_t)gridDim.x * kT) rows[e] = 0.0;
}

// Tile ranges of the sorted pair keys: four keys per thread (one vector
// load), boundaries found against the neighbours.  Tile ids stay below
// 2^31, so ~0 marks "no neighbour".
constexpr int kRangeItems = 4;

__global__ __launch_bounds__(kT) void k_ranges(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ total,
                                               uint32_t cap, uint2 *__restrict__ ranges)
{
    const uint32_t n = min(*total, cap);
    const uint32_t i0 = (blockIdx.x * kT + threadIdx.x) * kRangeItems;
    if (i0 >= n) return;
    uint32_t k[kRangeItems + 2];  // keys[i0 - 1 .. i0 + kRangeItems]
    k[0] = i0 > 0 ? keys[i0 - 1] : ~0u;
    if (i0 + kRangeItems <= n) {
        const uint4 v = *reinterpret_cast<const uint4 *>(keys + i0);
        k[1] = v.x;
        k[2] = v.y;
        k[3] = v.z;
        k[4] = v.w;
    } else {
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) k[1 + j] = i0 + j < n ? keys[i0 + j] : ~0u;
    }
    k[kRangeItems + 1] = i0 + kRangeItems < n ? keys[i0 + kRangeItems] : ~0u;
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) {
        const uint32_t i = i0 + j, t = k[1 + j];
        if (i >= n) break;
        if (k[j] != t) ranges[t].x = i;
        if (k[2 + j] != t) ranges[t].y = i + 1;
    }
}

// Scheduling key of every tile: 255 minus 8 log2(list length + 1), so that
// a stable ascending sort puts the longest lists first.
__global__ __launch_bounds__(kT) void k_tile_keys(const uint2 *__restrict__ ranges, uint32_t n_tiles,
                                                  uint32_t *__restrict__ keys, uint32_t *__restrict__ order,
                                                  uint32_t *__restrict__ n_out)
{
    const uint32_t i = blockIdx.x * kT + threadIdx.x;
    if (i == 0) *n_out = n_tiles;
    if (i >= n_tiles) return;
    const uint2 r = ranges[i];
    const uint32_t len = r.y - r.x + 1u;
    const uint32_t lg = 31u - (uint32_t)__clz(len);                   // floor(log2)
    const uint32_t frac = lg >= 3 ? (len >> (lg - 3)) & 7u : (len << (3 - lg)) & 7u;
    const uint32_t k = min(255u, lg * 8u + frac);
    keys[i] = 255u - k;
    order[i] = i;
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint32_t value, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ------------------------------------------------------------------ backward
// Thread v takes the v-th visible cut entry (vis_entry lists them in cut
// order, so that every wave holds visible entries only) and writes its
// attribute-gradient row at the entry's cut position; rows of entries that
// are not visible are never read.  With g_dt, thread k also clears dL/dt of
// cut entry k when it is not visible.
__global__ __launch_bounds__(kT, 3) void k_preprocess_bwd(DevHier h, const DevView *__restrict__ views, int nv,
                                                       const uint32_t *__restrict__ cut_base,
                                                       const int32_t *__restrict__ cut_ids,
                                                       const double *__restrict__ cut_t,
                                                       const uint32_t *__restrict__ cut_total, uint32_t cap,
                                                       const uint32_t *__restrict__ ntiles,
                                                       const SplatRec *__restrict__ recs,
                                                       const float *__restrict__ cjac,
                                                       const uint32_t *__restrict__ vis_entry,
                                                       const uint32_t *__restrict__ vis_total,
                                                       const double *__restrict__ sgrad, float *__restrict__ pg,
                                                       float *__restrict__ g_dt)
{
    const uint32_t total = min(*cut_total, cap);
    const uint32_t vis = min(*vis_total, total);
    const uint32_t tid = blockIdx.x * kT + threadIdx.x;
    if (g_dt && tid < total && ntiles[tid] == 0) g_dt[tid] = 0.0f;
    if (tid >= vis) return;
    const uint32_t k = vis_entry[tid];
    float *out = pg + (size_t)k * kPG;
    float row[kPG];  // the entry's attribute gradient, stored as five float4
    const double *sg = sgrad + (size_t)tid * 12;  // screen-gradient rows by visible rank
    const double du = sg[0], dv = sg[1], dAn = sg[5], dAp = sg[6];
    const double drgb[3] = {sg[7], sg[8], sg[9]};
    double dt = sg[10];
    const int vi = view_of_wave(cut_base, nv, k);
    const DevView &V = views[vi];
    Proj P;
    project_splat(h, V, (uint32_t)cut_ids[k], cut_t[k], P);
    if (!P.ok) {
        out[kPG - 1] = 0.0f;
        if (g_dt) g_dt[k] = 0.0f;
        return;
    }
    const uint32_t node = P.node, par = P.par;
    const bool node_leaf = (h.pinfo[node] & kLeafBit) != 0;
    const bool use_par = P.has_par && P.t > 0.0;
    const double t = P.t, w0 = 1.0 - t;

    // colour: rgb = max(0, raw); the forward kept rgb, d raw / d dir and
    // (SH_p - SH_n) . Y per channel
    const SplatRec rec = recs[k];
    const float *cj = cjac + (size_t)k * 12;
    double gr[3];
    gr[0] = rec.r > 0.0f ? drgb[0] : 0.0;
    gr[1] = rec.g > 0.0f ? drgb[1] : 0.0;
    gr[2] = rec.b > 0.0f ? drgb[2] : 0.0;
    double ddir[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ddir[0] += gr[c] * (double)cj[3 * c];
        ddir[1] += gr[c] * (double)cj[3 * c + 1];
        ddir[2] += gr[c] * (double)cj[3 * c + 2];
        if (use_par) dt += gr[c] * (double)cj[9 + c];
    }
    row[15] = (float)P.dir[0];
    row[16] = (float)P.dir[1];
    row[17] = (float)P.dir[2];
    row[18] = 0.0f;
    row[12] = (float)gr[0];
    row[13] = (float)gr[1];
    row[14] = (float)gr[2];
    double dmu[3];
    {
        const double dd = P.dir[0] * ddir[0] + P.dir[1] * ddir[1] + P.dir[2] * ddir[2];
#pragma unroll
        for (int m = 0; m < 3; ++m) dmu[m] = (ddir[m] - P.dir[m] * dd) / P.rlen;
    }

    // A_n = kappa o_n, A_p = kappa o_p
    const double dkappa = dAn * P.o_n + dAp * P.o_p;
    const double don = dAn * P.kappa, dop = dAp * P.kappa;

    // dL/d(a, b, c) of Sigma2 through the conic arrives accumulated per pixel
    // (the blend backward sums -dL/dq (conic d)(conic d)^T); add the part
    // through kappa = sqrt(det Sigma2 / det(Sigma2 + hI))
    const double a = P.a, b = P.b, c = P.c;
    const double ad = a + kDilation, cd = c + kDilation;
    const double Dd = P.Dd, D = P.D;
    double da = sg[2], db = sg[3], dc = sg[4];
    if (D > 0.0 && P.kappa > 0.0) {
        const double hk = 0.5 * P.kappa * dkappa;
        da += hk * (c / D - cd / Dd);
        dc += hk * (a / D - ad / Dd);
        db += hk * (2.0 * b / Dd - 2.0 * b / D);
    }

    // Sigma2 = Tm Sigma3 Tm^T
    const double *T0 = P.Tm, *T1 = P.Tm + 3;
    const double *S = P.cov3;
    const double Sf[9] = {S[0], S[1], S[2], S[1], S[3], S[4], S[2], S[4], S[5]};
    double T0S[3], T1S[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T0S[j] = T0[0] * Sf[j] + T0[1] * Sf[3 + j] + T0[2] * Sf[6 + j];
        T1S[j] = T1[0] * Sf[j] + T1[1] * Sf[3 + j] + T1[2] * Sf[6 + j];
    }
    double dS[9];  // gradient w.r.t. Sigma3 as a general matrix
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dS[3 * i + j] = da * T0[i] * T0[j] + db * T0[i] * T1[j] + dc * T1[i] * T1[j];
    double dT0[3], dT1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        dT0[j] = 2.0 * da * T0S[j] + db * T1S[j];
        dT1[j] = db * T0S[j] + 2.0 * dc * T1S[j];
    }
    // Tm = J R: row 0 = J00 R0 + J02 R2, row 1 = J11 R1 + J12 R2
    double R[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) R[q] = V.R[q];
    const double dJ00 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
    const double dJ02 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
    const double dJ11 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
    const double dJ12 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
    const double x = P.pc[0], y = P.pc[1], z = P.pc[2];
    const double iz = 1.0 / z, iz2 = iz * iz, iz3 = iz2 * iz;
    const double fx = V.fx, fy = V.fy;
    double dp[3];
    dp[0] = dJ02 * (-fx * iz2) + du * fx * iz;
    dp[1] = dJ12 * (-fy * iz2) + dv * fy * iz;
    dp[2] = dJ00 * (-fx * iz2) + dJ02 * (2.0 * fx * x * iz3) + dJ11 * (-fy * iz2) + dJ12 * (2.0 * fy * y * iz3) -
            du * fx * x * iz2 - dv * fy * y * iz2;
#pragma unroll
    for (int m = 0; m < 3; ++m) dmu[m] += R[m] * dp[0] + R[3 + m] * dp[1] + R[6 + m] * dp[2];

    // Sigma3 = M M^T, M = Rq diag(s)
    double Rq[9];
    quat_rot(P.q, Rq);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) M[3 * r + cc] = Rq[3 * r + cc] * P.s[cc];
    double ds[3] = {0.0, 0.0, 0.0}, dR[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) acc += (dS[3 * i + q] + dS[3 * q + i]) * M[3 * q + j];
            ds[j] += acc * Rq[3 * i + j];
            dR[3 * i + j] = acc * P.s[j];
        }
    const double qw = P.q[0], qx = P.q[1], qy = P.q[2], qz = P.q[3];
    double dq[4];
    dq[0] = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
    dq[1] = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - qw * dR[5] + qz * dR[6] + qw * dR[7] -
                   2.0 * qx * dR[8]);
    dq[2] = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] + qz * dR[7] -
                   2.0 * qy * dR[8]);
    dq[3] = 2.0 * (-2.0 * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.0 * qz * dR[4] + qy * dR[5] +
                   qx * dR[6] + qy * dR[7]);
    const double qd = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
    double dqr[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) dqr[m] = (dq[m] - P.q[m] * qd) / P.qlen;

    // gradient with respect to the interpolated attributes; the gather
    // weights it by (1 - t) for the node and t for the parent
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        row[m] = (float)dmu[m];
        row[3 + m] = (float)ds[m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) row[6 + m] = (float)dqr[m];
    if (use_par) {
        const float3 mn = *reinterpret_cast<const float3 *>(h.mean + 3 * (size_t)node);
        const float3 mp = *reinterpret_cast<const float3 *>(h.mean + 3 * (size_t)par);
        const float3 sn = *reinterpret_cast<const float3 *>(h.scale + 3 * (size_t)node);
        const float3 sp = *reinterpret_cast<const float3 *>(h.scale + 3 * (size_t)par);
        const float4 qn = *reinterpret_cast<const float4 *>(h.rot + 4 * (size_t)node);
        const float4 qp = *reinterpret_cast<const float4 *>(h.rot + 4 * (size_t)par);
        dt += dmu[0] * ((double)mp.x - (double)mn.x) + dmu[1] * ((double)mp.y - (double)mn.y) +
              dmu[2] * ((double)mp.z - (double)mn.z);
        dt += ds[0] * ((double)sp.x - (double)sn.x) + ds[1] * ((double)sp.y - (double)sn.y) +
              ds[2] * ((double)sp.z - (double)sn.z);
        dt += dqr[0] * ((double)qp.x - (double)qn.x) + dqr[1] * ((double)qp.y - (double)qn.y) +
              dqr[2] * ((double)qp.z - (double)qn.z) + dqr[3] * ((double)qp.w - (double)qn.w);
    }
    // opacity through |o|
    row[10] = (float)((P.on_raw > 0.0 ? 1.0 : (P.on_raw < 0.0 ? -1.0 : 0.0)) * don);
    row[11] = (float)((P.op_raw > 0.0 ? 1.0 : (P.op_raw < 0.0 ? -1.0 : 0.0)) * dop);
    row[kPG - 1] = 1.0f;
    float4 *out4 = reinterpret_cast<float4 *>(out);
#pragma unroll
    for (int q = 0; q < kPG / 4; ++q)
        out4[q] = make_float4(row[4 * q], row[4 * q + 1], row[4 * q + 2], row[4 * q + 3]);
    if (g_dt) g_dt[k] = use_par ? (float)dt : 0.0f;
}

// Gathers each interior node's parameter gradient from the cut entries of
// every view: its own entry weighted 1 - t, and the entry of each child in
// the cut with t > 0 weighted by that child's t (leaves are frozen; both
// opacity terms enter alpha directly, unweighted).  One thread per interior
// node, views and entries in a fixed order: no atomics, and the result is
// reproducible bit for bit.  Positions come from the cut's bit masks: node j
// of view v sits at word_off[v][j / 64] plus the selected nodes below j in
// its word.  The children of a node are contiguous ids, and those in the
// cut are consecutive cut entries, so one or two mask words give all of
// them at once.  The mask words of kGatherViews views are loaded together;
// positions and entries are read only for the views that hold one.
//
// FUSED: instead of adding the sum to the gradient arrays, the thread
// applies the optimiser step to its node right away (every interior node,
// those with no contribution too, whose gradient is zero): the gradient is
// never written, re-read or cleared.
constexpr int kGatherViews = 8;

// The fused optimiser step of one block: thread t holds the gathered
// gradient of interior node q0 + t (node id `node`; zero past the end).  The
// mean and scale rows (3 floats each) and the SH rows (48 floats, 64 rows at
// a time) go through LDS, so that the update walks the moments contiguously
// and each parameter row with consecutive lanes, as the separate step does;
// rotation (one 16-byte row) and opacity are stepped by the row's own
// thread from its registers.  The separate step reads 0 + sum
// from a cleared gradient array; the same value is formed here (it turns -0
// into +0), and the arithmetic is the same function, so both agree bit for
// bit.  Every thread of the block calls it (barriers).
constexpr int kAdamLds = 64 * 48;  // floats of the staging buffer (>= kT x 11)
static_assert(kT * 11 <= kAdamLds && kT % 64 == 0, "staging buffer");

__device__ __forceinline__ void adam_block(const AdamRows &ad, int64_t n_interior, int64_t q0, int32_t node,
                                           const float (&a)[11], const float (&ash)[48])
{
    __shared__ float s_g[kAdamLds];
    __shared__ int32_t s_node[kT];  // the block's node ids
    const int t = threadIdx.x;
    const int rows = (int)min<int64_t>(kT, n_interior - q0);  // >= 1: the block holds an interior node
    s_node[t] = node;
#pragma unroll
    for (int k = 0; k < 11; ++k) s_g[11 * t + k] = a[k];
    __syncthreads();
    // mean and scale: 3 floats per row
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
        const AdamScalars s = ad.sc[grp];
        float *p = ad.p[grp], *m = ad.m[grp] + 3 * q0, *v = ad.v[grp] + 3 * q0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = t + kT * k, r = e / 3, c = e - 3 * r;
            if (r < rows) {
                const int64_t pi = 3 * (int64_t)s_node[r] + c;
                float pk = p[pi], mk = m[e], vk = v[e];
                adam_one(pk, 0.0f + s_g[11 * r + 3 * grp + c], mk, vk, s);
                p[pi] = pk;
                m[e] = mk;
                v[e] = vk;
            }
        }
    }
    if (t < rows) {
        // rotation: one 16-byte row per thread; opacity: one float
        const AdamScalars s = ad.sc[2];
        float4 *p4 = reinterpret_cast<float4 *>(ad.p[2]) + node, *m4 = reinterpret_cast<float4 *>(ad.m[2]) + q0 + t,
               *v4 = reinterpret_cast<float4 *>(ad.v[2]) + q0 + t;
        float4 pk = *p4, mk = *m4, vk = *v4;
        adam_one(pk.x, 0.0f + a[6], mk.x, vk.x, s);
        adam_one(pk.y, 0.0f + a[7], mk.y, vk.y, s);
        adam_one(pk.z, 0.0f + a[8], mk.z, vk.z, s);
        adam_one(pk.w, 0.0f + a[9], mk.w, vk.w, s);
        *p4 = pk;
        *m4 = mk;
        *v4 = vk;
        const AdamScalars so = ad.sc[3];
        float po = ad.p[3][node], mo = ad.m[3][q0 + t], vo = ad.v[3][q0 + t];
        adam_one(po, 0.0f + a[10], mo, vo, so);
        ad.p[3][node] = po;
        ad.m[3][q0 + t] = mo;
        ad.v[3][q0 + t] = vo;
    }
    // SH: 64 rows of 12 float4 at a time
    const AdamScalars s = ad.sc[4];
    float4 *p4 = reinterpret_cast<float4 *>(ad.p[4]);
    float4 *m4 = reinterpret_cast<float4 *>(ad.m[4]) + 12 * q0, *v4 = reinterpret_cast<float4 *>(ad.v[4]) + 12 * q0;
    float4 *g4 = reinterpret_cast<float4 *>(s_g);
#pragma unroll 1
    for (int r0 = 0; r0 < rows; r0 += 64) {
        __syncthreads();  // the previous contents read
        if (t >= r0 && t < r0 + 64)
#pragma unroll
            for (int k = 0; k < 12; ++k)
                g4[12 * (t - r0) + k] = make_float4(ash[4 * k], ash[4 * k + 1], ash[4 * k + 2], ash[4 * k + 3]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = t + kT * k, r = e / 12, c = e - 12 * r;  // row r0 + r, vector c
            if (r0 + r < rows) {
                const int64_t pi = 12 * (int64_t)s_node[r0 + r] + c;
                const int64_t mi = 12 * (int64_t)r0 + e;
                const float4 g = g4[e];
                float4 pk = p4[pi], mk = m4[mi], vk = v4[mi];
                adam_one(pk.x, 0.0f + g.x, mk.x, vk.x, s);
                adam_one(pk.y, 0.0f + g.y, mk.y, vk.y, s);
                adam_one(pk.z, 0.0f + g.z, mk.z, vk.z, s);
                adam_one(pk.w, 0.0f + g.w, mk.w, vk.w, s);
                p4[pi] = pk;
                m4[mi] = mk;
                v4[mi] = vk;
            }
        }
    }
}

template <bool FUSED>
__global__ __launch_bounds__(kT, 4) void k_grad_gather(DevHier h, int nv, const uint64_t *__restrict__ masks,
                                                    int64_t words, const uint32_t *__restrict__ word_off,
                                                    const uint32_t *__restrict__ cut_total, uint32_t cap,
                                                    const double *__restrict__ cut_t,
                                                    const uint32_t *__restrict__ ntiles, const float *__restrict__ pg,
                                                    const int32_t *__restrict__ interior, int64_t n_interior,
                                                    float *__restrict__ g_mean, float *__restrict__ g_scale,
                                                    float *__restrict__ g_rot, float *__restrict__ g_op,
                                                    float *__restrict__ g_sh, AdamRows ad)
{
    const int64_t q = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool valid = q < n_interior;  // the fused step's threads past the end still help in its update
    if (!FUSED && !valid) return;
    const int64_t i = valid ? interior[q] : 0;
    float a[11];  // mean 3, scale 3, rotation 4, opacity
    float ash[48];
#pragma unroll
    for (int m = 0; m < 11; ++m) a[m] = 0.0f;
#pragma unroll
    for (int m = 0; m < 48; ++m) ash[m] = 0.0f;
    bool any = false;
    if (valid) {
        const uint32_t total = min(*cut_total, cap);
        const int64_t c0 = h.child_begin[i], c1 = c0 + h.child_count[i];  // children [c0, c1)
        // adds the attribute gradient of a contributing entry (row r), weighted
        // 1 - t as the node's own entry (op 10: node opacity term) or t as a
        // child's entry (op 11: parent opacity term)
        auto add = [&](const float4 (&r)[5], float t, int op) {
            const float w = op == 10 ? 1.0f - t : t;
            const float g[15] = {r[0].x, r[0].y, r[0].z, r[0].w, r[1].x, r[1].y, r[1].z, r[1].w,
                                 r[2].x, r[2].y, r[2].z, r[2].w, r[3].x, r[3].y, r[3].z};
#pragma unroll
            for (int m = 0; m < 10; ++m) a[m] += w * g[m];
            a[10] += op == 10 ? g[10] : g[11];
            float Y[16];  // the SH basis of the entry's direction, in FP32 as the forward evaluated it
            sh_eval_f(r[3].w, r[4].x, r[4].y, Y);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float wc = w * g[12 + c];
#pragma unroll
                for (int k = 0; k < 16; ++k) ash[3 * k + c] += wc * Y[k];
            }
            any = true;
        };
        // the entries at cut positions pa (op oa) and pb (op ob; ~0u: none),
        // added in that order: their tile counts and t first, then the rows
        // of those that are visible and contribute (a child's entry only with
        // t > 0; a row without a live splat adds nothing), the two entries'
        // loads in flight together
        auto take2 = [&](uint32_t pa, int oa, uint32_t pb, int ob) {
            const bool va = pa < total, vb = pb < total;
            uint32_t nta = 0, ntb = 0;
            float ta = 0.0f, tb = 0.0f;
            if (va) {
                nta = ntiles[pa];
                ta = (float)cut_t[pa];
            }
            if (vb) {
                ntb = ntiles[pb];
                tb = (float)cut_t[pb];
            }
            const bool ua = nta != 0 && (oa == 10 || ta > 0.0f), ub = ntb != 0 && (ob == 10 || tb > 0.0f);
            float4 ra[5], rb[5];
            if (ua) {
                const float4 *g4 = reinterpret_cast<const float4 *>(pg + (size_t)pa * kPG);
#pragma unroll
                for (int q = 0; q < 5; ++q) ra[q] = g4[q];
            }
            if (ub) {
                const float4 *g4 = reinterpret_cast<const float4 *>(pg + (size_t)pb * kPG);
#pragma unroll
                for (int q = 0; q < 5; ++q) rb[q] = g4[q];
            }
            if (ua && ra[4].w != 0.0f) add(ra, ta, oa);
            if (ub && rb[4].w != 0.0f) add(rb, tb, ob);
        };
        const int64_t wi = i >> 6, wa = c0 >> 6, wb = (c1 - 1) >> 6;
        const uint64_t below_i = (1ull << (i & 63)) - 1ull, own_bit = 1ull << (i & 63);
        // the children's bits in their first word (wa) and last word (wb)
        const int lo = (int)(c0 & 63), hi = (int)((c1 - 1) & 63);
        const uint64_t k_lo = ~((1ull << lo) - 1ull), k_hi = hi == 63 ? ~0ull : ((1ull << (hi + 1)) - 1ull);
        const uint64_t ka = wa == wb ? (k_lo & k_hi) : k_lo, kb = wa == wb ? 0ull : k_hi;
        const bool wide = wb - wa > 1;  // children over more than two words: every view is looked at
    #pragma unroll 1
        for (int v0 = 0; v0 < nv; v0 += kGatherViews) {
            // the views of this group that hold the node or one of its children
            // (their mask words loaded together)
            uint32_t hit = 0;
            if (wide) {
                hit = (1u << min(kGatherViews, nv - v0)) - 1u;
            } else {
    #pragma unroll
                for (int u = 0; u < kGatherViews; ++u) {
                    const int v = v0 + u;
                    if (v < nv) {
                        const uint64_t *mv = masks + (int64_t)v * words;
                        const uint64_t mo = mv[wi], ma = mv[wa], mb = kb ? mv[wb] : 0ull;
                        hit |= ((mo & own_bit) || (ma & ka) || (mb & kb)) ? 1u << u : 0u;
                    }
                }
            }
            while (hit) {
                const int v = v0 + __ffs(hit) - 1;
                hit &= hit - 1u;
                const uint64_t *mv = masks + (int64_t)v * words;
                const uint32_t *ov = word_off + (int64_t)v * words;
                // own entry
                const uint64_t mo = mv[wi];
                const uint32_t own = (mo & own_bit) ? ov[wi] + (uint32_t)__popcll(mo & below_i) : ~0u;
                // children: the selected ones among [c0, c1) are consecutive entries from p0
                uint32_t p0 = ~0u, nsel = 0;
                for (int64_t w = wa; w <= wb; ++w) {
                    const uint64_t mw = mv[w];
                    const uint64_t m = mw & (w == wa ? k_lo : ~0ull) & (w == wb ? k_hi : ~0ull);
                    if (!m) continue;
                    if (p0 == ~0u) p0 = ov[w] + (uint32_t)__popcll(mw & ((m & (~m + 1ull)) - 1ull));
                    nsel += (uint32_t)__popcll(m);
                }
                // the own entry, then the children's, two at a time
                uint32_t k = 0;
                if (own != ~0u) {
                    take2(own, 10, nsel ? p0 : ~0u, 11);
                    k = 1;
                }
                for (; k < nsel; k += 2) take2(p0 + k, 11, k + 1 < nsel ? p0 + k + 1 : ~0u, 11);
            }
        }
    }
    if constexpr (FUSED) {
        adam_block(ad, n_interior, (int64_t)blockIdx.x * kT, (int32_t)i, a, ash);
        return;
    }
    if (!any) return;
    // node-major records: vector read-modify-write
    float3 *gm = reinterpret_cast<float3 *>(g_mean + 3 * i), *gs = reinterpret_cast<float3 *>(g_scale + 3 * i);
    float4 *gr = reinterpret_cast<float4 *>(g_rot + 4 * i), *gh = reinterpret_cast<float4 *>(g_sh + 48 * i);
    float3 m3 = *gm, s3 = *gs;
    float4 r4 = *gr;
    m3.x += a[0];
    m3.y += a[1];
    m3.z += a[2];
    s3.x += a[3];
    s3.y += a[4];
    s3.z += a[5];
    r4.x += a[6];
    r4.y += a[7];
    r4.z += a[8];
    r4.w += a[9];
    *gm = m3;
    *gs = s3;
    *gr = r4;
    g_op[i] += a[10];
#pragma unroll
    for (int q = 0; q < 12; ++q) {
        float4 h4 = gh[q];
        h4.x += ash[4 * q];
        h4.y += ash[4 * q + 1];
        h4.z += ash[4 * q + 2];
        h4.w += ash[4 * q + 3];
        gh[q] = h4;
    }
}

}  // namespace

void launch_preprocess(const DevHier &h, const DevView *views, int nv, const uint32_t *cut_base,
                       const int32_t *cut_ids, const double *cut_t, const uint32_t *cut_total, uint32_t cap,
                       SplatRec *recs, double4 *axes, uint32_t *depth_key, uint4 *trec, uint32_t *ntiles,
                       float *cjac, uint64_t *vis_mask, uint32_t *vis_block_counts, int tile_w, int tile_h,
                       hipStream_t st)
{
    const uint32_t blocks = (cap + kT - 1) / kT;
    if (!blocks) return;
    hipLaunchKernelGGL(k_preprocess, dim3(blocks), dim3(kT), 0, st, h, views, nv, cut_base, cut_ids, cut_t, cut_total,
                       cap, recs, axes, depth_key, trec, ntiles, cjac, vis_mask, vis_block_counts, tile_w, tile_h);
}

void launch_compact_visible(const uint64_t *vis_mask, const uint32_t *vis_block_offsets, const uint32_t *cut_total,
                            uint32_t cap, const uint32_t *depth_key, uint32_t *keys, uint32_t *vals,
                            uint32_t *vis_rank, uint32_t *vis_entry, hipStream_t st)
{
    const uint32_t blocks = (cap + kT - 1) / kT;
    if (!blocks) return;
    hipLaunchKernelGGL(k_compact_visible, dim3(blocks), dim3(kT), 0, st, vis_mask, vis_block_offsets, cut_total, cap,
                       depth_key, keys, vals, vis_rank, vis_entry);
}

void launch_zero_rows(double *rows, int width, const uint32_t *vis_total, uint32_t vis_cap, hipStream_t st)
{
    const uint64_t need = ((uint64_t)vis_cap * width + kT - 1) / kT;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(need, 8192);
    if (!blocks) return;
    hipLaunchKernelGGL(k_zero_rows, dim3(blocks), dim3(kT), 0, st, rows, width, vis_total, vis_cap);
}

void launch_vis_bounds(const uint32_t *cut_base, int nv, const uint64_t *vis_mask, const uint32_t *vis_offsets,
                       const uint32_t *cut_total, uint32_t cap, const uint32_t *vis_total, uint32_t *bounds,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_vis_bounds, dim3((nv + 1 + 255) / 256), dim3(256), 0, st, cut_base, nv, vis_mask,
                       vis_offsets, cut_total, cap, vis_total, bounds);
}

void launch_pair_bounds(const uint32_t *vis_bounds, const DevView *views, int nv, const uint32_t *pair_offsets,
                        const uint32_t *vis_total, uint32_t vis_cap, const uint32_t *pair_total, uint32_t pair_cap,
                        uint32_t *bounds, uint32_t *tile_base, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_bounds, dim3((nv + 1 + 255) / 256), dim3(256), 0, st, vis_bounds, views, nv,
                       pair_offsets, vis_total, vis_cap, pair_total, pair_cap, bounds, tile_base);
}

void launch_gather_tiles(const uint4 *trec, const uint32_t *sorted_vals, const uint32_t *vis_total, uint32_t vis_cap,
                         uint32_t *counts, uint2 *rect, uint32_t *jrank, hipStream_t st)
{
    const uint32_t blocks = (vis_cap + kT - 1) / kT;
    if (!blocks) return;
    hipLaunchKernelGGL(k_gather_tiles, dim3(blocks), dim3(kT), 0, st, trec, sorted_vals, vis_total, vis_cap, counts,
                       rect, jrank);
}

void launch_det_sum(const double *part, const uint32_t *pair_offsets, const uint32_t *sorted_vals,
                    const uint32_t *vis_rank, const uint32_t *vis_total, uint32_t vis_cap,
                    const uint32_t *pair_total, uint32_t pair_cap, double *sgrad, hipStream_t st)
{
    const uint32_t blocks = (vis_cap + kT - 1) / kT;
    if (!blocks) return;
    hipLaunchKernelGGL(k_det_sum, dim3(blocks), dim3(kT), 0, st, part, pair_offsets, sorted_vals, vis_rank, vis_total,
                       vis_cap, pair_total, pair_cap, sgrad);
}

void launch_duplicate(const uint2 *rect, const DevView *views, int nv, const uint32_t *cut_base,
                      const uint32_t *sorted_vals, const uint32_t *pair_offsets, uint32_t *block_first,
                      const uint32_t *vis_total, uint32_t vis_cap, const uint32_t *pair_total, uint32_t pair_cap,
                      uint32_t *pair_keys, uint32_t *pair_vals, Counters *ctr, hipStream_t st)
{
    const uint32_t sblocks = (vis_cap + kT - 1) / kT;
    const uint32_t dblocks = (pair_cap + kDupPairs - 1) / kDupPairs;
    if (!sblocks || !dblocks) return;
    hipLaunchKernelGGL(k_dup_starts, dim3(sblocks), dim3(kT), 0, st, pair_offsets, vis_total, vis_cap, pair_total,
                       pair_cap, block_first);
    hipLaunchKernelGGL(k_duplicate, dim3(dblocks), dim3(kT), 0, st, rect, views, nv, cut_base, sorted_vals,
                       pair_offsets, block_first, vis_total, vis_cap, pair_total, pair_cap, pair_keys, pair_vals, ctr);
}

uint32_t duplicate_blocks(uint32_t pair_cap)
{
    return (pair_cap + kDupPairs - 1) / kDupPairs;
}

void launch_ranges(const uint32_t *pair_keys, const uint32_t *pair_total, uint32_t pair_cap, uint2 *ranges,
                   hipStream_t st)
{
    const uint32_t blocks = (uint32_t)(((uint64_t)pair_cap + kT * kRangeItems - 1) / (kT * kRangeItems));
    if (!blocks) return;
    hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(kT), 0, st, pair_keys, pair_total, pair_cap, ranges);
}

void launch_tile_keys(const uint2 *ranges, uint32_t n_tiles, uint32_t *keys, uint32_t *order, uint32_t *n_out,
                      hipStream_t st)
{
    if (!n_tiles) return;
    hipLaunchKernelGGL(k_tile_keys, dim3((n_tiles + kT - 1) / kT), dim3(kT), 0, st, ranges, n_tiles, keys, order,
                       n_out);
}

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st)
{
    if (!n) return;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, value, n);
}

void launch_preprocess_backward(const DevHier &h, const DevView *views, int nv, const uint32_t *cut_base,
                                const int32_t *cut_ids, const double *cut_t, const uint32_t *cut_total, uint32_t cap,
                                const uint32_t *ntiles, const SplatRec *recs, const float *cjac,
                                const uint32_t *vis_entry, const uint32_t *vis_total, const double *sgrad, float *pg,
                                const uint64_t *masks, int64_t words, const uint32_t *word_off,
                                const int32_t *interior, int64_t n_interior,
                                float *g_mean, float *g_scale, float *g_rot, float *g_opacity, float *g_sh,
                                float *g_dt, const AdamRows *fused, hipStream_t st)
{
    const uint32_t blocks = (cap + kT - 1) / kT;
    if (!blocks) return;
    hipLaunchKernelGGL(k_preprocess_bwd, dim3(blocks), dim3(kT), 0, st, h, views, nv, cut_base, cut_ids, cut_t,
                       cut_total, cap, ntiles, recs, cjac, vis_entry, vis_total, sgrad, pg, g_dt);
    const int64_t gblocks = (n_interior + kT - 1) / kT;
    if (!gblocks) return;
    if (fused)
        hipLaunchKernelGGL(k_grad_gather<true>, dim3((uint32_t)gblocks), dim3(kT), 0, st, h, nv, masks, words,
                           word_off, cut_total, cap, cut_t, ntiles, pg, interior, n_interior, nullptr, nullptr,
                           nullptr, nullptr, nullptr, *fused);
    else
        hipLaunchKernelGGL(k_grad_gather<false>, dim3((uint32_t)gblocks), dim3(kT), 0, st, h, nv, masks, words,
                           word_off, cut_total, cap, cut_t, ntiles, pg, interior, n_interior, g_mean, g_scale, g_rot,
                           g_opacity, g_sh, AdamRows{});
}

}  // namespace hgs
