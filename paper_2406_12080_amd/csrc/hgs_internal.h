// Internal declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace hgs {

// Conventions of the splatting stage (3D Gaussian splatting defaults that the
// paper's renderer builds on; the 0.99 clamp is the one of Sec. 7.3).
constexpr float kAlphaMin = 1.0f / 255.0f;  // a splat with alpha below this is skipped
constexpr float kTMin = 1e-4f;              // stop before transmittance would fall below
constexpr float kAlphaMax = 0.99f;          // alpha clamp
constexpr double kDilation = 0.3;           // EWA screen-space low-pass variance (px^2)
constexpr int kMaxViews = 1024;

constexpr uint32_t kRootParent = 0x7FFFFFFFu;
constexpr uint32_t kLeafBit = 0x80000000u;

struct DevView {
    float R[9];
    float eye[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    float z_near, tau;
    float cut_klo, cut_khi;  // tau^2 (1 -+ kCutMargin) / max(fx, fy)^2: the cut's FP32 prefilter (NaN: off)
    int32_t tiles_x, tiles_y;
    uint32_t tile_base;  // first global tile id of this view
    uint32_t pix_base;   // first pixel of this view in per-pixel state arrays
    float *out_rgb;      // [H][W][3]
    const float *dL;     // [H][W][3], backward (read) and loss (written) only
    const float *target; // [H][W][3], loss only
};

// Relative band around the cut threshold inside which the FP32 prefilter
// defers to the FP64 evaluation.
constexpr float kCutMargin = 1e-5f;

struct DevHier {
    int64_t n;
    const uint32_t *pinfo;  // parent index | leaf bit
    const float *box;       // [6][n]: bmin x y z, bmax x y z
    const int32_t *child_count;
    const int32_t *child_begin;  // first child (children are contiguous); 0 for leaves
    const float *mean, *scale, *rot, *opacity, *sh;  // node-major: [N][3] [N][3] [N][4] [N] [N][48]
    // out-of-core rendering: the parameters above are a cache indexed by
    // slot[node] (< 0: not resident); nullptr: indexed by node id
    const int32_t *slot;
};

// Index of a node's parameters (its cache slot when rendering out of core).
__device__ __forceinline__ size_t param_index(const DevHier &h, uint32_t node)
{
    return h.slot ? (size_t)h.slot[node] : (size_t)node;
}

// ---------------------------------------------------- out-of-core rendering
struct StreamParams {
    float *mean, *scale, *rot, *opacity, *sh;  // node-major records (host: N nodes, cache: cap slots)
};
struct StreamDev {
    int32_t *slot;          // [N] cache slot of every node (-1 absent, -2 claimed)
    int32_t *node_in_slot;  // [cap] (-1 free)
    uint32_t *last_used;    // [cap] frame of the last cut that used the slot
    uint32_t *free_stack;   // [cap], free_top entries valid
    uint32_t *free_top, *frame, *req_count, *overflow;
    unsigned long long *transferred;  // total nodes transferred
    uint32_t *req;          // [req_cap] nodes requested this frame
    uint32_t cap, req_cap;
};
void launch_stream_init(const StreamDev &s, int64_t n_nodes, hipStream_t st);
void launch_stream_frame(const StreamDev &s, const uint32_t *pinfo, const int32_t *cut_ids,
                         const uint32_t *cut_total, uint32_t cap, const StreamParams &host,
                         const StreamParams &cache, hipStream_t st);
void launch_stream_cleanup(const StreamDev &s, uint32_t max_age, hipStream_t st);

// Blend record of one splat (48 bytes).  The mean is kept as an integer pixel
// anchor plus an FP32 fraction.  The conic (inverse dilated 2D covariance)
// is used through its eigen-axes scaled so that, for a pixel offset d from
// the mean, u_i = w_i . d and G = exp2(-(u_1^2 + u_2^2)) = exp(-d^T conic d / 2):
// a sum of squares, which FP32 evaluates without the cancellation the
// expanded quadratic form suffers for thin splats far from their centre.
struct __align__(16) SplatRec {
    int32_t ax, ay;
    float fx, fy;          // mean - anchor
    float An, Ap;          // kappa |o_n|, kappa |o_p|
    float t, invK;
    float r, g, b;
    float unused;
};
// The axes w = (w1x, w1y, w2x, w2y) are kept beside the record in FP64
// (double4): the per-8x8-block offsets w . (corner - mean) are formed from
// them in FP64, since a splat's centre can lie far off screen, where the FP32
// rounding of the axis direction alone would move the evaluated position by
// whole 1e-4s; the lanes use their FP32 rounding.
// 1/2 log2(e): exp(-q/2) = exp2(-kHalfLog2e q)
constexpr double kHalfLog2e = 0.72134752044448170368;
static_assert(sizeof(SplatRec) == 48, "record layout");

// Device-side counters of one render.
struct Counters {
    uint32_t cut_total;
    uint32_t vis_total;
    uint32_t pair_total;
    uint32_t overflow;
    unsigned long long evaluated;
    unsigned long long blended;
    unsigned long long evaluated_t;      // evaluated pairs of interpolated splats (t > 0)
    unsigned long long bwd_evaluated;    // backward: pairs re-evaluated
    unsigned long long bwd_evaluated_t;
    unsigned long long bwd_contrib;      // backward: pairs that contributed
};

// ---------------------------------------------------------------- launchers
// All launchers queue work on `st`; sizes that only the device knows are read
// from device memory (`*_dev`) and clamped to the host-side capacity.

// cut: per-node predicate over all views, bitmask + per-block counts
constexpr int kCutThreads = 256;
constexpr int kCutItems = 4;
constexpr int kCutBlock = kCutThreads * kCutItems;  // nodes per block
// masks: one bit per (view, node), words * nv; block_counts: per view and
// block of kCutBlock nodes.
// Hierarchy compaction: per-node maximum of eps over a batch of views
// (first batch: written, else folded in), then the keep flags for the
// granularity ladder tau_min 2^i, i < levels.
void launch_compact_emax(const DevHier &h, const DevView *views, int nv, bool first, double *emax, hipStream_t st);
void launch_compact_keep(const DevHier &h, const double *emax, double tau_min, int levels, uint8_t *keep,
                         hipStream_t st);
void launch_cut_flags(const DevHier &h, const DevView *views, int nv, uint64_t *masks, uint32_t *block_counts,
                      int nblocks, hipStream_t st);
// Also writes word_off[v][w]: the cut position of the first selected node of
// mask word w of view v (words holding a selected node only).
void launch_cut_emit(const DevHier &h, const DevView *views, int nv, const uint64_t *masks,
                     const uint32_t *block_offsets, int nblocks, uint32_t *word_off, int32_t *out_ids, float *out_t,
                     double *out_t64, uint32_t cap, hipStream_t st);
void launch_cut_finish(const uint32_t *block_offsets, const uint32_t *block_counts, int nblocks, int nv,
                       uint32_t *cut_base, Counters *ctr, hipStream_t st);

// exclusive scan of uint32 (optionally of in[idx[i]], gathered once into
// out); writes *total
void launch_scan(const uint32_t *in, const uint32_t *idx, uint32_t n_host, const uint32_t *n_dev, uint32_t *out,
                 uint32_t *total, uint32_t *partial, hipStream_t st);
constexpr int kScanBlocks = 512;

// stable LSD radix sort of (uint32 key, uint32 value) over bit range [0, bits)
struct SortBlock {  // work of one block of a segmented sort
    uint32_t b0, b1;    // its elements [b0, b1)
    uint32_t hbase;     // histogram slot of digit 0; digit d at hbase + d * hstride
    uint32_t hstride;   // 0: the block has no work
    uint32_t kbase;     // subtracted from every key of its segment before the digits are taken
    uint32_t pad[3];
};
struct SortScratch {
    uint32_t *k2, *v2;   // ping-pong buffers (capacity elements)
    uint32_t *hist;      // 256 * kSortBlocksMax
    uint32_t *hist_scan; // 256 * kSortBlocksMax
    uint32_t *partial;   // kScanBlocks
    uint32_t *total;     // 2: scan total, histogram length of a segmented sort
    SortBlock *plan;     // kSortBlocksMax
};
constexpr int kSortBlocksMax = 4096;
// Returns true when the sorted result is in (s.k2, s.v2) (odd pass count).
// With seg_bounds (device, nseg + 1 positions, ascending; nseg <= kMaxViews)
// every segment [seg_bounds[i], seg_bounds[i + 1]) is sorted on its own and
// stays in place, on the digits of key - seg_kbase[i] (seg_kbase may be NULL
// for zero).
bool launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t cap, const uint32_t *n_dev, int bits,
                       const SortScratch &s, hipStream_t st, const uint32_t *seg_bounds = nullptr, int nseg = 0,
                       const uint32_t *seg_kbase = nullptr);

// preprocess: interpolation, EWA projection, SH colour, footprint, per cut entry
void launch_preprocess(const DevHier &h, const DevView *views, int nv, const uint32_t *cut_base,
                       const int32_t *cut_ids, const double *cut_t, const uint32_t *cut_total, uint32_t cap,
                       SplatRec *recs, double4 *axes, uint32_t *depth_key, uint4 *trec, uint32_t *ntiles,
                       float *cjac, uint64_t *vis_mask, uint32_t *vis_block_counts, int tile_w, int tile_h,
                       hipStream_t st);
// Also writes vis_rank[k] = compaction position of visible cut entry k (the
// row of its screen-space gradient).
void launch_compact_visible(const uint64_t *vis_mask, const uint32_t *vis_block_offsets, const uint32_t *cut_total,
                            uint32_t cap, const uint32_t *depth_key, uint32_t *keys, uint32_t *vals,
                            uint32_t *vis_rank, uint32_t *vis_entry, hipStream_t st);
// Tile records of the visible splats in depth order (one gather through
// the sorted values): counts[i] = tile count and rect[i] = tile rectangle of
// the splat at depth slot i, from trec (per cut entry: rect.x, rect.y,
// tile count, unused; written for visible entries).
void launch_gather_tiles(const uint4 *trec, const uint32_t *sorted_vals, const uint32_t *vis_total, uint32_t vis_cap,
                         uint32_t *counts, uint2 *rect, uint32_t *jrank, hipStream_t st);
// Per view: the depth-order slot of its first visible splat (vis_bounds,
// nv + 1 entries, the last = visible total).
void launch_vis_bounds(const uint32_t *cut_base, int nv, const uint64_t *vis_mask, const uint32_t *vis_offsets,
                       const uint32_t *cut_total, uint32_t cap, const uint32_t *vis_total, uint32_t *bounds,
                       hipStream_t st);
// Per view: the position of its first (tile, splat) pair (nv + 1 entries,
// the last = pair total) and its first global tile id.
void launch_pair_bounds(const uint32_t *vis_bounds, const DevView *views, int nv, const uint32_t *pair_offsets,
                        const uint32_t *vis_total, uint32_t vis_cap, const uint32_t *pair_total, uint32_t pair_cap,
                        uint32_t *bounds, uint32_t *tile_base, hipStream_t st);
// block_first: duplicate_blocks(pair_cap) + 1 entries of workspace.  rect:
// tile rectangles in depth order (launch_gather_tiles).
void launch_duplicate(const uint2 *rect, const DevView *views, int nv, const uint32_t *cut_base,
                      const uint32_t *sorted_vals, const uint32_t *pair_offsets, uint32_t *block_first,
                      const uint32_t *vis_total, uint32_t vis_cap, const uint32_t *pair_total, uint32_t pair_cap,
                      uint32_t *pair_keys, uint32_t *pair_vals, Counters *ctr, hipStream_t st);
uint32_t duplicate_blocks(uint32_t pair_cap);
void launch_ranges(const uint32_t *pair_keys, const uint32_t *pair_total, uint32_t pair_cap, uint2 *ranges,
                   hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t st);
// tiles ordered by descending list length (longest first) for the blend grid
void launch_tile_keys(const uint2 *ranges, uint32_t n_tiles, uint32_t *keys, uint32_t *order, uint32_t *n_out,
                      hipStream_t st);

// blend (tile_w x tile_h pixels per workgroup, `batch` records staged per step)
bool blend_supported(int tw, int th, int batch);
// Looks up the persistent grids of this configuration (device attributes
// and occupancy), so that no such query runs while a launch is captured.
void blend_prepare(int tw, int th, int batch);
// persist: a grid of the chip's resident workgroups takes tile slots from
// the device-side queue (*queue, cleared by the launch sequence first)
// instead of one workgroup per tile.
// The deterministic mode of the blend backward (launch_blend_backward with a
// non-NULL DetArgs): per (tile, splat) pair, the tile's 11 screen-space terms
// go to part[11 p] by plain stores, p = the pair's position in the list
// k_duplicate emitted (pair_offsets[j] + the tile's row-major index in the
// tile rectangle rect[j] of depth-sorted visible splat j = jrank[cut entry]);
// launch_det_sum then writes each splat's screen gradient as the in-order sum
// of its pairs' rows.  No floating-point atomics: results are bit-identical
// from run to run.
struct DetArgs {
    const uint32_t *jrank;
    const uint32_t *pair_offsets;
    const uint2 *rect;
    double *part;
};
void launch_det_sum(const double *part, const uint32_t *pair_offsets, const uint32_t *sorted_vals,
                    const uint32_t *vis_rank, const uint32_t *vis_total, uint32_t vis_cap,
                    const uint32_t *pair_total, uint32_t pair_cap, double *sgrad, hipStream_t st);

// Quarter records of the forward, read by the backward: byte b * qstride + p
// (b < the tile's 8x8 blocks, at most kMaxBlocks; qstride >= the pair count)
// holds, for the splat at position p of the sorted pair list and block b of
// its tile, bit q set when some pixel of quarter q of the block blended it
// or stopped at it (a superset of the blends; the backward's per-pixel test
// of the last contributor drops the rest).
constexpr int kMaxBlocks = 8;
void launch_blend(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *tile_order, const uint2 *ranges,
                  const uint32_t *pair_vals,
                  const SplatRec *recs, const double4 *axes, float *T_final, uint32_t *n_last, uint32_t *n_blend,
                  uint8_t *qbits, uint32_t qstride, uint4 *wstats, Counters *ctr, int tw, int th, int batch,
                  bool persist, uint32_t *queue, hipStream_t st);

// ---------------------------------------------------- hierarchy generation
// Node arrays of the tree under construction (breadth-first ids).
struct BuildTree {
    int32_t *start, *size;  // first sorted leaf position and leaf count
    int32_t *parent, *child_begin, *child_count;
};
// Leaf inputs, node-major: pos [n][3], scale [n][3], rot [n][4], opacity [n], sh [n][48].
struct BuildLeaves {
    const float *pos, *scale, *rot, *opacity, *sh;
};
// FP64 working values per node (mean [3], cov [6], op, surf, axes [9],
// scales [3], matched R [9] and q [4]) and the interior nodes' SH [48] by
// interior rank.
struct BuildWork {
    double *mean, *cov, *op, *surf, *axes, *sc;
    double *sh;
    int32_t *irank;
    double *R, *q;
};
// FP32 outputs, node-major (bmin / bmax [N][3]).
struct BuildOut {
    float *mean, *scale, *rot, *opacity, *sh, *bmin, *bmax;
};
void build_axis_maps_upload(hipStream_t st);
void launch_build_bounds(const float *pos, int64_t n, float *part, int nblocks, hipStream_t st);
void launch_build_morton(const float *pos, int64_t n, const double lo[3], double s, uint32_t *key_lo,
                         uint32_t *key_hi, uint32_t *idx, hipStream_t st);
void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t n, uint32_t *dst, hipStream_t st);
void launch_split_level(const uint32_t *lo, const uint32_t *hi, int64_t n, uint8_t *sl, hipStream_t st);
void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
void launch_level_starts(const int32_t *node_of, const uint8_t *sl, const BuildTree &t, int64_t n, int next_level,
                         uint32_t *flag, hipStream_t st);
void launch_level_nodes(const int32_t *node_of, const uint32_t *flag, const uint32_t *rank, const BuildTree &t,
                        int64_t n, int32_t base, int32_t *node_of_next, hipStream_t st);
void launch_level_sizes(const BuildTree &t, int32_t base, int32_t count, int64_t n, const uint32_t *sorted_idx,
                        int32_t *leaf_src, hipStream_t st);
void launch_interior_ranks(const int32_t *child_count, int64_t N, uint32_t *flag, hipStream_t st);
void launch_interior_list(const int32_t *child_count, const uint32_t *irank, int64_t N, int32_t *interior,
                          hipStream_t st);
void launch_merge_level(const BuildTree &t, const int32_t *leaf_src, const BuildLeaves &in, const BuildWork &w,
                        int32_t base, int32_t count, hipStream_t st);
void launch_match_level(const BuildTree &t, const BuildWork &w, int32_t base, int32_t count, const BuildOut &o,
                        const int32_t *leaf_src, const float *in_sh, hipStream_t st);
void launch_box_level(const BuildTree &t, int32_t base, int32_t count, float *bmin, float *bmax, hipStream_t st);
// pinfo (parent | leaf bit) and the component-major boxes [6][N] of a built tree
void launch_build_finish(const BuildTree &t, int64_t N, const float *bmin, const float *bmax, uint32_t *pinfo,
                         float *box, hipStream_t st);
// the inverse, for downloads: parent and node-major boxes from pinfo and [6][N]
void launch_unpack_nodes(const uint32_t *pinfo, const float *box, int64_t N, int32_t *parent, float *bmin,
                         float *bmax, hipStream_t st);

// L1 loss of the rendered images (views[v].out_rgb) against views[v].target
// over n_pix pixels of all views: dL/dC written to views[v].dL, the mean
// absolute difference to *loss (device), summed over at most kL1Blocks
// per-block partials (partial: workspace of that many doubles).
// Floats per cut entry of the attribute-gradient rows between the
// preprocess backward and the gradient gather.
constexpr int kPGradFloats = 20;

constexpr int kL1Blocks = 1024;
void launch_l1(const DevView *views, int nv, uint32_t n_pix, double *partial, double *loss, hipStream_t st);

// backward
void launch_blend_backward(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *tile_order,
                           const uint2 *ranges,
                           const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, const float *T_final,
                           const uint32_t *n_last, const uint8_t *qbits, uint32_t qstride, const uint32_t *vis_rank,
                           double *sgrad, const DetArgs *det, uint4 *wstats,
                           Counters *ctr, int tw, int th, int batch, bool want_dt, bool persist, uint32_t *queue,
                           hipStream_t st);
// optimiser step (Adam) over the interior nodes of one parameter group
// (0 mean, 1 scale, 2 rotation, 3 opacity, 4 SH); bc1 = 1 / (1 - beta1^t),
// bc2 = 1 / (1 - beta2^t)
struct AdamScalars {
    float lr, beta1, beta2, eps, bc1, bc2;
};

// One Adam update of one element (the step of 3D Gaussian Splatting's
// optimiser, bias-corrected): the separate optimiser step and the one fused
// into the gradient gather both call it, so that they agree bit for bit.
// The fused multiply-adds are written out and no other contraction is
// allowed: left to the compiler, the choice of which product to fuse
// differed between the two kernels.
__device__ __forceinline__ void adam_one(float &p, float g, float &m, float &v, const AdamScalars &s)
{
#pragma clang fp contract(off)
    m = fmaf(s.beta1, m, (1.0f - s.beta1) * g);
    v = fmaf(s.beta2, v, ((1.0f - s.beta2) * g) * g);
    p -= s.lr * (m * s.bc1) / (sqrtf(v * s.bc2) + s.eps);
}

// The optimiser step fused into the backward's gradient gather: per group
// the parameters (node-major) and both moments (by interior rank), and the
// group's scalars in device memory (5 records, written before each launch).
struct AdamRows {
    float *p[5], *m[5], *v[5];
    const AdamScalars *sc;
};
void launch_zero_rows(double *rows, int width, const uint32_t *vis_total, uint32_t vis_cap, hipStream_t st);
void launch_preprocess_backward(const DevHier &h, const DevView *views, int nv, const uint32_t *cut_base,
                                const int32_t *cut_ids, const double *cut_t, const uint32_t *cut_total, uint32_t cap,
                                const uint32_t *ntiles, const SplatRec *recs, const float *cjac,
                                const uint32_t *vis_entry, const uint32_t *vis_total, const double *sgrad, float *pg,
                                const uint64_t *masks, int64_t words, const uint32_t *word_off,
                                const int32_t *interior, int64_t n_interior, float *g_mean, float *g_scale,
                                float *g_rot, float *g_opacity, float *g_sh, float *g_dt, const AdamRows *fused,
                                hipStream_t st);

void launch_adam(int group, const int32_t *interior, int64_t n_interior, float *p, float *g, float *m, float *v,
                 const AdamScalars &s, hipStream_t st);

// ------------------------------------------------------------ wave helpers
// Lane exchange through DPP (no LDS traffic); CTRL is a DPP control word:
// 0x128 rotates each row of 16 lanes by 8 (lane l reads l ^ 8), 0x141
// mirrors each half row (l ^ 7), quad permutations 0x4E (l ^ 2) and 0xB1
// (l ^ 1).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

}  // namespace hgs
