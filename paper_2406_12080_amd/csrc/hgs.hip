// Host side of the C ABI declared in include/hgs.h: context, hierarchy
// upload and validation, workspace management, the launch sequence of the
// cut -> preprocess -> sort -> blend pipeline (direct for one view, captured
// in a HIP graph for several), and the backward.
#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hgs.h"
#include "hgs_internal.h"

using namespace hgs;

namespace {

template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t cap = 0;
};

constexpr int kTimedKernels = 4;  // blend, blend backward, preprocess backward, preprocess
constexpr int kStageRing = 4;     // pinned staging slots for the view copies

struct RenderKey {
    int nv = -1;
    std::vector<int> wh;
    int tw = 0, th = 0, batch = 0;
    bool persist = false;
    uint64_t layout = 0;
    bool profiled = false;
    bool operator==(const RenderKey &o) const
    {
        return nv == o.nv && wh == o.wh && tw == o.tw && th == o.th && batch == o.batch && persist == o.persist &&
               layout == o.layout && profiled == o.profiled;
    }
};

}  // namespace

struct hgs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;   // caller's (borrowed)
    hipStream_t gstream = nullptr;  // library-owned, for graph capture/launch
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string err;

    // hierarchy
    bool has_hier = false;
    int64_t n = 0, n_leaves = 0;
    uint32_t *pinfo = nullptr;
    float *box = nullptr;
    int32_t *child_count = nullptr, *child_begin = nullptr;
    int32_t *interior = nullptr;  // ids of the interior nodes, ascending
    int32_t *leaf_src = nullptr;  // after hgs_build: input index of every leaf node (-1 interior)
    // out-of-core rendering: parameters in pinned host memory, a device cache
    bool streaming = false;
    StreamDev sd{};
    StreamParams host_params{}, host_params_dev{}, cache_params{};
    void *host_block = nullptr;          // the pinned allocation behind host_params
    uint32_t *stream_host = nullptr;     // pinned readback: free_top, frame, req_count, overflow, transferred (2)
    int64_t n_interior = 0;
    float *own[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    float *bound[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool use_bound = false;
    uint64_t param_gen = 1;

    int tile_w = 16, tile_h = 16, batch = 0;
    bool persist = false;  // blend over a persistent grid and a device-side tile queue
    uint32_t *queue = nullptr;  // [0] forward, [1] backward: next tile slot
    double *l1_partial = nullptr;  // per-block partial sums of the L1 loss

    // workspaces
    uint64_t layout_gen = 1;
    std::vector<void *> allocs;
    DevView *views_dev = nullptr;
    double *cmp_emax = nullptr;  // compaction: per-node maximum granularity over the views
    int64_t cmp_emax_n = 0;
    DevView *views_host = nullptr;  // host records of the current views (pageable, changed freely)
    // pinned staging slots of the asynchronous view copies: a slot is reused
    // only after the copy that reads it has run (its event)
    DevView *stage[kStageRing] = {};
    hipEvent_t stage_ev[kStageRing] = {};
    bool stage_used[kStageRing] = {};
    int stage_next = 0;
    Counters *ctr = nullptr;
    Counters *ctr_host = nullptr;   // pinned
    uint32_t cut_cap = 0, pair_cap = 0;
    size_t pix_cap = 0, tile_cap = 0;
    int nblocks_cap = 0, nv_cap = 0;
    uint64_t *masks = nullptr;
    uint32_t *word_off = nullptr;  // per view and mask word: cut position of its first selected node
    uint32_t *blk_counts = nullptr, *blk_offsets = nullptr, *cut_base = nullptr;
    int32_t *cut_ids = nullptr;
    double *cut_t = nullptr;
    SplatRec *recs = nullptr;
    double4 *axes = nullptr;
    uint32_t *depth_key = nullptr, *ntiles = nullptr;
    uint4 *trec = nullptr;  // per cut entry: tile rectangle and count (visible entries)
    uint2 *rect = nullptr;  // tile rectangles of the visible splats in depth order
    uint32_t *jrank = nullptr;  // per cut entry: its slot in the depth order of the visible splats
    double *part = nullptr;     // deterministic backward: 11 doubles per emitted pair
    uint32_t part_cap = 0;
    bool deterministic = false;
    uint64_t *vis_mask = nullptr;
    uint32_t *vis_counts = nullptr, *vis_offsets = nullptr;
    uint32_t *skeys = nullptr, *svals = nullptr, *pair_offsets = nullptr;
    uint32_t *pkeys = nullptr, *pvals = nullptr;
    uint8_t *qbits = nullptr;  // forward quarter records, kMaxBlocks planes of pair_cap bytes
    uint32_t *dup_first = nullptr;  // first splat of every pair-emission block
    uint32_t *k2 = nullptr, *v2 = nullptr;
    uint32_t *hist = nullptr, *hist_scan = nullptr, *partial = nullptr, *scan_total = nullptr;
    SortBlock *sort_plan = nullptr;  // work of every block of a per-view (segmented) sort
    uint32_t *vis_bounds = nullptr, *pair_bounds = nullptr, *seg_tile_base = nullptr;  // per view
    uint2 *ranges = nullptr;
    uint32_t *tile_keys = nullptr, *tile_order = nullptr, *tile_k2 = nullptr, *tile_v2 = nullptr;
    uint32_t *tile_n = nullptr;
    uint4 *wstats = nullptr;  // per-wave work counts of the blend kernels
    size_t wstats_cap = 0;
    const uint32_t *tile_sorted = nullptr;  // the longest-first order (one of tile_order / tile_v2)
    float *T_final = nullptr;
    uint32_t *n_last = nullptr, *n_blend = nullptr;
    double *sgrad = nullptr;     // [visible rank][12] screen-space gradients
    uint32_t *vis_rank = nullptr;  // per cut entry: its visible rank (visible entries only)
    uint32_t *vis_entry = nullptr;  // per visible rank: its cut entry
    float *pgrad = nullptr;  // per cut entry, kPGradFloats floats
    float *cjac = nullptr;   // per cut entry, 12 floats: d colour / d dir, parent - node colour

    // state of the last render
    bool have_render = false;
    uint64_t render_seq = 0;  // id of the last successful render (ids start at 1)
    uint64_t render_param_gen = 0;
    int last_nv = 0;
    uint32_t last_tiles = 0;
    uint32_t last_cut = 0, last_visible = 0;
    size_t last_pix = 0;
    bool pairs_in_scratch = false;
    bool g_pairs_in_scratch = false;
    int r_tw = 16, r_th = 16, r_batch = 0;
    bool r_persist = false;

    // graph
    hipGraphExec_t gexec = nullptr;
    RenderKey gkey;
    bool g_profiled = false;
    // backward graph: keyed by the forward graph it follows and the
    // gradient outputs its launches name
    hipGraphExec_t bexec = nullptr;
    RenderKey bkey;
    const void *bkey_out[21] = {};  // gradient outputs, or the fused step's parameters and moments
    AdamScalars *adam_sc = nullptr;  // device: the fused optimiser step's scalars, one record per group
    bool bgraph_valid = false;
    bool last_graphed = false;  // the last render ran through the forward graph

    // kernel timing (HIP events around selected launches)
    bool profile = false;
    struct Pending {
        int which;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    double k_ms[kTimedKernels] = {};
    int64_t k_launches[kTimedKernels] = {};
};

namespace {

hgs_status fail(hgs_ctx *c, hgs_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIPC(call)                                                                                     \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(ctx, HGS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Queues the copy of `bytes` host bytes (at most the size of kMaxViews view
// records) to dst on st.  The DMA reads a pinned staging slot, not src: the
// copy may run long after this returns (behind earlier work on st), and the
// host bytes may change meanwhile.  A slot is reused only once its previous
// copy has run.  Called through stage_records, which counts in records.
hgs_status stage_bytes(hgs_ctx *ctx, const void *src, size_t bytes, void *dst, hipStream_t st)
{
    const int k = ctx->stage_next;
    ctx->stage_next = (k + 1) % kStageRing;
    if (ctx->stage_used[k]) HIPC(hipEventSynchronize(ctx->stage_ev[k]));
    memcpy(ctx->stage[k], src, bytes);
    HIPC(hipMemcpyAsync(dst, ctx->stage[k], bytes, hipMemcpyHostToDevice, st));
    HIPC(hipEventRecord(ctx->stage_ev[k], st));
    ctx->stage_used[k] = true;
    return HGS_OK;
}

// stage_bytes for n records of type T
template <typename T>
hgs_status stage_records(hgs_ctx *ctx, const T *src, size_t n, T *dst, hipStream_t st)
{
    static_assert(sizeof(T) <= sizeof(DevView) * kMaxViews, "staging slot");
    return stage_bytes(ctx, src, sizeof(T) * n, dst, st);
}

hgs_status push_views(hgs_ctx *ctx, int n, hipStream_t st)
{
    return stage_records(ctx, ctx->views_host, (size_t)n, ctx->views_dev, st);
}

hgs_status dalloc(hgs_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, HGS_ERR_OOM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    ctx->allocs.push_back(*p);
    return HGS_OK;
}

void dfree(hgs_ctx *ctx, void *p)
{
    if (!p) return;
    auto it = std::find(ctx->allocs.begin(), ctx->allocs.end(), p);
    if (it != ctx->allocs.end()) ctx->allocs.erase(it);
    (void)hipFree(p);
}

template <typename T>
hgs_status realloc_buf(hgs_ctx *ctx, T *&p, size_t count)
{
    dfree(ctx, p);
    p = nullptr;
    void *q = nullptr;
    hgs_status s = dalloc(ctx, &q, count * sizeof(T));
    p = (T *)q;
    return s;
}

hipEvent_t take_event(hgs_ctx *ctx)
{
    if (!ctx->event_pool.empty()) {
        hipEvent_t e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when profiling is on.
struct KernelTimer {
    hgs_ctx *ctx;
    int which;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    KernelTimer(hgs_ctx *c, int w, hipStream_t s) : ctx(c), which(w), st(s)
    {
        if (!ctx->profile) return;
        a = take_event(ctx);
        b = take_event(ctx);
        if (a) (void)hipEventRecord(a, st);
    }
    ~KernelTimer()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        ctx->pending.push_back({which, a, b});
    }
};

void collect_times(hgs_ctx *ctx)
{
    for (auto &p : ctx->pending) {
        (void)hipEventSynchronize(p.b);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->k_ms[p.which] += ms;
            ctx->k_launches[p.which] += 1;
        }
        ctx->event_pool.push_back(p.a);
        ctx->event_pool.push_back(p.b);
    }
    ctx->pending.clear();
}

DevHier dev_hier(const hgs_ctx *c)
{
    DevHier h;
    h.n = c->n;
    h.pinfo = c->pinfo;
    h.box = c->box;
    h.child_count = c->child_count;
    h.child_begin = c->child_begin;
    float *const *P = c->use_bound ? c->bound : c->own;
    h.mean = P[0];
    h.scale = P[1];
    h.rot = P[2];
    h.opacity = P[3];
    h.sh = P[4];
    h.slot = nullptr;
    if (c->streaming) {
        h.mean = c->cache_params.mean;
        h.scale = c->cache_params.scale;
        h.rot = c->cache_params.rot;
        h.opacity = c->cache_params.opacity;
        h.sh = c->cache_params.sh;
        h.slot = c->sd.slot;
    }
    return h;
}

int cut_blocks(int64_t n) { return (int)((n + kCutBlock - 1) / kCutBlock); }

bool finite_view(const hgs_view &v)
{
    for (float x : v.R)
        if (!std::isfinite(x)) return false;
    for (float x : v.eye)
        if (!std::isfinite(x)) return false;
    return std::isfinite(v.fx) && std::isfinite(v.fy) && std::isfinite(v.cx) && std::isfinite(v.cy) &&
           std::isfinite(v.z_near) && std::isfinite(v.tau) && v.fx > 0 && v.fy > 0 && v.z_near > 0 && v.tau >= 0 &&
           v.width > 0 && v.height > 0 && v.width <= 32768 && v.height <= 32768;
}

// The device record of one view (tile grid at tw x th, bases and output
// pointers left for the caller).
void fill_dev_view(const hgs_view &s, int tw, int th, DevView &d)
{
    memcpy(d.R, s.R, sizeof d.R);
    memcpy(d.eye, s.eye, sizeof d.eye);
    d.fx = s.fx;
    d.fy = s.fy;
    d.cx = s.cx;
    d.cy = s.cy;
    d.W = s.width;
    d.H = s.height;
    d.z_near = s.z_near;
    d.tau = s.tau;
    {
        // eps <= tau  <=>  L^2 <= (tau / f)^2 d^2; the prefilter decides it
        // in FP32 outside a band of kCutMargin and stays off (NaN) where the
        // constant is so small or large that FP32 products could leave the
        // normal range
        const double f = s.fx > s.fy ? s.fx : s.fy, k = (double)s.tau * (double)s.tau / (f * f);
        const bool use = s.tau == 0.0f || (k >= 1e-12 && k <= 1e12);
        d.cut_klo = use ? (float)(k * (1.0 - (double)kCutMargin)) : NAN;
        d.cut_khi = use ? (float)(k * (1.0 + (double)kCutMargin)) : NAN;
    }
    d.tiles_x = (s.width + tw - 1) / tw;
    d.tiles_y = (s.height + th - 1) / th;
    d.tile_base = 0;
    d.pix_base = 0;
    d.out_rgb = nullptr;
    d.dL = nullptr;
    d.target = nullptr;
}

// Per-view device records and global tile/pixel bases.
hgs_status setup_views(hgs_ctx *ctx, const hgs_view *views, int nv, float *const *out_rgb, uint32_t &n_tiles,
                       size_t &n_pix)
{
    n_tiles = 0;
    n_pix = 0;
    for (int v = 0; v < nv; ++v) {
        const hgs_view &s = views[v];
        if (!finite_view(s)) return fail(ctx, HGS_ERR_INVALID_ARG, "view " + std::to_string(v) + " is invalid");
        DevView &d = ctx->views_host[v];
        fill_dev_view(s, ctx->tile_w, ctx->tile_h, d);
        d.tile_base = n_tiles;
        d.pix_base = (uint32_t)n_pix;
        d.out_rgb = out_rgb ? out_rgb[v] : nullptr;
        d.dL = nullptr;
        d.target = nullptr;
        const uint64_t nt = (uint64_t)d.tiles_x * d.tiles_y;
        if ((uint64_t)n_tiles + nt >= (1ull << 31)) return fail(ctx, HGS_ERR_INVALID_ARG, "too many tiles");
        n_tiles += (uint32_t)nt;
        n_pix += (size_t)s.width * s.height;
        if (n_pix >= (1ull << 32)) return fail(ctx, HGS_ERR_INVALID_ARG, "too many pixels");
    }
    return HGS_OK;
}

hgs_status ensure_fixed(hgs_ctx *ctx, int nv, uint32_t n_tiles, size_t n_pix)
{
    hgs_status s;
    const int nb = cut_blocks(ctx->n);
    if (nv > ctx->nv_cap || nb > ctx->nblocks_cap) {
        const int nvc = std::max(nv, ctx->nv_cap), nbc = std::max(nb, ctx->nblocks_cap);
        const size_t words = (size_t)((ctx->n + 63) / 64);
        if ((s = realloc_buf(ctx, ctx->masks, words * nvc + 1))) return s;
        if ((s = realloc_buf(ctx, ctx->word_off, words * nvc + 1))) return s;
        if ((s = realloc_buf(ctx, ctx->blk_counts, (size_t)nbc * nvc))) return s;
        if ((s = realloc_buf(ctx, ctx->blk_offsets, (size_t)nbc * nvc))) return s;
        if ((s = realloc_buf(ctx, ctx->cut_base, (size_t)nvc + 1))) return s;
        ctx->nv_cap = nvc;
        ctx->nblocks_cap = nbc;
        ctx->layout_gen++;
    }
    if (n_tiles > ctx->tile_cap) {
        if ((s = realloc_buf(ctx, ctx->ranges, n_tiles))) return s;
        if ((s = realloc_buf(ctx, ctx->tile_keys, n_tiles))) return s;
        if ((s = realloc_buf(ctx, ctx->tile_order, n_tiles))) return s;
        if ((s = realloc_buf(ctx, ctx->tile_k2, n_tiles))) return s;
        if ((s = realloc_buf(ctx, ctx->tile_v2, n_tiles))) return s;
        if (!ctx->tile_n && (s = realloc_buf(ctx, ctx->tile_n, 4))) return s;
        ctx->tile_cap = n_tiles;
        ctx->layout_gen++;
    }
    const size_t n_waves = (size_t)n_tiles * (size_t)(ctx->tile_w * ctx->tile_h / 64);
    if (n_waves > ctx->wstats_cap) {
        if ((s = realloc_buf(ctx, ctx->wstats, n_waves))) return s;
        ctx->wstats_cap = n_waves;
        ctx->layout_gen++;
    }
    if (n_pix > ctx->pix_cap) {
        if ((s = realloc_buf(ctx, ctx->T_final, n_pix))) return s;
        if ((s = realloc_buf(ctx, ctx->n_last, n_pix))) return s;
        if ((s = realloc_buf(ctx, ctx->n_blend, n_pix))) return s;
        ctx->pix_cap = n_pix;
        ctx->layout_gen++;
    }
    return HGS_OK;
}

hgs_status ensure_cut_cap(hgs_ctx *ctx, uint32_t cap)
{
    if (cap <= ctx->cut_cap) return HGS_OK;
    hgs_status s;
    if ((s = realloc_buf(ctx, ctx->cut_ids, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->cut_t, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->recs, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->axes, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->depth_key, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->ntiles, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->rect, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->jrank, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->trec, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->vis_mask, (size_t)cap / 64 + 8))) return s;
    if ((s = realloc_buf(ctx, ctx->vis_counts, (size_t)cap / 256 + 2))) return s;
    if ((s = realloc_buf(ctx, ctx->vis_offsets, (size_t)cap / 256 + 2))) return s;
    if ((s = realloc_buf(ctx, ctx->skeys, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->svals, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->pair_offsets, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->sgrad, (size_t)cap * 12))) return s;
    if ((s = realloc_buf(ctx, ctx->vis_rank, (size_t)cap))) return s;
    if ((s = realloc_buf(ctx, ctx->vis_entry, (size_t)cap))) return s;
    if ((s = realloc_buf(ctx, ctx->pgrad, (size_t)cap * kPGradFloats))) return s;
    if ((s = realloc_buf(ctx, ctx->cjac, (size_t)cap * 12))) return s;
    ctx->cut_cap = cap;
    const size_t scratch = std::max<size_t>(ctx->cut_cap, ctx->pair_cap);
    if ((s = realloc_buf(ctx, ctx->k2, scratch))) return s;
    if ((s = realloc_buf(ctx, ctx->v2, scratch))) return s;
    ctx->layout_gen++;
    return HGS_OK;
}

hgs_status ensure_pair_cap(hgs_ctx *ctx, uint32_t cap)
{
    if (cap <= ctx->pair_cap) return HGS_OK;
    hgs_status s;
    if ((s = realloc_buf(ctx, ctx->pkeys, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->pvals, cap))) return s;
    if ((s = realloc_buf(ctx, ctx->qbits, (size_t)cap * kMaxBlocks))) return s;
    if ((s = realloc_buf(ctx, ctx->dup_first, (size_t)duplicate_blocks(cap) + 1))) return s;
    ctx->pair_cap = cap;
    const size_t scratch = std::max<size_t>(ctx->cut_cap, ctx->pair_cap);
    if ((s = realloc_buf(ctx, ctx->k2, scratch))) return s;
    if ((s = realloc_buf(ctx, ctx->v2, scratch))) return s;
    ctx->layout_gen++;
    return HGS_OK;
}

int bits_for(uint32_t n)
{
    int b = 1;
    while (b < 32 && (1ull << b) < n) ++b;
    return b;
}

// The whole forward for nv views, queued on st.  `ev` (9 events, optional)
// marks stage boundaries.
void enqueue_blend(hgs_ctx *ctx, int nv, uint32_t n_tiles, hipStream_t st)
{
    const uint32_t *vals = ctx->pairs_in_scratch ? ctx->v2 : ctx->pvals;
    launch_blend(ctx->views_dev, nv, n_tiles, ctx->tile_sorted, ctx->ranges, vals, ctx->recs, ctx->axes, ctx->T_final,
                 ctx->n_last, ctx->n_blend, ctx->qbits, ctx->pair_cap, ctx->wstats, ctx->ctr, ctx->tile_w,
                 ctx->tile_h, ctx->batch, ctx->persist, ctx->queue, st);
}

void enqueue_forward(hgs_ctx *ctx, int nv, uint32_t n_tiles, hipStream_t st, hipEvent_t *ev, bool with_blend)
{
    const DevHier h = dev_hier(ctx);
    const int nb = cut_blocks(ctx->n);
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], st);
    };
    mark(0);
    launch_fill_u32((uint32_t *)ctx->ctr, 0u, sizeof(Counters) / 4, st);
    launch_cut_flags(h, ctx->views_dev, nv, ctx->masks, ctx->blk_counts, nb, st);
    launch_scan(ctx->blk_counts, nullptr, (uint32_t)(nb * nv), nullptr, ctx->blk_offsets, &ctx->ctr->cut_total,
                ctx->partial, st);
    launch_cut_emit(h, ctx->views_dev, nv, ctx->masks, ctx->blk_offsets, nb, ctx->word_off, ctx->cut_ids, nullptr,
                    ctx->cut_t,
                    ctx->cut_cap, st);
    launch_cut_finish(ctx->blk_offsets, ctx->blk_counts, nb, nv, ctx->cut_base, ctx->ctr, st);
    if (ctx->streaming)  // the cut's nodes and parents made resident in the cache
        launch_stream_frame(ctx->sd, ctx->pinfo, ctx->cut_ids, &ctx->ctr->cut_total, ctx->cut_cap,
                            ctx->host_params_dev, ctx->cache_params, st);
    mark(1);
    launch_preprocess(h, ctx->views_dev, nv, ctx->cut_base, ctx->cut_ids, ctx->cut_t, &ctx->ctr->cut_total,
                      ctx->cut_cap, ctx->recs, ctx->axes, ctx->depth_key, ctx->trec, ctx->ntiles, ctx->cjac,
                      ctx->vis_mask,
                      ctx->vis_counts, ctx->tile_w, ctx->tile_h, st);
    mark(2);
    const uint32_t vblocks = (ctx->cut_cap + 255) / 256;
    launch_scan(ctx->vis_counts, nullptr, vblocks, nullptr, ctx->vis_offsets, &ctx->ctr->vis_total, ctx->partial, st);
    launch_compact_visible(ctx->vis_mask, ctx->vis_offsets, &ctx->ctr->cut_total, ctx->cut_cap, ctx->depth_key,
                           ctx->skeys, ctx->svals, ctx->vis_rank, ctx->vis_entry, st);
    // the visible splats keep the cut's view-major order: each view's run is
    // sorted by depth on its own (4 passes, in place), so that its pairs are
    // emitted as one run, which the tile sort then orders by the view's own
    // tile id (16 bits or fewer: 2 passes)
    SortScratch sc{ctx->k2, ctx->v2, ctx->hist, ctx->hist_scan, ctx->partial, ctx->scan_total, ctx->sort_plan};
    launch_vis_bounds(ctx->cut_base, nv, ctx->vis_mask, ctx->vis_offsets, &ctx->ctr->cut_total, ctx->cut_cap,
                      &ctx->ctr->vis_total, ctx->vis_bounds, st);
    launch_radix_sort(ctx->skeys, ctx->svals, ctx->cut_cap, &ctx->ctr->vis_total, 32, sc, st, ctx->vis_bounds, nv);
    mark(3);
    launch_gather_tiles(ctx->trec, ctx->svals, &ctx->ctr->vis_total, ctx->cut_cap, ctx->pair_offsets, ctx->rect,
                        ctx->jrank, st);
    launch_scan(ctx->pair_offsets, nullptr, ctx->cut_cap, &ctx->ctr->vis_total, ctx->pair_offsets,
                &ctx->ctr->pair_total, ctx->partial, st);  // in place
    launch_pair_bounds(ctx->vis_bounds, ctx->views_dev, nv, ctx->pair_offsets, &ctx->ctr->vis_total, ctx->cut_cap,
                       &ctx->ctr->pair_total, ctx->pair_cap, ctx->pair_bounds, ctx->seg_tile_base, st);
    launch_duplicate(ctx->rect, ctx->views_dev, nv, ctx->cut_base, ctx->svals, ctx->pair_offsets, ctx->dup_first,
                     &ctx->ctr->vis_total, ctx->cut_cap, &ctx->ctr->pair_total, ctx->pair_cap, ctx->pkeys,
                     ctx->pvals, ctx->ctr, st);
    mark(4);
    uint32_t view_tiles = 1;  // tiles of the largest view
    for (int v = 0; v < nv; ++v)
        view_tiles = std::max(view_tiles, (uint32_t)(ctx->views_host[v].tiles_x * ctx->views_host[v].tiles_y));
    ctx->pairs_in_scratch = launch_radix_sort(ctx->pkeys, ctx->pvals, ctx->pair_cap, &ctx->ctr->pair_total,
                                              bits_for(view_tiles), sc, st, ctx->pair_bounds, nv, ctx->seg_tile_base);
    mark(5);
    const uint32_t *keys = ctx->pairs_in_scratch ? ctx->k2 : ctx->pkeys;
    const uint32_t *vals = ctx->pairs_in_scratch ? ctx->v2 : ctx->pvals;
    launch_fill_u32((uint32_t *)ctx->ranges, 0u, (size_t)n_tiles * 2, st);
    launch_ranges(keys, &ctx->ctr->pair_total, ctx->pair_cap, ctx->ranges, st);
    // longest tile lists first (one stable 8-bit pass over log-scaled lengths)
    launch_tile_keys(ctx->ranges, n_tiles, ctx->tile_keys, ctx->tile_order, ctx->tile_n, st);
    {
        SortScratch ts{ctx->tile_k2, ctx->tile_v2, ctx->hist, ctx->hist_scan, ctx->partial, ctx->scan_total,
                       ctx->sort_plan};
        const bool in_scratch = launch_radix_sort(ctx->tile_keys, ctx->tile_order, n_tiles, ctx->tile_n, 8, ts, st);
        ctx->tile_sorted = in_scratch ? ctx->tile_v2 : ctx->tile_order;
    }
    (void)vals;
    mark(6);
    if (with_blend) {
        KernelTimer kt(ctx, 0, st);
        enqueue_blend(ctx, nv, n_tiles, st);
    }
    mark(7);
}

// Frees the hierarchy's buffers (topology, boxes, parameters, interior list).
void stream_release(hgs_ctx *ctx)
{
    if (!ctx->streaming) return;
    void **bufs[] = {(void **)&ctx->sd.slot, (void **)&ctx->sd.node_in_slot, (void **)&ctx->sd.last_used,
                     (void **)&ctx->sd.free_stack, (void **)&ctx->sd.free_top, (void **)&ctx->sd.req,
                     (void **)&ctx->cache_params.mean, (void **)&ctx->cache_params.scale,
                     (void **)&ctx->cache_params.rot, (void **)&ctx->cache_params.opacity,
                     (void **)&ctx->cache_params.sh};
    for (void **b : bufs) {
        dfree(ctx, *b);
        *b = nullptr;
    }
    if (ctx->host_block) (void)hipHostFree(ctx->host_block);
    ctx->host_block = nullptr;
    ctx->host_params = ctx->host_params_dev = StreamParams{};
    ctx->sd = StreamDev{};
    ctx->streaming = false;
}

void drop_hierarchy(hgs_ctx *ctx)
{
    stream_release(ctx);
    for (int k = 0; k < 5; ++k) {
        dfree(ctx, ctx->own[k]);
        ctx->own[k] = nullptr;
        ctx->bound[k] = nullptr;
    }
    void **bufs[] = {(void **)&ctx->pinfo, (void **)&ctx->box, (void **)&ctx->child_count,
                     (void **)&ctx->child_begin, (void **)&ctx->interior, (void **)&ctx->leaf_src};
    for (void **b : bufs) {
        dfree(ctx, *b);
        *b = nullptr;
    }
    ctx->use_bound = false;
    ctx->has_hier = false;
    ctx->have_render = false;
}

// The backward of the last render, queued on st: screen-gradient rows and
// counters cleared, blend backward, preprocess backward and the gather into
// the gradient outputs.  Every size it launches with is a capacity or a
// count the kernels read on the device, so that a captured copy stays valid
// for every render of the same forward graph.
// With `fused` the gather applies the optimiser step instead of writing
// gradients (out is then unused).
void enqueue_backward(hgs_ctx *ctx, int nv, const hgs_grads *out, const AdamRows *fused, hipStream_t st)
{
    const bool det = ctx->deterministic;
    if (det)  // every row of the emitted pair list is written or stays zero
        launch_zero_rows(ctx->part, 11, &ctx->ctr->pair_total, ctx->pair_cap, st);
    else
        launch_zero_rows(ctx->sgrad, 12, &ctx->ctr->vis_total, ctx->cut_cap, st);
    launch_fill_u32((uint32_t *)&ctx->ctr->bwd_evaluated, 0u, 6, st);
    const uint32_t *vals = ctx->pairs_in_scratch ? ctx->v2 : ctx->pvals;
    {
        KernelTimer kt(ctx, 1, st);
        const DetArgs da{ctx->jrank, ctx->pair_offsets, ctx->rect, ctx->part};
        launch_blend_backward(ctx->views_dev, nv, ctx->last_tiles, ctx->tile_sorted, ctx->ranges, vals, ctx->recs,
                              ctx->axes, ctx->T_final, ctx->n_last, ctx->qbits, ctx->pair_cap, ctx->vis_rank,
                              ctx->sgrad, det ? &da : nullptr, ctx->wstats, ctx->ctr, ctx->r_tw, ctx->r_th,
                              ctx->r_batch, out && out->dt != nullptr, ctx->r_persist, ctx->queue + 1, st);
        if (det)
            launch_det_sum(ctx->part, ctx->pair_offsets, ctx->svals, ctx->vis_rank, &ctx->ctr->vis_total,
                           ctx->cut_cap, &ctx->ctr->pair_total, ctx->pair_cap, ctx->sgrad, st);
    }
    const DevHier h = dev_hier(ctx);
    {
        KernelTimer kt(ctx, 2, st);
        launch_preprocess_backward(h, ctx->views_dev, nv, ctx->cut_base, ctx->cut_ids, ctx->cut_t,
                                   &ctx->ctr->cut_total, ctx->cut_cap, ctx->ntiles, ctx->recs, ctx->cjac,
                                   ctx->vis_entry, &ctx->ctr->vis_total, ctx->sgrad, ctx->pgrad, ctx->masks,
                                   (ctx->n + 63) / 64,
                                   ctx->word_off, ctx->interior, ctx->n_interior, out ? out->mean : nullptr,
                                   out ? out->scale : nullptr, out ? out->rot : nullptr,
                                   out ? out->opacity : nullptr, out ? out->sh : nullptr, out ? out->dt : nullptr,
                                   fused, st);
    }
}

// ------------------------------------------------ allocation-free cut
// Scratch of hgs_cut_noalloc in a file-scope device array: every device the
// library runs on holds one copy until the process ends.  It covers
// hierarchies of up to kNoAllocMaxNodes nodes: the cut's bit masks and mask
// word positions, its per-block counts and offsets, the scan partials, the
// counters and the view record.  In host code `scratch` names a host-side
// stand-in, never the device memory: its device address comes from
// hipGetSymbolAddress, once per device (g_scratch), and only that address is
// handed to kernels and copies.
constexpr int64_t kNoAllocMaxNodes = int64_t(1) << 26;
constexpr size_t kNaWords = (size_t)(kNoAllocMaxNodes / 64) + 1;
constexpr size_t kNaBlocks = (size_t)(kNoAllocMaxNodes / kCutBlock);
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaMasks = 0;
constexpr size_t kNaWordOff = align256(kNaMasks + 8 * kNaWords);
constexpr size_t kNaCounts = align256(kNaWordOff + 4 * kNaWords);
constexpr size_t kNaOffsets = align256(kNaCounts + 4 * kNaBlocks);
constexpr size_t kNaPartial = align256(kNaOffsets + 4 * kNaBlocks);
constexpr size_t kNaCtr = align256(kNaPartial + 4 * (size_t)kScanBlocks);
constexpr size_t kNaView = align256(kNaCtr + sizeof(Counters));
constexpr size_t kNaBytes = align256(kNaView + sizeof(DevView));
static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned char *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

// With ctx->device current: looks up this device's copy of the scratch once.
hgs_status scratch_init(hgs_ctx *ctx)
{
    if (ctx->device >= kMaxDevices) return fail(ctx, HGS_ERR_INVALID_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[ctx->device]) return HGS_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(ctx, HGS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch[ctx->device] = (unsigned char *)p;
    return HGS_OK;
}

unsigned char *scratch_of(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return device >= 0 && device < kMaxDevices ? g_scratch[device] : nullptr;
}

}  // namespace

extern "C" {

hgs_status hgs_create(hgs_ctx **out, int device, void *hip_stream)
{
    if (!out) return HGS_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return HGS_ERR_INVALID_ARG;
    }
    hgs_ctx *ctx = new hgs_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    hgs_status s = HGS_OK;
    do {
        if (hipSetDevice(device) != hipSuccess) { s = HGS_ERR_HIP; break; }
        if (hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking) != hipSuccess) { s = HGS_ERR_HIP; break; }
        if (hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess) { s = HGS_ERR_HIP; break; }
        if (hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess) { s = HGS_ERR_HIP; break; }
        ctx->views_host = new (std::nothrow) DevView[kMaxViews];
        if (!ctx->views_host) { s = HGS_ERR_OOM; break; }
        for (int k = 0; k < kStageRing && s == HGS_OK; ++k) {
            if (hipHostMalloc((void **)&ctx->stage[k], sizeof(DevView) * kMaxViews, hipHostMallocDefault) != hipSuccess)
                s = HGS_ERR_OOM;
            else if (hipEventCreateWithFlags(&ctx->stage_ev[k], hipEventDisableTiming) != hipSuccess)
                s = HGS_ERR_HIP;
        }
        if (s != HGS_OK) break;
        if (hipHostMalloc((void **)&ctx->ctr_host, sizeof(Counters), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ctx->stream_host, 32, hipHostMallocDefault) != hipSuccess) {
            s = HGS_ERR_OOM;
            break;
        }
        if ((s = dalloc(ctx, (void **)&ctx->views_dev, sizeof(DevView) * kMaxViews))) break;
        if ((s = dalloc(ctx, (void **)&ctx->ctr, sizeof(Counters)))) break;
        if ((s = dalloc(ctx, (void **)&ctx->hist, sizeof(uint32_t) * 256 * kSortBlocksMax))) break;
        if ((s = dalloc(ctx, (void **)&ctx->hist_scan, sizeof(uint32_t) * 256 * kSortBlocksMax))) break;
        if ((s = dalloc(ctx, (void **)&ctx->partial, sizeof(uint32_t) * kScanBlocks))) break;
        if ((s = dalloc(ctx, (void **)&ctx->scan_total, sizeof(uint32_t) * 4))) break;
        if ((s = dalloc(ctx, (void **)&ctx->sort_plan, sizeof(SortBlock) * kSortBlocksMax))) break;
        if ((s = dalloc(ctx, (void **)&ctx->vis_bounds, sizeof(uint32_t) * (kMaxViews + 1)))) break;
        if ((s = dalloc(ctx, (void **)&ctx->pair_bounds, sizeof(uint32_t) * (kMaxViews + 1)))) break;
        if ((s = dalloc(ctx, (void **)&ctx->seg_tile_base, sizeof(uint32_t) * kMaxViews))) break;
        if ((s = dalloc(ctx, (void **)&ctx->queue, sizeof(uint32_t) * 2))) break;
        if ((s = dalloc(ctx, (void **)&ctx->l1_partial, sizeof(double) * kL1Blocks))) break;
        if ((s = dalloc(ctx, (void **)&ctx->adam_sc, sizeof(AdamScalars) * 5))) break;
        if ((s = scratch_init(ctx))) break;
    } while (0);
    if (s != HGS_OK) {
        hgs_destroy(ctx);
        return s;
    }
    *out = ctx;
    return HGS_OK;
}

void hgs_destroy(hgs_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->gstream) (void)hipStreamSynchronize(ctx->gstream);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->bexec) (void)hipGraphExecDestroy(ctx->bexec);
    if (ctx->host_block) (void)hipHostFree(ctx->host_block);
    if (ctx->stream_host) (void)hipHostFree(ctx->stream_host);
    collect_times(ctx);
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    for (void *p : ctx->allocs) (void)hipFree(p);
    ctx->allocs.clear();
    delete[] ctx->views_host;
    for (int k = 0; k < kStageRing; ++k) {
        if (ctx->stage[k]) (void)hipHostFree(ctx->stage[k]);
        if (ctx->stage_ev[k]) (void)hipEventDestroy(ctx->stage_ev[k]);
    }
    if (ctx->ctr_host) (void)hipHostFree(ctx->ctr_host);
    if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    delete ctx;
}

const char *hgs_last_error(const hgs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hgs_status hgs_set_stream(hgs_ctx *ctx, void *hip_stream)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return HGS_OK;
}

// Checks the optimiser arguments (the gradient arrays only when `grads`)
// and fills the scalars of the five groups.
static hgs_status check_adam(hgs_ctx *ctx, const hgs_adam *a, bool grads, AdamScalars sc[5])
{
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (ctx->streaming) return fail(ctx, HGS_ERR_STATE, "no optimiser step while rendering out of core");
    if (!a) return fail(ctx, HGS_ERR_INVALID_ARG, "NULL optimiser arguments");
    for (int k = 0; k < 5; ++k) {
        if (!a->param[k] || (grads && !a->grad[k]) || !a->m[k] || !a->v[k])
            return fail(ctx, HGS_ERR_INVALID_ARG, "NULL array of parameter group " + std::to_string(k));
        if (!std::isfinite(a->lr[k]) || a->lr[k] < 0.0f)
            return fail(ctx, HGS_ERR_INVALID_ARG, "bad learning rate of parameter group " + std::to_string(k));
        // rotation and SH rows are stepped in 16-byte vectors
        const void *arrs[4] = {a->param[k], grads ? a->grad[k] : nullptr, a->m[k], a->v[k]};
        if (k == 2 || k == 4)
            for (const void *q : arrs)
                if (reinterpret_cast<uintptr_t>(q) % 16 != 0)
                    return fail(ctx, HGS_ERR_INVALID_ARG, "array of parameter group " + std::to_string(k) +
                                                              " not 16-byte aligned");
    }
    if (a->step < 1 || !(a->beta1 >= 0.0f && a->beta1 < 1.0f) || !(a->beta2 >= 0.0f && a->beta2 < 1.0f) ||
        !(a->eps > 0.0f) || !std::isfinite(a->eps))
        return fail(ctx, HGS_ERR_INVALID_ARG, "bad step, beta1, beta2 or eps");
    const double bc1 = 1.0 / (1.0 - std::pow((double)a->beta1, (double)a->step));
    const double bc2 = 1.0 / (1.0 - std::pow((double)a->beta2, (double)a->step));
    for (int k = 0; k < 5; ++k) sc[k] = AdamScalars{a->lr[k], a->beta1, a->beta2, a->eps, (float)bc1, (float)bc2};
    return HGS_OK;
}

// stepping the parameters the renderer reads makes the last render stale
static void adam_stepped(hgs_ctx *ctx, const hgs_adam *a)
{
    for (int k = 0; k < 5; ++k)
        if (a->param[k] == (ctx->use_bound ? ctx->bound[k] : ctx->own[k])) ctx->have_render = false;
}

hgs_status hgs_adam_step(hgs_ctx *ctx, const hgs_adam *a)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    AdamScalars sc[5];
    if (hgs_status s = check_adam(ctx, a, true, sc)) return s;
    HIPC(hipSetDevice(ctx->device));
    adam_stepped(ctx, a);
    for (int k = 0; k < 5; ++k)
        launch_adam(k, ctx->interior, ctx->n_interior, a->param[k], a->grad[k], a->m[k], a->v[k], sc[k],
                    ctx->stream);
    HIPC(hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_set_deterministic(hgs_ctx *ctx, int32_t on)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (on != 0 && on != 1) return fail(ctx, HGS_ERR_INVALID_ARG, "on must be 0 or 1");
    ctx->deterministic = on != 0;
    ctx->bgraph_valid = false;  // the captured backward follows the mode
    return HGS_OK;
}

hgs_status hgs_interior(hgs_ctx *ctx, int32_t *ids, int64_t cap, int64_t *count)
{
    if (!ctx || !count) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (cap < 0) return fail(ctx, HGS_ERR_INVALID_ARG, "negative capacity");
    *count = ctx->n_interior;
    if (ids && cap > 0 && ctx->n_interior > 0) {
        HIPC(hipSetDevice(ctx->device));
        const size_t n = (size_t)std::min<int64_t>(cap, ctx->n_interior);
        HIPC(hipMemcpyAsync(ids, ctx->interior, 4 * n, hipMemcpyDeviceToDevice, ctx->stream));
    }
    return HGS_OK;
}

hgs_status hgs_set_tuning(hgs_ctx *ctx, int32_t tile_w, int32_t tile_h, int32_t batch, int32_t persistent)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!blend_supported(tile_w, tile_h, batch))
        return fail(ctx, HGS_ERR_INVALID_ARG, "unsupported tile/batch combination");
    if (persistent != 0 && persistent != 1) return fail(ctx, HGS_ERR_INVALID_ARG, "persistent must be 0 or 1");
    ctx->tile_w = tile_w;
    ctx->tile_h = tile_h;
    ctx->batch = batch == tile_w * tile_h ? 0 : batch;
    ctx->persist = persistent != 0;
    ctx->have_render = false;
    return HGS_OK;
}

hgs_status hgs_upload(hgs_ctx *ctx, const hgs_hierarchy_desc *d, int src_on_device)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!d) return fail(ctx, HGS_ERR_INVALID_ARG, "desc is NULL");
    HIPC(hipSetDevice(ctx->device));
    const int64_t N = d->n_nodes;
    if (N <= 0 || N >= (int64_t)kRootParent) return fail(ctx, HGS_ERR_INVALID_ARG, "n_nodes out of range");
    if (d->sh_degree != 3) return fail(ctx, HGS_ERR_INVALID_ARG, "only sh_degree 3 is supported");
    const void *ptrs[] = {d->parent, d->child_begin, d->child_count, d->bmin, d->bmax,
                          d->mean,   d->scale,       d->rot,         d->opacity, d->sh};
    for (const void *p : ptrs)
        if (!p) return fail(ctx, HGS_ERR_INVALID_ARG, "NULL array in desc");
    // topology and boxes to the host for validation
    std::vector<int32_t> par(N), cb(N), cc(N);
    std::vector<float> bmin(3 * N), bmax(3 * N);
    const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
    HIPC(hipMemcpy(par.data(), d->parent, 4 * N, kind));
    HIPC(hipMemcpy(cb.data(), d->child_begin, 4 * N, kind));
    HIPC(hipMemcpy(cc.data(), d->child_count, 4 * N, kind));
    HIPC(hipMemcpy(bmin.data(), d->bmin, 12 * N, kind));
    HIPC(hipMemcpy(bmax.data(), d->bmax, 12 * N, kind));
    ctx->has_hier = false;
    ctx->have_render = false;
    if (par[0] != -1) return fail(ctx, HGS_ERR_INVALID_ARG, "parent[0] must be -1 (root first)");
    int64_t kids = 0, leaves = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (i > 0 && (par[i] < 0 || par[i] >= i))
            return fail(ctx, HGS_ERR_INVALID_ARG, "parent[" + std::to_string(i) + "] must lie in [0, i)");
        if (cc[i] < 0) return fail(ctx, HGS_ERR_INVALID_ARG, "negative child_count");
        if (cc[i] == 0) {
            ++leaves;
        } else {
            if (cb[i] <= i || (int64_t)cb[i] + cc[i] > N)
                return fail(ctx, HGS_ERR_INVALID_ARG, "child range of node " + std::to_string(i) + " out of bounds");
            for (int32_t k = 0; k < cc[i]; ++k)
                if (par[cb[i] + k] != i)
                    return fail(ctx, HGS_ERR_INVALID_ARG,
                                "children of node " + std::to_string(i) + " are not contiguous");
            kids += cc[i];
        }
        for (int k = 0; k < 3; ++k) {
            const float lo = bmin[3 * i + k], hi = bmax[3 * i + k];
            if (!(lo <= hi) || !std::isfinite(lo) || !std::isfinite(hi))
                return fail(ctx, HGS_ERR_INVALID_ARG, "box of node " + std::to_string(i) + " is invalid");
        }
    }
    if (kids != N - 1) return fail(ctx, HGS_ERR_INVALID_ARG, "child counts do not cover every non-root node once");
    std::vector<uint32_t> pinfo(N);
    for (int64_t i = 0; i < N; ++i)
        pinfo[i] = (i == 0 ? kRootParent : (uint32_t)par[i]) | (cc[i] == 0 ? kLeafBit : 0u);

    // (re)allocate hierarchy buffers
    drop_hierarchy(ctx);
    hgs_status s;
    if ((s = dalloc(ctx, (void **)&ctx->pinfo, 4 * N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->box, 24 * N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->child_count, 4 * N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->child_begin, 4 * N))) return s;
    std::vector<int32_t> interior;
    interior.reserve((size_t)(N - leaves));
    for (int64_t i = 0; i < N; ++i)
        if (cc[i] > 0) interior.push_back((int32_t)i);
    if ((s = dalloc(ctx, (void **)&ctx->interior, 4 * std::max<size_t>(interior.size(), 1)))) return s;
    const size_t comp[5] = {3, 3, 4, 1, 48};
    const float *src[5] = {d->mean, d->scale, d->rot, d->opacity, d->sh};
    for (int k = 0; k < 5; ++k)
        if ((s = dalloc(ctx, (void **)&ctx->own[k], 4 * comp[k] * N))) return s;
    HIPC(hipMemcpy(ctx->pinfo, pinfo.data(), 4 * N, hipMemcpyHostToDevice));
    {
        // the cut sweep reads the boxes component-major ([6][N]), one thread per node
        std::vector<float> box(6 * (size_t)N);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                box[k * N + i] = bmin[3 * i + k];
                box[(3 + k) * N + i] = bmax[3 * i + k];
            }
        HIPC(hipMemcpy(ctx->box, box.data(), 24 * N, hipMemcpyHostToDevice));
    }
    HIPC(hipMemcpy(ctx->child_count, cc.data(), 4 * N, hipMemcpyHostToDevice));
    for (int64_t i = 0; i < N; ++i)
        if (cc[i] == 0) cb[i] = 0;  // unused for leaves
    HIPC(hipMemcpy(ctx->child_begin, cb.data(), 4 * N, hipMemcpyHostToDevice));
    if (!interior.empty())
        HIPC(hipMemcpy(ctx->interior, interior.data(), 4 * interior.size(), hipMemcpyHostToDevice));
    ctx->n_interior = (int64_t)interior.size();
    const hipMemcpyKind k2 = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (int k = 0; k < 5; ++k) HIPC(hipMemcpy(ctx->own[k], src[k], 4 * comp[k] * N, k2));
    HIPC(hipDeviceSynchronize());
    ctx->n = N;
    ctx->n_leaves = leaves;
    ctx->has_hier = true;
    ctx->param_gen++;
    ctx->layout_gen++;
    // cut workspace sized for the hierarchy (the grid of the cut sweep depends on N)
    ctx->nblocks_cap = 0;
    ctx->nv_cap = 0;
    return HGS_OK;
}

hgs_status hgs_build(hgs_ctx *ctx, const hgs_leaves_desc *L, int src_on_device, int64_t *n_nodes)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!L || !n_nodes) return fail(ctx, HGS_ERR_INVALID_ARG, "leaves or n_nodes is NULL");
    const int64_t n = L->n_leaves;
    if (n < 1 || n > (int64_t)1 << 29) return fail(ctx, HGS_ERR_INVALID_ARG, "n_leaves out of [1, 2^29]");
    const void *in_ptrs[] = {L->mean, L->scale, L->rot, L->opacity, L->sh};
    for (const void *p : in_ptrs)
        if (!p) return fail(ctx, HGS_ERR_INVALID_ARG, "NULL leaf array");
    HIPC(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    HIPC(hipStreamSynchronize(st));
    // temporaries: freed on every exit
    std::vector<void *> tmp;
    auto talloc = [&](void **p, size_t bytes) -> hgs_status {
        *p = nullptr;
        const hipError_t e = hipMalloc(p, bytes ? bytes : 16);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, HGS_ERR_OOM, "hipMalloc(" + std::to_string(bytes) + ") in the hierarchy build");
        }
        tmp.push_back(*p);
        return HGS_OK;
    };
    struct Cleanup {
        std::vector<void *> &v;
        ~Cleanup()
        {
            for (void *p : v) (void)hipFree(p);
        }
    } cleanup{tmp};
    hgs_status s;
    const size_t comp[5] = {3, 3, 4, 1, 48};
    const float *in[5];
    for (int k = 0; k < 5; ++k) {
        if (src_on_device) {
            in[k] = (const float *)in_ptrs[k];
        } else {
            void *d = nullptr;
            if ((s = talloc(&d, 4 * comp[k] * (size_t)n))) return s;
            HIPC(hipMemcpyAsync(d, in_ptrs[k], 4 * comp[k] * (size_t)n, hipMemcpyHostToDevice, st));
            in[k] = (const float *)d;
        }
    }
    const BuildLeaves leaves{in[0], in[1], in[2], in[3], in[4]};
    // 1. the grid: per-axis minimum and the largest extent of the means
    const int nbb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    float *part = nullptr;
    if ((s = talloc((void **)&part, sizeof(float) * 6 * nbb))) return s;
    launch_build_bounds(in[0], n, part, nbb, st);
    std::vector<float> hp(6 * (size_t)nbb);
    HIPC(hipMemcpyAsync(hp.data(), part, sizeof(float) * hp.size(), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        float a = hp[k], b = hp[3 + k];
        for (int j = 1; j < nbb; ++j) {
            a = std::min(a, hp[6 * j + k]);
            b = std::max(b, hp[6 * j + 3 + k]);
        }
        lo[k] = a;
        hi[k] = b;
    }
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    if (ext == 0.0) ext = 1.0;
    if (!std::isfinite(ext)) return fail(ctx, HGS_ERR_INVALID_ARG, "leaf means must be finite");
    const double scale = (double)((1u << 21) - 1u) / ext;
    // 2. Morton codes, sorted by (code, leaf index): two stable passes over
    // the low and the high 32 bits
    uint32_t *lo0, *hi0, *keyA, *valA, *keyB, *tk, *tv, *ndev;
    for (uint32_t **p : {&lo0, &hi0, &keyA, &valA, &keyB, &tk, &tv})
        if ((s = talloc((void **)p, 4 * (size_t)n))) return s;
    if ((s = talloc((void **)&ndev, 16))) return s;
    const uint32_t nn = (uint32_t)n;
    HIPC(hipMemcpyAsync(ndev, &nn, 4, hipMemcpyHostToDevice, st));
    launch_build_morton(in[0], n, lo, scale, lo0, hi0, valA, st);
    HIPC(hipMemcpyAsync(keyA, lo0, 4 * (size_t)n, hipMemcpyDeviceToDevice, st));
    const SortScratch sc1{tk, tv, ctx->hist, ctx->hist_scan, ctx->partial, ctx->scan_total, ctx->sort_plan};
    const bool sw1 = launch_radix_sort(keyA, valA, nn, ndev, 32, sc1, st);
    uint32_t *idx1 = sw1 ? tv : valA;
    uint32_t *spare = sw1 ? valA : tv;  // the values buffer the first pass left free
    launch_gather_u32(hi0, idx1, n, keyB, st);
    const SortScratch sc2{tk, spare, ctx->hist, ctx->hist_scan, ctx->partial, ctx->scan_total, ctx->sort_plan};
    const bool sw2 = launch_radix_sort(keyB, idx1, nn, ndev, 31, sc2, st);
    uint32_t *idx2 = sw2 ? spare : idx1;  // leaves in (code, index) order
    uint32_t *slo = keyA, *shi = tk;       // their codes (both buffers are free again)
    launch_gather_u32(lo0, idx2, n, slo, st);
    launch_gather_u32(hi0, idx2, n, shi, st);
    uint8_t *sl = nullptr;
    if ((s = talloc((void **)&sl, (size_t)n))) return s;
    launch_split_level(slo, shi, n, sl, st);
    // 3. the tree, one level at a time
    int64_t cap = 2 * n + 64;
    BuildTree t{};
    int32_t *leaf_src = nullptr;
    auto grow = [&](int64_t need) -> hgs_status {
        if (need <= cap && t.start) return HGS_OK;
        int64_t nc = std::max<int64_t>(need, t.start ? cap + cap / 2 : cap);
        int32_t **arrs[] = {&t.start, &t.size, &t.parent, &t.child_begin, &t.child_count, &leaf_src};
        for (int32_t **a : arrs) {
            int32_t *q = nullptr;
            hgs_status e = talloc((void **)&q, 4 * (size_t)nc);
            if (e) return e;
            if (*a) HIPC(hipMemcpyAsync(q, *a, 4 * (size_t)cap, hipMemcpyDeviceToDevice, st));
            *a = q;
        }
        cap = nc;
        return HGS_OK;
    };
    if ((s = grow(cap))) return s;
    {
        // the root holds every leaf; with one leaf it is that leaf (index 0)
        static const int32_t root1[6] = {0, 1, -1, 0, 0, 0};
        const int32_t root[6] = {0, (int32_t)n, -1, 0, 0, n == 1 ? 0 : -1};
        int32_t *dst[6] = {t.start, t.size, t.parent, t.child_begin, t.child_count, leaf_src};
        for (int k = 0; k < 6; ++k)
            HIPC(hipMemcpyAsync(dst[k], n == 1 ? &root1[k] : &root[k], 4, hipMemcpyHostToDevice, st));
        HIPC(hipStreamSynchronize(st));  // the host values above are locals
    }
    int32_t *node_of = nullptr, *node_next = nullptr;
    uint32_t *flag = nullptr, *rank = nullptr, *cnt = nullptr;
    if ((s = talloc((void **)&node_of, 4 * (size_t)n))) return s;
    if ((s = talloc((void **)&node_next, 4 * (size_t)n))) return s;
    if ((s = talloc((void **)&flag, 4 * (size_t)n))) return s;
    if ((s = talloc((void **)&rank, 4 * (size_t)n))) return s;
    if ((s = talloc((void **)&cnt, 16))) return s;
    launch_fill_i32(node_of, 0, n, st);
    std::vector<int64_t> base{0, 1};
    int64_t total = 1;
    for (int level = 1;; ++level) {
        if (level > 4096) return fail(ctx, HGS_ERR_INVALID_ARG, "hierarchy deeper than 4096 levels");
        launch_level_starts(node_of, sl, t, n, level, flag, st);
        launch_scan(flag, nullptr, nn, nullptr, rank, cnt, ctx->partial, st);
        uint32_t c = 0;
        HIPC(hipMemcpyAsync(&c, cnt, 4, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        if (c == 0) break;
        if (total + c >= (int64_t)kRootParent) return fail(ctx, HGS_ERR_INVALID_ARG, "too many nodes");
        if ((s = grow(total + c))) return s;
        launch_level_nodes(node_of, flag, rank, t, n, (int32_t)total, node_next, st);
        launch_level_sizes(t, (int32_t)total, (int32_t)c, n, idx2, leaf_src, st);
        std::swap(node_of, node_next);
        total += c;
        base.push_back(total);
    }
    const int64_t N = total;
    const int nlev = (int)base.size() - 1;
    // interior ranks and the interior list
    uint32_t *irank = nullptr;
    if ((s = talloc((void **)&irank, 4 * (size_t)N))) return s;
    {
        uint32_t *ifl = nullptr;
        if ((s = talloc((void **)&ifl, 4 * (size_t)N))) return s;
        launch_interior_ranks(t.child_count, N, ifl, st);
        launch_scan(ifl, nullptr, (uint32_t)N, nullptr, irank, cnt, ctx->partial, st);
    }
    uint32_t n_int = 0;
    HIPC(hipMemcpyAsync(&n_int, cnt, 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    // 4. merges bottom up (FP64 working values)
    BuildWork w{};
    {
        double **arrs[] = {&w.mean, &w.cov, &w.op, &w.surf, &w.axes, &w.sc, &w.R, &w.q};
        const size_t per[] = {3, 6, 1, 1, 9, 3, 9, 4};
        for (int k = 0; k < 8; ++k)
            if ((s = talloc((void **)arrs[k], 8 * per[k] * (size_t)N))) return s;
        if ((s = talloc((void **)&w.sh, 8 * 48 * (size_t)std::max<uint32_t>(n_int, 1)))) return s;
        w.irank = (int32_t *)irank;
    }
    for (int d = nlev - 1; d >= 0; --d)
        launch_merge_level(t, leaf_src, leaves, w, (int32_t)base[d], (int32_t)(base[d + 1] - base[d]), st);
    // 5. the hierarchy's own buffers, then matching top down and boxes bottom up
    drop_hierarchy(ctx);
    float *bmin = nullptr, *bmax = nullptr;
    if ((s = talloc((void **)&bmin, 12 * (size_t)N))) return s;
    if ((s = talloc((void **)&bmax, 12 * (size_t)N))) return s;
    for (int k = 0; k < 5; ++k)
        if ((s = dalloc(ctx, (void **)&ctx->own[k], 4 * comp[k] * (size_t)N))) return s;
    const BuildOut o{ctx->own[0], ctx->own[1], ctx->own[2], ctx->own[3], ctx->own[4], bmin, bmax};
    build_axis_maps_upload(st);
    for (int d = 0; d < nlev; ++d)
        launch_match_level(t, w, (int32_t)base[d], (int32_t)(base[d + 1] - base[d]), o, leaf_src, in[4], st);
    for (int d = nlev - 1; d >= 0; --d)
        launch_box_level(t, (int32_t)base[d], (int32_t)(base[d + 1] - base[d]), bmin, bmax, st);
    if ((s = dalloc(ctx, (void **)&ctx->pinfo, 4 * (size_t)N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->box, 24 * (size_t)N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->child_count, 4 * (size_t)N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->child_begin, 4 * (size_t)N))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->interior, 4 * (size_t)std::max<uint32_t>(n_int, 1)))) return s;
    if ((s = dalloc(ctx, (void **)&ctx->leaf_src, 4 * (size_t)N))) return s;
    launch_build_finish(t, N, bmin, bmax, ctx->pinfo, ctx->box, st);
    HIPC(hipMemcpyAsync(ctx->child_count, t.child_count, 4 * (size_t)N, hipMemcpyDeviceToDevice, st));
    HIPC(hipMemcpyAsync(ctx->child_begin, t.child_begin, 4 * (size_t)N, hipMemcpyDeviceToDevice, st));
    HIPC(hipMemcpyAsync(ctx->leaf_src, leaf_src, 4 * (size_t)N, hipMemcpyDeviceToDevice, st));
    launch_interior_list(t.child_count, irank, N, ctx->interior, st);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    ctx->n = N;
    ctx->n_leaves = n;
    ctx->n_interior = n_int;
    ctx->has_hier = true;
    ctx->param_gen++;
    ctx->layout_gen++;
    ctx->nblocks_cap = 0;
    ctx->nv_cap = 0;
    *n_nodes = N;
    return HGS_OK;
}

hgs_status hgs_download(hgs_ctx *ctx, const hgs_hierarchy_out *o, int dst_on_device)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy");
    if (!o) return fail(ctx, HGS_ERR_INVALID_ARG, "out is NULL");
    if (o->leaf_src && !ctx->leaf_src)
        return fail(ctx, HGS_ERR_STATE, "leaf_src exists only for a hierarchy made by hgs_build");
    HIPC(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t N = ctx->n;
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    // parent and node-major boxes: unpacked on the device first
    int32_t *par = nullptr;
    float *bmn = nullptr, *bmx = nullptr;
    std::vector<void *> tmp;
    struct Cleanup {
        std::vector<void *> &v;
        ~Cleanup()
        {
            for (void *p : v) (void)hipFree(p);
        }
    } cleanup{tmp};
    if (o->parent || o->bmin || o->bmax) {
        if (dst_on_device) {
            par = o->parent;
            bmn = o->bmin;
            bmx = o->bmax;
        } else {
            for (void **p : {(void **)&par, (void **)&bmn, (void **)&bmx}) {
                if (hipMalloc(p, 12 * (size_t)N) != hipSuccess) {
                    (void)hipGetLastError();
                    return fail(ctx, HGS_ERR_OOM, "hipMalloc in hgs_download");
                }
                tmp.push_back(*p);
            }
        }
        launch_unpack_nodes(ctx->pinfo, ctx->box, N, o->parent ? par : nullptr, o->bmin ? bmn : nullptr,
                            o->bmax ? bmx : nullptr, st);
        if (!dst_on_device) {
            if (o->parent) HIPC(hipMemcpyAsync(o->parent, par, 4 * (size_t)N, kind, st));
            if (o->bmin) HIPC(hipMemcpyAsync(o->bmin, bmn, 12 * (size_t)N, kind, st));
            if (o->bmax) HIPC(hipMemcpyAsync(o->bmax, bmx, 12 * (size_t)N, kind, st));
        }
    }
    if (o->child_begin) HIPC(hipMemcpyAsync(o->child_begin, ctx->child_begin, 4 * (size_t)N, kind, st));
    if (o->child_count) HIPC(hipMemcpyAsync(o->child_count, ctx->child_count, 4 * (size_t)N, kind, st));
    if (o->leaf_src) HIPC(hipMemcpyAsync(o->leaf_src, ctx->leaf_src, 4 * (size_t)N, kind, st));
    float *const *P = ctx->use_bound ? ctx->bound : ctx->own;
    float *dst[5] = {o->mean, o->scale, o->rot, o->opacity, o->sh};
    const size_t comp[5] = {3, 3, 4, 1, 48};
    for (int k = 0; k < 5; ++k)
        if (dst[k]) HIPC(hipMemcpyAsync(dst[k], P[k], 4 * comp[k] * (size_t)N, kind, st));
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    return HGS_OK;
}

hgs_status hgs_bind_params(hgs_ctx *ctx, float *mean, float *scale, float *rot, float *opacity, float *sh)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (ctx->streaming) return fail(ctx, HGS_ERR_STATE, "parameters cannot be bound while rendering out of core");
    float *p[5] = {mean, scale, rot, opacity, sh};
    bool same = true;
    for (int k = 0; k < 5; ++k) same = same && ctx->bound[k] == p[k];
    if (same && ctx->use_bound == (p[0] != nullptr)) return HGS_OK;  // nothing changes
    int nn = 0;
    for (float *q : p) nn += q == nullptr;
    if (nn != 0 && nn != 5) return fail(ctx, HGS_ERR_INVALID_ARG, "bind all five parameter arrays or none");
    for (int k = 0; k < 5; ++k) ctx->bound[k] = p[k];
    ctx->use_bound = nn == 0;
    ctx->param_gen++;
    ctx->layout_gen++;
    ctx->have_render = false;
    return HGS_OK;
}

hgs_status hgs_cut(hgs_ctx *ctx, const hgs_view *view, int32_t *out_ids, float *out_t, int64_t capacity,
                   int64_t *out_count)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (!view || !out_count || capacity < 0 || (capacity > 0 && !out_ids))
        return fail(ctx, HGS_ERR_INVALID_ARG, "bad arguments");
    HIPC(hipSetDevice(ctx->device));
    ctx->have_render = false;  // shares the cut workspace and counters
    uint32_t n_tiles;
    size_t n_pix;
    hgs_status s;
    if ((s = setup_views(ctx, view, 1, nullptr, n_tiles, n_pix))) return s;
    if ((s = ensure_fixed(ctx, 1, 0, 0))) return s;
    hipStream_t st = ctx->stream;
    if ((s = push_views(ctx, 1, st))) return s;
    const DevHier h = dev_hier(ctx);
    const int nb = cut_blocks(ctx->n);
    launch_fill_u32((uint32_t *)ctx->ctr, 0u, sizeof(Counters) / 4, st);
    launch_cut_flags(h, ctx->views_dev, 1, ctx->masks, ctx->blk_counts, nb, st);
    launch_scan(ctx->blk_counts, nullptr, (uint32_t)nb, nullptr, ctx->blk_offsets, &ctx->ctr->cut_total, ctx->partial,
                st);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(ctx->ctr_host, ctx->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    *out_count = ctx->ctr_host->cut_total;
    if (*out_count > capacity)
        return fail(ctx, HGS_ERR_CAPACITY, "cut has " + std::to_string(*out_count) + " nodes, capacity " +
                                               std::to_string(capacity));
    if (*out_count > 0)
        launch_cut_emit(h, ctx->views_dev, 1, ctx->masks, ctx->blk_offsets, nb, ctx->word_off, out_ids, out_t, nullptr,
                        (uint32_t)capacity, st);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    return HGS_OK;
}

hgs_status hgs_cut_noalloc(hgs_ctx *ctx, const hgs_view *view, int32_t *out_ids, float *out_t, int64_t capacity,
                           int64_t *out_count)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (!view || !out_count || capacity < 0 || (capacity > 0 && !out_ids))
        return fail(ctx, HGS_ERR_INVALID_ARG, "bad arguments");
    if (ctx->n > kNoAllocMaxNodes)
        return fail(ctx, HGS_ERR_INVALID_ARG, "hierarchy of " + std::to_string(ctx->n) +
                                                  " nodes exceeds the static scratch (at most " +
                                                  std::to_string(kNoAllocMaxNodes) + " nodes)");
    if (!finite_view(*view)) return fail(ctx, HGS_ERR_INVALID_ARG, "view is invalid");
    HIPC(hipSetDevice(ctx->device));
    unsigned char *base = scratch_of(ctx->device);
    if (!base) return fail(ctx, HGS_ERR_STATE, "static scratch not set up on this device");
    uint64_t *masks = (uint64_t *)(base + kNaMasks);
    uint32_t *word_off = (uint32_t *)(base + kNaWordOff);
    uint32_t *counts = (uint32_t *)(base + kNaCounts);
    uint32_t *offsets = (uint32_t *)(base + kNaOffsets);
    uint32_t *partial = (uint32_t *)(base + kNaPartial);
    Counters *ctr = (Counters *)(base + kNaCtr);
    DevView *dview = (DevView *)(base + kNaView);
    hipStream_t st = ctx->stream;
    DevView hv;
    fill_dev_view(*view, ctx->tile_w, ctx->tile_h, hv);
    hgs_status s;
    if ((s = stage_records(ctx, &hv, 1, dview, st))) return s;
    const DevHier h = dev_hier(ctx);
    const int nb = cut_blocks(ctx->n);
    launch_fill_u32((uint32_t *)ctr, 0u, sizeof(Counters) / 4, st);
    launch_cut_flags(h, dview, 1, masks, counts, nb, st);
    launch_scan(counts, nullptr, (uint32_t)nb, nullptr, offsets, &ctr->cut_total, partial, st);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(ctx->ctr_host, ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    *out_count = ctx->ctr_host->cut_total;
    if (*out_count > capacity)
        return fail(ctx, HGS_ERR_CAPACITY, "cut has " + std::to_string(*out_count) + " nodes, capacity " +
                                               std::to_string(capacity));
    if (*out_count > 0)
        launch_cut_emit(h, dview, 1, masks, offsets, nb, word_off, out_ids, out_t, nullptr, (uint32_t)capacity, st);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    return HGS_OK;
}

hgs_status hgs_compact_mark(hgs_ctx *ctx, const hgs_view *views, int32_t n_views, float tau_min, float tau_max,
                            uint8_t *keep)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (!views || n_views <= 0 || !keep) return fail(ctx, HGS_ERR_INVALID_ARG, "bad views / n_views / keep");
    if (!std::isfinite(tau_min) || !std::isfinite(tau_max) || !(tau_min > 0.0f))
        return fail(ctx, HGS_ERR_INVALID_ARG, "tau_min must be positive and finite, tau_max finite");
    int levels = 0;
    for (double t = tau_min; t <= (double)tau_max; t *= 2.0)
        if (++levels > 64) return fail(ctx, HGS_ERR_INVALID_ARG, "more than 64 granularity levels");
    HIPC(hipSetDevice(ctx->device));
    ctx->have_render = false;  // the view records are replaced
    hgs_status s;
    if (ctx->cmp_emax_n != ctx->n) {
        if ((s = realloc_buf(ctx, ctx->cmp_emax, (size_t)ctx->n))) return s;
        ctx->cmp_emax_n = ctx->n;
    }
    hipStream_t st = ctx->stream;
    const DevHier h = dev_hier(ctx);
    for (int v0 = 0; v0 < n_views; v0 += kMaxViews) {
        const int nb = std::min(kMaxViews, n_views - v0);
        uint32_t n_tiles;
        size_t n_pix;
        if ((s = setup_views(ctx, views + v0, nb, nullptr, n_tiles, n_pix))) return s;
        if ((s = push_views(ctx, nb, st))) return s;
        launch_compact_emax(h, ctx->views_dev, nb, v0 == 0, ctx->cmp_emax, st);
        HIPC(hipGetLastError());
    }
    launch_compact_keep(h, ctx->cmp_emax, (double)tau_min, levels, keep, st);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    return HGS_OK;
}

hgs_status hgs_render(hgs_ctx *ctx, const hgs_view *views, int32_t n_views, float *const *out_rgb, hgs_stats *stats)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy uploaded");
    if (!views || n_views <= 0 || n_views > kMaxViews || !out_rgb)
        return fail(ctx, HGS_ERR_INVALID_ARG, "bad views / n_views / out_rgb");
    for (int v = 0; v < n_views; ++v)
        if (!out_rgb[v]) return fail(ctx, HGS_ERR_INVALID_ARG, "out_rgb[" + std::to_string(v) + "] is NULL");
    HIPC(hipSetDevice(ctx->device));
    ctx->have_render = false;
    uint32_t n_tiles;
    size_t n_pix;
    hgs_status s;
    if ((s = setup_views(ctx, views, n_views, out_rgb, n_tiles, n_pix))) return s;
    if ((s = ensure_fixed(ctx, n_views, n_tiles, n_pix))) return s;
    if (ctx->persist) blend_prepare(ctx->tile_w, ctx->tile_h, ctx->batch);
    const bool timed = stats && stats->ms[0] < 0.0f && n_views == 1;
    if (ctx->cut_cap == 0) {
        const uint64_t guess = std::min<uint64_t>((uint64_t)n_views * (uint64_t)std::min<int64_t>(ctx->n_leaves, 1 << 21),
                                                  0x7FFFFFFFull);
        if ((s = ensure_cut_cap(ctx, (uint32_t)std::max<uint64_t>(guess, 4096)))) return s;
    }
    if (ctx->pair_cap == 0) {
        const uint64_t guess = std::min<uint64_t>((uint64_t)n_pix * 4 + 65536, 0x7FFFFFFFull);
        if ((s = ensure_pair_cap(ctx, (uint32_t)guess))) return s;
    }
    hipEvent_t ev[8] = {};
    if (timed)
        for (auto &e : ev) HIPC(hipEventCreate(&e));
    for (int attempt = 0; attempt < 4; ++attempt) {
        const bool graph = n_views > 1;
        hipStream_t st = graph ? ctx->gstream : ctx->stream;
        if (graph) {
            HIPC(hipEventRecord(ctx->ev_in, ctx->stream));
            HIPC(hipStreamWaitEvent(ctx->gstream, ctx->ev_in, 0));
        }
        if ((s = push_views(ctx, n_views, st))) return s;
        if (graph) {
            RenderKey key;
            key.nv = n_views;
            for (int v = 0; v < n_views; ++v) {
                key.wh.push_back(views[v].width);
                key.wh.push_back(views[v].height);
            }
            key.tw = ctx->tile_w;
            key.th = ctx->tile_h;
            key.batch = ctx->batch;
            key.persist = ctx->persist;
            key.layout = ctx->layout_gen * 1000003ull + ctx->param_gen;
            key.profiled = ctx->profile;
            if (!ctx->gexec || !(key == ctx->gkey)) {
                if (ctx->gexec) {
                    HIPC(hipGraphExecDestroy(ctx->gexec));
                    ctx->gexec = nullptr;
                }
                hipGraph_t g = nullptr;
                HIPC(hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
                enqueue_forward(ctx, n_views, n_tiles, ctx->gstream, nullptr, !ctx->profile);
                HIPC(hipStreamEndCapture(ctx->gstream, &g));
                hipError_t e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return fail(ctx, HGS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
                ctx->gkey = key;
                ctx->g_pairs_in_scratch = ctx->pairs_in_scratch;
            }
            ctx->pairs_in_scratch = ctx->g_pairs_in_scratch;
            HIPC(hipGraphLaunch(ctx->gexec, ctx->gstream));
            if (ctx->profile) {
                // timed blend outside the graph
                KernelTimer kt(ctx, 0, ctx->gstream);
                enqueue_blend(ctx, n_views, n_tiles, ctx->gstream);
            }
        } else {
            enqueue_forward(ctx, n_views, n_tiles, st, timed ? ev : nullptr, true);
        }
        HIPC(hipGetLastError());
        HIPC(hipMemcpyAsync(ctx->ctr_host, ctx->ctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
        if (ctx->streaming)
            HIPC(hipMemcpyAsync(ctx->stream_host + 3, ctx->sd.overflow, 4, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        const Counters c = *ctx->ctr_host;
        bool grow = false;
        if (c.cut_total > ctx->cut_cap) {
            if ((s = ensure_cut_cap(ctx, (uint32_t)std::min<uint64_t>((uint64_t)c.cut_total * 5 / 4 + 1024, 0x7FFFFFFFull))))
                return s;
            grow = true;
        }
        if (!grow && c.pair_total > ctx->pair_cap) {
            if ((s = ensure_pair_cap(ctx, (uint32_t)std::min<uint64_t>((uint64_t)c.pair_total * 5 / 4 + 4096, 0x7FFFFFFFull))))
                return s;
            grow = true;
        }
        if (grow) continue;
        if (ctx->streaming && ctx->stream_host[3]) {
            if (timed)
                for (auto &e : ev) (void)hipEventDestroy(e);
            return fail(ctx, HGS_ERR_CAPACITY, "the parameter cache cannot hold the nodes this render needs "
                                               "(the image lacks them): hgs_stream_cleanup or a larger cache");
        }
        ctx->have_render = true;
        ++ctx->render_seq;
        ctx->render_param_gen = ctx->param_gen;
        ctx->last_nv = n_views;
        ctx->last_tiles = n_tiles;
        ctx->last_cut = c.cut_total;
        ctx->last_visible = c.vis_total;
        ctx->last_pix = n_pix;
        ctx->r_tw = ctx->tile_w;
        ctx->r_th = ctx->tile_h;
        ctx->r_batch = ctx->batch;
        ctx->r_persist = ctx->persist;
        ctx->last_graphed = n_views > 1 && !ctx->profile;
        if (stats) {
            stats->cut = c.cut_total;
            stats->visible = c.vis_total;
            stats->pairs = c.pair_total;
            stats->evaluated = (int64_t)c.evaluated;
            stats->blended = (int64_t)c.blended;
            stats->render_id = ctx->render_seq;
            for (int k = 0; k < 8; ++k) stats->ms[k] = 0.0f;
            if (timed) {
                for (int k = 0; k < 7; ++k) (void)hipEventElapsedTime(&stats->ms[k], ev[k], ev[k + 1]);
                (void)hipEventElapsedTime(&stats->ms[7], ev[0], ev[7]);
            }
        }
        if (timed)
            for (auto &e : ev) (void)hipEventDestroy(e);
        return HGS_OK;
    }
    if (timed)
        for (auto &e : ev) (void)hipEventDestroy(e);
    return fail(ctx, HGS_ERR_CAPACITY, "render did not fit after growing buffers");
}

hgs_status hgs_last_render(hgs_ctx *ctx, uint64_t *render_id, int32_t *n_views)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    const bool live = ctx->have_render && ctx->render_param_gen == ctx->param_gen;
    if (render_id) *render_id = live ? ctx->render_seq : 0;
    if (n_views) *n_views = live ? ctx->last_nv : 0;
    return HGS_OK;
}

// Checks the arguments of a backward of render `render_id` and puts the
// cotangent pointers into the host view records.
static hgs_status check_backward(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *dL_drgb)
{
    if (ctx->streaming) return fail(ctx, HGS_ERR_STATE, "no backward while rendering out of core");
    if (!ctx->have_render || ctx->render_param_gen != ctx->param_gen)
        return fail(ctx, HGS_ERR_STATE, "render_backward needs a render with the current parameters");
    if (render_id != ctx->render_seq)
        return fail(ctx, HGS_ERR_STATE, "render " + std::to_string(render_id) +
                                            " has been replaced: the ctx holds the state of render " +
                                            std::to_string(ctx->render_seq));
    if (n_views != ctx->last_nv)
        return fail(ctx, HGS_ERR_INVALID_ARG, "render " + std::to_string(render_id) + " has " +
                                                  std::to_string(ctx->last_nv) + " views, not " +
                                                  std::to_string(n_views));
    if (!dL_drgb) return fail(ctx, HGS_ERR_INVALID_ARG, "bad gradient arguments");
    for (int v = 0; v < ctx->last_nv; ++v) {
        if (!dL_drgb[v]) return fail(ctx, HGS_ERR_INVALID_ARG, "dL_drgb[" + std::to_string(v) + "] is NULL");
        ctx->views_host[v].dL = dL_drgb[v];
    }
    return HGS_OK;
}

// Queues the backward of the last render into `out`, or, with `fused`,
// with the optimiser step applied in the gather (scalars: 5 host records).
// A render of several views replays a captured graph, keyed by the render's
// graph and every output array.
static hgs_status run_backward(hgs_ctx *ctx, const hgs_grads *out, const AdamRows *fused, const AdamScalars *scalars)
{
    const int nv = ctx->last_nv;
    HIPC(hipSetDevice(ctx->device));
    if (ctx->deterministic && ctx->part_cap < ctx->pair_cap) {
        if (hgs_status s = realloc_buf(ctx, ctx->part, (size_t)ctx->pair_cap * 11)) return s;
        ctx->part_cap = ctx->pair_cap;
        ctx->bgraph_valid = false;
    }
    const void *outs[21] = {};
    if (fused) {
        for (int k = 0; k < 5; ++k) {
            outs[6 + k] = fused->p[k];
            outs[11 + k] = fused->m[k];
            outs[16 + k] = fused->v[k];
        }
    } else {
        const void *g[6] = {out->mean, out->scale, out->rot, out->opacity, out->sh, out->dt};
        memcpy(outs, g, sizeof g);
    }
    hipStream_t st = ctx->last_graphed ? ctx->gstream : ctx->stream;
    if (ctx->last_graphed) {
        // replay (or capture once) the backward on the library stream, in
        // order with the caller's stream on both sides
        if (!ctx->bexec || !ctx->bgraph_valid || !(ctx->bkey == ctx->gkey) ||
            memcmp(ctx->bkey_out, outs, sizeof outs) != 0) {
            if (ctx->bexec) {
                HIPC(hipGraphExecDestroy(ctx->bexec));
                ctx->bexec = nullptr;
            }
            hipGraph_t g = nullptr;
            HIPC(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            enqueue_backward(ctx, nv, out, fused, st);
            HIPC(hipStreamEndCapture(st, &g));
            hipError_t e = hipGraphInstantiate(&ctx->bexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
                return fail(ctx, HGS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            ctx->bkey = ctx->gkey;
            memcpy(ctx->bkey_out, outs, sizeof outs);
            ctx->bgraph_valid = true;
        }
        HIPC(hipEventRecord(ctx->ev_in, ctx->stream));
        HIPC(hipStreamWaitEvent(st, ctx->ev_in, 0));
    }
    if (hgs_status s = push_views(ctx, nv, st)) return s;
    if (fused)
        if (hgs_status s = stage_records(ctx, scalars, 5, ctx->adam_sc, st)) return s;
    if (ctx->last_graphed) {
        HIPC(hipGraphLaunch(ctx->bexec, st));
        HIPC(hipEventRecord(ctx->ev_out, st));
        HIPC(hipStreamWaitEvent(ctx->stream, ctx->ev_out, 0));
    } else {
        enqueue_backward(ctx, nv, out, fused, st);
    }
    HIPC(hipGetLastError());
    // host copy of views keeps dL for nothing else
    for (int v = 0; v < nv; ++v) ctx->views_host[v].dL = nullptr;
    return HGS_OK;
}

hgs_status hgs_render_backward(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *dL_drgb,
                               hgs_grads *out)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (hgs_status s = check_backward(ctx, render_id, n_views, dL_drgb)) return s;
    if (!out || !out->mean || !out->scale || !out->rot || !out->opacity || !out->sh)
        return fail(ctx, HGS_ERR_INVALID_ARG, "bad gradient arguments");
    return run_backward(ctx, out, nullptr, nullptr);
}

hgs_status hgs_backward_adam_step(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *dL_drgb,
                                  const hgs_adam *a)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (hgs_status s = check_backward(ctx, render_id, n_views, dL_drgb)) return s;
    AdamScalars sc[5];
    if (hgs_status s = check_adam(ctx, a, false, sc)) return s;
    AdamRows rows{};
    for (int k = 0; k < 5; ++k) {
        rows.p[k] = a->param[k];
        rows.m[k] = a->m[k];
        rows.v[k] = a->v[k];
    }
    rows.sc = ctx->adam_sc;
    if (hgs_status s = run_backward(ctx, nullptr, &rows, sc)) return s;
    adam_stepped(ctx, a);
    return HGS_OK;
}

hgs_status hgs_l1_loss(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *target,
                       float *const *dL_drgb, double *loss)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->have_render) return fail(ctx, HGS_ERR_STATE, "no render whose images the loss could read");
    if (render_id != ctx->render_seq)
        return fail(ctx, HGS_ERR_STATE, "render " + std::to_string(render_id) +
                                            " has been replaced: the ctx holds the state of render " +
                                            std::to_string(ctx->render_seq));
    if (n_views != ctx->last_nv)
        return fail(ctx, HGS_ERR_INVALID_ARG, "render " + std::to_string(render_id) + " has " +
                                                  std::to_string(ctx->last_nv) + " views, not " +
                                                  std::to_string(n_views));
    if (!target || !dL_drgb || !loss) return fail(ctx, HGS_ERR_INVALID_ARG, "bad loss arguments");
    const int nv = ctx->last_nv;
    for (int v = 0; v < nv; ++v) {
        if (!target[v] || !dL_drgb[v])
            return fail(ctx, HGS_ERR_INVALID_ARG, "target or dL_drgb of view " + std::to_string(v) + " is NULL");
        if (!ctx->views_host[v].out_rgb) return fail(ctx, HGS_ERR_STATE, "the last render kept no images");
    }
    HIPC(hipSetDevice(ctx->device));
    for (int v = 0; v < nv; ++v) {
        ctx->views_host[v].target = target[v];
        ctx->views_host[v].dL = dL_drgb[v];
    }
    hipStream_t st = ctx->stream;
    hgs_status s = push_views(ctx, nv, st);
    for (int v = 0; v < nv; ++v) {
        ctx->views_host[v].target = nullptr;
        ctx->views_host[v].dL = nullptr;
    }
    if (s) return s;
    launch_l1(ctx->views_dev, nv, (uint32_t)ctx->last_pix, ctx->l1_partial, loss, st);
    HIPC(hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_stream_begin(hgs_ctx *ctx, int64_t cache_nodes)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->has_hier) return fail(ctx, HGS_ERR_STATE, "no hierarchy");
    if (ctx->streaming) return fail(ctx, HGS_ERR_STATE, "already rendering out of core");
    if (ctx->use_bound) return fail(ctx, HGS_ERR_STATE, "unbind the parameters first");
    if (cache_nodes < 1 || cache_nodes > ctx->n || cache_nodes >= ((int64_t)1 << 31))
        return fail(ctx, HGS_ERR_INVALID_ARG, "cache_nodes must lie in [1, n_nodes]");
    HIPC(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    HIPC(hipStreamSynchronize(st));
    const int64_t N = ctx->n;
    const size_t comp[5] = {3, 3, 4, 1, 48};
    size_t total = 0;
    for (int k = 0; k < 5; ++k) total += 4 * comp[k] * (size_t)N;
    void *block = nullptr;
    if (hipHostMalloc(&block, total, hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, HGS_ERR_OOM, "hipHostMalloc(" + std::to_string(total) + ") for the host parameters");
    }
    void *block_dev = nullptr;
    if (hipHostGetDevicePointer(&block_dev, block, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(block);
        return fail(ctx, HGS_ERR_HIP, "hipHostGetDevicePointer of the host parameters");
    }
    float *hp[5], *dp[5];
    size_t off = 0;
    for (int k = 0; k < 5; ++k) {
        hp[k] = (float *)((char *)block + off);
        dp[k] = (float *)((char *)block_dev + off);
        off += 4 * comp[k] * (size_t)N;
        if (hipMemcpy(hp[k], ctx->own[k], 4 * comp[k] * (size_t)N, hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(block);
            return fail(ctx, HGS_ERR_HIP, "copying the parameters to host memory");
        }
    }
    // device side first; on failure everything allocated here goes again
    const size_t C = (size_t)cache_nodes;
    StreamParams cache{};
    StreamDev d{};
    std::vector<void *> mine;
    auto take = [&](void **p, size_t bytes) -> bool {
        if (dalloc(ctx, p, bytes) != HGS_OK) return false;
        mine.push_back(*p);
        return true;
    };
    bool ok = take((void **)&cache.mean, 12 * C) && take((void **)&cache.scale, 12 * C) &&
              take((void **)&cache.rot, 16 * C) && take((void **)&cache.opacity, 4 * C) &&
              take((void **)&cache.sh, 192 * C) && take((void **)&d.slot, 4 * (size_t)N) &&
              take((void **)&d.node_in_slot, 4 * C) && take((void **)&d.last_used, 4 * C) &&
              take((void **)&d.free_stack, 4 * C) && take((void **)&d.req, 4 * C) &&
              take((void **)&d.free_top, 64);
    if (!ok) {
        const std::string msg = ctx->err;
        for (void *p : mine) dfree(ctx, p);
        (void)hipHostFree(block);
        return fail(ctx, HGS_ERR_OOM, msg);
    }
    d.frame = d.free_top + 1;
    d.req_count = d.free_top + 2;
    d.overflow = d.free_top + 3;
    d.transferred = (unsigned long long *)(d.free_top + 4);
    d.cap = (uint32_t)C;
    d.req_cap = (uint32_t)C;
    ctx->host_block = block;
    ctx->host_params = StreamParams{hp[0], hp[1], hp[2], hp[3], hp[4]};
    ctx->host_params_dev = StreamParams{dp[0], dp[1], dp[2], dp[3], dp[4]};
    ctx->cache_params = cache;
    ctx->sd = d;
    ctx->streaming = true;
    for (int k = 0; k < 5; ++k) {
        dfree(ctx, ctx->own[k]);
        ctx->own[k] = nullptr;
    }
    launch_stream_init(d, N, st);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
    ctx->have_render = false;
    ctx->param_gen++;
    ctx->layout_gen++;
    return HGS_OK;
}

hgs_status hgs_stream_end(hgs_ctx *ctx)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->streaming) return fail(ctx, HGS_ERR_STATE, "not rendering out of core");
    HIPC(hipSetDevice(ctx->device));
    HIPC(hipStreamSynchronize(ctx->stream));
    const size_t comp[5] = {3, 3, 4, 1, 48};
    float *hp[5] = {ctx->host_params.mean, ctx->host_params.scale, ctx->host_params.rot, ctx->host_params.opacity,
                    ctx->host_params.sh};
    hgs_status s;
    for (int k = 0; k < 5; ++k) {
        if ((s = dalloc(ctx, (void **)&ctx->own[k], 4 * comp[k] * (size_t)ctx->n))) return s;
        HIPC(hipMemcpy(ctx->own[k], hp[k], 4 * comp[k] * (size_t)ctx->n, hipMemcpyHostToDevice));
    }
    stream_release(ctx);
    ctx->have_render = false;
    ctx->param_gen++;
    ctx->layout_gen++;
    return HGS_OK;
}

hgs_status hgs_stream_cleanup(hgs_ctx *ctx, int32_t max_age)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    if (!ctx->streaming) return fail(ctx, HGS_ERR_STATE, "not rendering out of core");
    if (max_age < 0) return fail(ctx, HGS_ERR_INVALID_ARG, "max_age must be >= 0");
    HIPC(hipSetDevice(ctx->device));
    launch_stream_cleanup(ctx->sd, (uint32_t)max_age, ctx->stream);
    HIPC(hipGetLastError());
    return HGS_OK;
}

hgs_status hgs_stream_info(hgs_ctx *ctx, hgs_stream_stats *out)
{
    if (!ctx || !out) return HGS_ERR_INVALID_ARG;
    if (!ctx->streaming) return fail(ctx, HGS_ERR_STATE, "not rendering out of core");
    HIPC(hipSetDevice(ctx->device));
    HIPC(hipMemcpyAsync(ctx->stream_host, ctx->sd.free_top, 24, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    const uint32_t *h = ctx->stream_host;
    out->cache_nodes = ctx->sd.cap;
    out->resident = (int64_t)ctx->sd.cap - h[0];
    out->frame = h[1];
    out->requested = h[2];
    out->overflow = (int32_t)h[3];
    uint64_t tr = 0;
    memcpy(&tr, h + 4, 8);
    out->transferred_total = (int64_t)tr;
    return HGS_OK;
}

hgs_status hgs_counters(hgs_ctx *ctx, int64_t *out, int32_t n)
{
    if (!ctx || !out || n <= 0) return HGS_ERR_INVALID_ARG;
    HIPC(hipSetDevice(ctx->device));
    HIPC(hipMemcpyAsync(ctx->ctr_host, ctx->ctr, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    const Counters &c = *ctx->ctr_host;
    const int64_t v[] = {c.cut_total, c.vis_total, c.pair_total, (int64_t)c.evaluated, (int64_t)c.blended,
                         (int64_t)c.evaluated_t, (int64_t)c.bwd_evaluated, (int64_t)c.bwd_evaluated_t,
                         (int64_t)c.bwd_contrib};
    for (int32_t k = 0; k < n && k < (int32_t)(sizeof v / sizeof v[0]); ++k) out[k] = v[k];
    return HGS_OK;
}

hgs_status hgs_set_profiling(hgs_ctx *ctx, int32_t on)
{
    if (!ctx) return HGS_ERR_INVALID_ARG;
    HIPC(hipSetDevice(ctx->device));
    collect_times(ctx);
    ctx->profile = on != 0;
    for (int k = 0; k < kTimedKernels; ++k) {
        ctx->k_ms[k] = 0.0;
        ctx->k_launches[k] = 0;
    }
    return HGS_OK;
}

hgs_status hgs_kernel_time(hgs_ctx *ctx, int32_t which, double *total_ms, int64_t *launches)
{
    if (!ctx || !total_ms || !launches || which < 0 || which >= kTimedKernels) return HGS_ERR_INVALID_ARG;
    HIPC(hipSetDevice(ctx->device));
    collect_times(ctx);
    *total_ms = ctx->k_ms[which];
    *launches = ctx->k_launches[which];
    return HGS_OK;
}

hgs_status hgs_get_buffer(hgs_ctx *ctx, int32_t which, const void **dev_ptr, int64_t *count)
{
    if (!ctx || !dev_ptr || !count) return HGS_ERR_INVALID_ARG;
    if (!ctx->have_render) return fail(ctx, HGS_ERR_STATE, "no render yet");
    switch (which) {
    case 0: *dev_ptr = ctx->cut_ids; *count = ctx->last_cut; break;
    case 1: *dev_ptr = ctx->cut_t; *count = ctx->last_cut; break;
    case 2: *dev_ptr = ctx->T_final; *count = (int64_t)ctx->last_pix; break;
    case 3: *dev_ptr = ctx->n_last; *count = (int64_t)ctx->last_pix; break;
    case 4: *dev_ptr = ctx->n_blend; *count = (int64_t)ctx->last_pix; break;
    case 5: *dev_ptr = ctx->sgrad; *count = (int64_t)ctx->last_visible * 12; break;
    case 8: *dev_ptr = ctx->vis_rank; *count = (int64_t)ctx->last_cut; break;
    case 6: *dev_ptr = ctx->cut_base; *count = ctx->last_nv + 1; break;
    case 7: *dev_ptr = ctx->ranges; *count = (int64_t)ctx->last_tiles * 2; break;
    default: return fail(ctx, HGS_ERR_INVALID_ARG, "unknown buffer");
    }
    return HGS_OK;
}

}  // extern "C"
