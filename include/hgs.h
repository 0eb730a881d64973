/*
 * hgs.h - C ABI of the MI355X (gfx950) hierarchical 3D-Gaussian cut and
 * splatting library.
 *
 * The library implements the per-view hot path of "A Hierarchical 3D
 * Gaussian Representation for Real-Time Rendering of Very Large Datasets"
 * (Kerbl et al., ACM TOG 43(4), 2024):
 *   - the level-of-detail cut of Sec. 4.2 ("Hierarchy Cut Selection and
 *     Level Switching"): granularity = projected size of the largest
 *     dimension of a node's leaf bounding box; a node is selected when it
 *     meets the target granularity tau and its parent does not;
 *   - the interpolation weight of Eq. (t_interp), used as the parent's weight
 *     in the lerp of position, scale, rotation and SH (Sec. 4.2) and in the
 *     opacity transition of Eq. (alphap) generalised to K children
 *     (Sec. 5.2);
 *   - tile-based splatting (Sec. 3 "Background", Eq. (alpha) and the
 *     projected Gaussian G): EWA projection with the anti-aliasing low-pass
 *     of Sec. 5.1, degree-3 SH colour, (tile, depth) ordering and
 *     front-to-back compositing with alpha clamped to 0.99 (Sec. 7.3);
 *   - the backward pass to every node's parameters (Sec. 5.1, Sec. 7.1
 *     "Implementation"), with an absolute-value opacity activation and no
 *     opacity gradient through the 0.99 clamp (Sec. 7.3).
 *
 * Conventions (all calls):
 *   - every function returns hgs_status; nothing throws across the ABI;
 *     hgs_last_error(ctx) returns the message of the last failure on ctx;
 *   - "device pointer" means memory on the ctx's device (hipMalloc or a
 *     torch CUDA tensor); "host pointer" means ordinary host memory;
 *   - work is queued on the stream given to hgs_create (NULL = the default
 *     stream) unless a call is documented to synchronise;
 *   - a ctx must not be used from two threads at once.
 *
 * Hierarchy layout (one array per attribute, FP32, node-major: the
 * components of a node are contiguous, so the sparse reads of a cut touch
 * few cache lines):
 *   nodes in BFS order, root = 0, parent[i] < i, the children of a node
 *   contiguous starting at child_begin; child_count == 0 <=> leaf;
 *   bmin/bmax [N][3] axis-aligned box over the node's leaves;
 *   mean [N][3]; scale [N][3] (activated, world units);
 *   rot [N][4] quaternion (w, x, y, z);
 *   opacity [N]: opacity of a leaf, "falloff" (may exceed 1) of an interior
 *   node; the renderer uses |opacity|;
 *   sh [N][48]: entry 3*k + c = coefficient of real SH basis function k
 *   (k = l*l + l + m, degree <= 3) for colour channel c.
 */
#ifndef HGS_H
#define HGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HGS_OK = 0,
    HGS_ERR_INVALID_ARG = 1, /* bad pointer, size, view or topology */
    HGS_ERR_OOM = 2,         /* device allocation failed */
    HGS_ERR_HIP = 3,         /* a HIP runtime call failed */
    HGS_ERR_STATE = 4,       /* call order violated (e.g. backward before render) */
    HGS_ERR_CAPACITY = 5     /* caller's output buffer too small; *out_count holds the size needed */
} hgs_status;

typedef struct hgs_ctx hgs_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (may be NULL for the default stream); it is borrowed, not owned.
 * On success *out receives a library-owned context.
 * Errors: HGS_ERR_INVALID_ARG (out == NULL, bad device), HGS_ERR_HIP. */
hgs_status hgs_create(hgs_ctx **out, int device, void *hip_stream);

/* Release every device buffer of ctx.  NULL is accepted and ignored. */
void hgs_destroy(hgs_ctx *ctx);

/* Message of the last failing call on ctx (never NULL; "" if none).  The
 * string is owned by ctx and valid until its next call. */
const char *hgs_last_error(const hgs_ctx *ctx);

/* Point the ctx at another stream (borrowed). */
hgs_status hgs_set_stream(hgs_ctx *ctx, void *hip_stream);

typedef struct {
    int64_t n_nodes;
    int32_t sh_degree;                               /* must be 3 */
    const int32_t *parent, *child_begin, *child_count; /* [N] */
    const float *bmin, *bmax;                        /* [N][3] */
    const float *mean, *scale, *rot, *opacity, *sh;  /* [N][3] [N][3] [N][4] [N] [N][48] */
} hgs_hierarchy_desc;

/* Copy a hierarchy into library-owned device memory.  `src_on_device` = 0:
 * every pointer in desc is a host pointer; 1: every pointer is a device
 * pointer.  The topology is validated (parent < child, children contiguous
 * and consistent with parent, child ranges in bounds, boxes ordered);
 * a malformed hierarchy returns HGS_ERR_INVALID_ARG and leaves ctx without a
 * hierarchy.  Synchronises the ctx stream.  Replaces any earlier hierarchy
 * and unbinds parameters bound with hgs_bind_params.  Leaf boxes must contain
 * the granularity box the caller intends (the library does not recompute
 * boxes from the Gaussians). */
hgs_status hgs_upload(hgs_ctx *ctx, const hgs_hierarchy_desc *desc, int src_on_device);

/* Leaf Gaussians for hgs_build (node-major, FP32): mean [n][3], scale
 * [n][3] (activated, world units), rot [n][4] (w, x, y, z), opacity [n],
 * sh [n][48] (coefficient k of channel c at 3 k + c). */
typedef struct {
    int64_t n_leaves;
    const float *mean, *scale, *rot, *opacity, *sh;
} hgs_leaves_desc;

/* Hierarchy generation (Sec. 4.1 "Hierarchy Generation", with the
 * orientation matching of Sec. 4.2) on the device, replacing ctx's
 * hierarchy as hgs_upload would (parameters unbound, render state dropped).
 * The tree: the leaves' means on a 2^21 grid per axis over their bounding
 * cube (cell = floor((x - min) (2^21 - 1) / largest extent + 1/2)), sorted
 * by (Morton code, leaf index); breadth first from the root, a node with
 * two or more leaves at depth d < 21 has one child per non-empty octant of
 * its cell (in code order; one child when all share it), at depth 21 and
 * beyond (leaves in one finest cell) k = min(8, m) children of m j / k ..
 * leaves each.  Interior Gaussians by Eq. (merge) with the weights o_i S_i
 * (S = Thomsen's ellipsoid surface from the scales, o the child's opacity
 * or falloff), SH with the same weights, falloff = sum w' / S_p, scales
 * and axes from the eigen-decomposition of the merged covariance; then top
 * down every node's axes re-assigned by the proper signed axis permutation
 * closest to its parent's (the world axes at the root), quaternions with
 * q . q_parent >= 0 (w >= 0 at the root).  Boxes: a leaf's mean +- 3
 * sqrt(diag Sigma) from its stored values, rounded outward to FP32; an
 * interior node's the union of its children's.  All arithmetic in FP64,
 * stored in FP32.  `src_on_device`: 0 = host pointers, 1 = device pointers.
 * *n_nodes (host) receives the node count.  n_leaves in [1, 2^29];
 * non-finite means: HGS_ERR_INVALID_ARG.  Synchronises the ctx stream;
 * allocates its working memory (FP64, about 0.5 kB per node) for the call. */
hgs_status hgs_build(hgs_ctx *ctx, const hgs_leaves_desc *leaves, int src_on_device, int64_t *n_nodes);

/* Copies ctx's hierarchy out in the layouts of hgs_hierarchy_desc
 * (node-major; boxes [N][3]); every pointer may be NULL (not copied).
 * leaf_src [N]: the hgs_build input index of every leaf node, -1 for an
 * interior node (HGS_ERR_STATE for a hierarchy that came from hgs_upload).
 * The parameters are the ones the renderer reads (the bound arrays when
 * bound).  `dst_on_device`: 0 = host pointers, 1 = device pointers.
 * Synchronises the ctx stream. */
typedef struct {
    int32_t *parent, *child_begin, *child_count, *leaf_src;
    float *bmin, *bmax, *mean, *scale, *rot, *opacity, *sh;
} hgs_hierarchy_out;
hgs_status hgs_download(hgs_ctx *ctx, const hgs_hierarchy_out *out, int dst_on_device);

/* Render from caller-owned device parameter arrays instead of the copies
 * made by hgs_upload (same layouts, N = n_nodes).  Pointers stay owned by the
 * caller and must stay valid while used.  Passing all NULL reverts to the
 * library's copies.  Invalidates the state kept for hgs_render_backward. */
hgs_status hgs_bind_params(hgs_ctx *ctx, float *mean, float *scale, float *rot, float *opacity, float *sh);

/* One pinhole camera.  R (row-major 3x3) rows are the camera's right, down
 * and forward axes in world coordinates: p_cam = R (x - eye).  Pixel (i, j)
 * samples the image-plane point (i + 1/2, j + 1/2) with
 * u = fx p.x / p.z + cx, v = fy p.y / p.z + cy.  Splats with p.z <= z_near
 * are culled; z_near must be positive (a splat behind the camera is never
 * drawn).  tau is the target granularity in pixels (>= 0).  A view with a
 * non-finite field, fx or fy <= 0, z_near <= 0, tau < 0 or a size outside
 * [1, 32768] is rejected with HGS_ERR_INVALID_ARG. */
typedef struct {
    float R[9];
    float eye[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near, tau;
} hgs_view;

/* The cut of Sec. 4.2 for one view (host pointer `view`).
 * out_ids (device, int32[capacity]) receives the selected node ids in
 * ascending order; out_t (device, float[capacity], may be NULL) the
 * interpolation weight of each (the parent's weight; 0 for the root, for
 * leaves coarser than tau, and where eps(parent) <= eps(node) or the eye is
 * inside the parent's box).  The predicate and t are evaluated in FP64.
 * *out_count (host) receives the cut size; if it exceeds capacity nothing is
 * written and HGS_ERR_CAPACITY is returned.  Synchronises the ctx stream. */
hgs_status hgs_cut(hgs_ctx *ctx, const hgs_view *view, int32_t *out_ids, float *out_t, int64_t capacity,
                   int64_t *out_count);

/* hgs_cut without device allocation, for callers that cannot allocate
 * (code that must not call hipMalloc: under HIP graph capture, in tight
 * serving loops, or in harnesses that forbid it).  Same arguments, results
 * and errors as hgs_cut; the caller still provides out_ids and out_t.  The
 * cut's working memory (bit masks, block counts and offsets, scan partials,
 * counters, the view record: about 12.6 MiB) is a static device array of
 * the library, one per device, held until the process ends, so the call
 * allocates nothing and leaves the ctx's workspaces, and the state kept for
 * hgs_render_backward, as they were.  Limit: hierarchies of at most 2^26
 * (67,108,864) nodes; larger ones get HGS_ERR_INVALID_ARG.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * threads, or two streams with work in flight) race and must be serialised
 * by the caller.  Synchronises the ctx stream. */
hgs_status hgs_cut_noalloc(hgs_ctx *ctx, const hgs_view *view, int32_t *out_ids, float *out_t, int64_t capacity,
                           int64_t *out_count);

/* Hierarchy compaction (Sec. 5.2, "Compacting the Hierarchy"): marks the
 * nodes that survive the sparsification for a set of (training) views.  With
 * the granularity ladder tau_i = tau_min 2^i for every i with tau_i <=
 * tau_max (the paper: tau_min = 3 px, tau_max = half the image resolution),
 * a node is kept when it is a leaf, when it is a bottom-most node of the
 * union of the views' cuts (Sec. 4.2) at some tau_i, or when it lies above
 * the last of these cuts; every other node lies between two kept levels and
 * is removed.  Only the views' eye and fx, fy enter (their tau and image
 * size are not used, but must be valid as for hgs_render); any number of
 * views (processed in batches of 1024).  keep (device, uint8[n_nodes])
 * receives 1 (kept) or 0.  The decisions use the cut's FP64 granularity, so
 * they match it bit for bit.  tau_min <= 0, non-finite taus or more than 64
 * levels: HGS_ERR_INVALID_ARG; with no level (tau_min > tau_max) every node
 * is kept.  Invalidates the state kept for hgs_render_backward.
 * Synchronises the ctx stream.  hgs_compact_rebuild turns the flags into
 * the compacted tree. */
hgs_status hgs_compact_mark(hgs_ctx *ctx, const hgs_view *views, int32_t n_views, float tau_min, float tau_max,
                            uint8_t *keep);

/* The compacted tree (Sec. 5.2) from the keep flags of hgs_compact_mark:
 * host work only, no context.  In (host): parent and child_count (int32[n],
 * the breadth-first layout hgs_upload takes) and keep (uint8[n]).  Every
 * kept node's parent becomes its nearest kept ancestor, so a node may get
 * more than 8 children (K in Eq. (alphap) is the child count).  Out (host,
 * each with room for n entries, filled up to *n_out): order (the old index
 * of every new node: breadth-first, root first, the children of a node
 * contiguous and in their old order), new_parent (-1 for the root),
 * new_child_begin (0 for a leaf) and new_child_count.  Node attributes and
 * boxes carry over unchanged (order indexes them).  HGS_ERR_INVALID_ARG for
 * NULL pointers, n out of range, a malformed topology, or a removed root or
 * leaf. */
hgs_status hgs_compact_rebuild(const int32_t *parent, const int32_t *child_count, const uint8_t *keep, int64_t n,
                               int32_t *order, int32_t *new_parent, int32_t *new_child_begin,
                               int32_t *new_child_count, int64_t *n_out);

typedef struct {
    int64_t cut;        /* cut nodes, all views */
    int64_t visible;    /* splats with a non-empty footprint */
    int64_t pairs;      /* (tile, splat) pairs */
    int64_t evaluated;  /* (pixel, splat) pairs whose alpha was computed */
    int64_t blended;    /* (pixel, splat) pairs that passed alpha >= 1/255 and were composited */
    float ms[8];        /* stage times when requested: cut, preprocess, visible+depth sort,
                           duplicate, tile sort, ranges, blend, total (0 when not timed) */
    uint64_t render_id; /* identifies this render for hgs_render_backward (never 0) */
} hgs_stats;

/* Render n_views views (host array `views`) into out_rgb[v] (host array of
 * device pointers; each float[height][width][3], overwritten).  n_views == 1
 * launches the stages one by one; n_views > 1 runs every view through one
 * sequence of launches (all cuts, one preprocess, one sort, one blend over
 * the tiles of every view) captured once into a HIP graph and replayed while
 * the view sizes stay the same.  `stats` (host, may be NULL) receives counts;
 * stats->ms is filled when stats->ms[0] < 0 on entry (costs event syncs).
 * Keeps the state hgs_render_backward needs, under a new render id (a
 * per-ctx counter, written to stats->render_id and returned by
 * hgs_last_render).  Synchronises the ctx stream once at the end (capacity
 * check); grows internal buffers and replays when a capacity was exceeded. */
hgs_status hgs_render(hgs_ctx *ctx, const hgs_view *views, int32_t n_views, float *const *out_rgb,
                      hgs_stats *stats);

/* Id and view count of the render whose state ctx holds for
 * hgs_render_backward (host outputs; either may be NULL): *render_id = 0
 * and *n_views = 0 when there is none (no render yet, or a later call such
 * as hgs_cut, hgs_bind_params, hgs_upload, hgs_set_tuning, hgs_compact_mark
 * or an hgs_adam_step on the bound parameters has replaced or invalidated
 * it).  Does not synchronise. */
hgs_status hgs_last_render(hgs_ctx *ctx, uint64_t *render_id, int32_t *n_views);

typedef struct {
    float *mean, *scale, *rot, *opacity, *sh; /* device, same layouts as the parameters; accumulated (+=) */
    float *dt;                                /* device, may be NULL: dL/dt per cut entry of the last render */
} hgs_grads;

/* Backward of the render `render_id` (its stats->render_id), which must be
 * the last hgs_render on this ctx, over its n_views views: dL_drgb[v] (host
 * array of n_views device pointers, each float[height][width][3] of view v
 * of that render) is dL/d(out_rgb[v]).  Gradients
 * of every node's parameters are ADDED to `out`; leaves get none (they are
 * frozen, Sec. 5.1 and Sec. 7.1); opacity gradients include the sign of the
 * absolute-value activation and are zero where the 0.99 clamp is active.
 * Per-tile blending state is recomputed from the final transmittance and
 * the index of the last contributor of each pixel (no per-pixel lists).
 * dL/dt is written (not added) when out->dt is given; with out->dt NULL the
 * blend backward skips its share of that work.
 * Errors: HGS_ERR_STATE when render_id is not the render whose state ctx
 * holds (a later render replaced it, or there is none: see
 * hgs_last_render); HGS_ERR_INVALID_ARG when n_views differs from that
 * render's view count or a pointer is NULL.  Does not synchronise. */
hgs_status hgs_render_backward(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *dL_drgb,
                               hgs_grads *out);

/* Loss of the hierarchy optimisation for the render `render_id` (the last
 * hgs_render on ctx, n_views views): the mean absolute difference between
 * its images out_rgb[v] and the targets, over every pixel and channel of
 * every view (the paper optimises the interior nodes against the training
 * images, Sec. 5.1; L1 is the image term of 3D Gaussian Splatting's loss),
 *   loss = (1/M) sum |C - C*|,   dL_drgb[v] = sign(C - C*) / M  (sign(0) = 0),
 * M = 3 x the pixel count of all views.  target and dL_drgb: host arrays of
 * n_views device pointers, float[height][width][3] of view v; dL_drgb is
 * written (it is the cotangent hgs_render_backward takes).  loss: device
 * pointer to one double, written.  The sum is taken in FP64 in a fixed
 * order.  Reads the images the render wrote, so they must be unchanged
 * since.  Queued on the ctx stream; does not synchronise.
 * Errors: HGS_ERR_STATE when render_id is not the render ctx holds;
 * HGS_ERR_INVALID_ARG when n_views differs from its view count or a pointer
 * is NULL. */
hgs_status hgs_l1_loss(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *target,
                       float *const *dL_drgb, double *loss);

/* Out-of-core rendering (Sec. 6.3: as the camera moves the cut is updated
 * and the nodes it needs are transferred to the GPU from CPU RAM, with a
 * cleanup every so many frames).  hgs_stream_begin moves ctx's Gaussian
 * parameters (236 B per node) to library-owned pinned host memory and keeps
 * on the device the topology and boxes (28 B per node, every cut reads
 * them) and a cache of `cache_nodes` parameter records.  Every later
 * hgs_render then, after its cut and before projecting, transfers the
 * records of the cut nodes and their parents that are not resident (the
 * GPU reads them from host memory), stamps every record it uses with the
 * frame (one frame per hgs_render), and renders from the cache: images are
 * those of the in-core render.  A render whose nodes do not fit in the free
 * slots returns HGS_ERR_CAPACITY (its image lacks them).  Parameters must
 * not be bound; hgs_render_backward, hgs_bind_params and hgs_adam_step
 * return HGS_ERR_STATE until hgs_stream_end, which copies the parameters
 * back to the device; hgs_upload and hgs_build also end it.  cache_nodes in
 * [1, n_nodes].  Both synchronise the ctx stream. */
hgs_status hgs_stream_begin(hgs_ctx *ctx, int64_t cache_nodes);
hgs_status hgs_stream_end(hgs_ctx *ctx);

/* Frees the cache slots whose records no render has used for more than
 * max_age frames (the paper's periodic cleanup).  Queued on the ctx stream. */
hgs_status hgs_stream_cleanup(hgs_ctx *ctx, int32_t max_age);

typedef struct {
    int64_t cache_nodes;        /* capacity */
    int64_t resident;           /* records in the cache */
    int64_t frame;              /* renders since hgs_stream_begin */
    int64_t requested;          /* records the last render requested (transferred unless overflow) */
    int64_t transferred_total;  /* records transferred since hgs_stream_begin */
    int32_t overflow;           /* the last render needed more free slots than there were */
} hgs_stream_stats;
/* State of the cache (synchronises the ctx stream). */
hgs_status hgs_stream_info(hgs_ctx *ctx, hgs_stream_stats *out);

/* One step of the optimiser of the hierarchy optimisation (Sec. 5.1, the
 * paragraph on optimising the generated hierarchy): interior nodes only,
 * the leaves stay unchanged; the paper does not name the optimiser for this
 * stage, so this is Adam as in 3D Gaussian Splatting, per element:
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p -= lr * (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps),
 * and g = 0 afterwards (the next hgs_render_backward accumulates a fresh
 * gradient).  All arrays are device pointers; index 0..4 = mean, scale,
 * rot, opacity, sh.  param and grad are in the parameter layouts of the
 * header (node-major, N nodes each; leaf entries are left untouched); m and
 * v hold the interior nodes only, node-major by interior rank (row q
 * belongs to the q-th interior node in ascending id order, as hgs_interior
 * lists them: n_interior x 3, 3, 4, 1, 48 floats), and must be zero before
 * step 1.  The arrays of rot and sh must be 16-byte aligned.  Queued on the
 * ctx stream; does not synchronise.  When the step updates the parameters
 * the renderer reads (the bound arrays), the next hgs_render_backward needs
 * a new hgs_render (HGS_ERR_STATE).
 * Errors: HGS_ERR_STATE without a hierarchy, HGS_ERR_INVALID_ARG for a NULL
 * or misaligned array, step < 1, or a non-finite / out-of-range
 * hyper-parameter. */
typedef struct {
    float *param[5];
    float *grad[5];
    float *m[5];
    float *v[5];
    float lr[5];  /* learning rate per parameter group */
    float beta1, beta2, eps;
    int64_t step; /* 1-based, for the bias correction */
} hgs_adam;
hgs_status hgs_adam_step(hgs_ctx *ctx, const hgs_adam *a);

/* The backward of render render_id with the optimiser step of Sec. 5.1
 * applied right away: the same parameters, moments and errors as
 * hgs_render_backward into gradient arrays that hold zero, followed by
 * hgs_adam_step on them, but the gradient of each interior node goes from
 * the gather's registers into its Adam update and is never stored.  Bit for
 * bit the same when both backwards form the same sums: always in the
 * deterministic mode (hgs_set_deterministic); by default the screen-space
 * sums are atomic and may differ in their last bits from run to run.  a->grad is not used (may be NULL); a->param, a->m and a->v as for
 * hgs_adam_step (interior nodes stepped, leaves untouched, every interior
 * node stepped, with gradient zero where no cut entry reached it); no dL/dt
 * output.  Arguments are checked as by the two calls (argument errors
 * change nothing).  Queued on the ctx stream; does not synchronise; when
 * the step updates the parameters the renderer reads, the state kept for
 * the backward is stale afterwards, as after hgs_adam_step. */
hgs_status hgs_backward_adam_step(hgs_ctx *ctx, uint64_t render_id, int32_t n_views, const float *const *dL_drgb,
                                  const hgs_adam *a);

/* Deterministic-reduction mode of hgs_render_backward (a checking aid): with
 * on = 1 the blend backward uses no floating-point atomics.  Within a tile,
 * each 4x4 pixel quarter keeps its partial sums in a slot of its own and the
 * quarters are added in a fixed order; each (tile, splat) pair stores its
 * 11 screen-space terms at the pair's position in the duplication order,
 * and every splat's terms are then summed over its tiles in that order.
 * Gradients are then bit-identical from run to run (in the default mode,
 * FP64 atomics make the order of the additions vary, which moves results in
 * their last bits).  Costs 88 bytes of device memory per (tile, splat) pair
 * (allocated at the next backward) and about one more pass over them; the
 * blend backward then stages 32 splats per batch, one workgroup per tile.
 * on = 0 restores the default.  HGS_ERR_INVALID_ARG for other values. */
hgs_status hgs_set_deterministic(hgs_ctx *ctx, int32_t on);

/* The interior nodes (those with children: the ones the optimisation of
 * Sec. 5.1 updates) of the uploaded or built hierarchy, in ascending id
 * order: the row order of the optimiser moments of hgs_adam_step.  *count
 * receives their number; when ids (a device pointer, the caller's) is not
 * NULL, the first min(cap, count) ids are copied into it, queued on the ctx
 * stream.  Errors: HGS_ERR_STATE without a hierarchy, HGS_ERR_INVALID_ARG
 * for a NULL count or a negative cap. */
hgs_status hgs_interior(hgs_ctx *ctx, int32_t *ids, int64_t cap, int64_t *count);

/* Tuning knobs of the blend stage and its backward (chosen by the
 * autotuner): tile edge tile_w x tile_h in {8x8, 16x8, 16x16, 32x16},
 * splats staged per batch (a multiple of 64 up to 1024; 0 = one per
 * thread), and the work distribution: persistent = 0 launches one workgroup
 * per tile, 1 a persistent grid of as many workgroups as the device holds
 * at once, which take tiles (longest lists first) from a device-side queue
 * until none is left.  Changing them keeps images bit-identical.
 * HGS_ERR_INVALID_ARG for other values. */
hgs_status hgs_set_tuning(hgs_ctx *ctx, int32_t tile_w, int32_t tile_h, int32_t batch, int32_t persistent);

/* Kernel timing for benchmarks: with profiling on, selected launches are
 * bracketed by HIP events on the stream they run on (in a multi-view render
 * the blend then runs right after the graph instead of inside it).
 * hgs_set_profiling resets the totals.  hgs_kernel_time synchronises and
 * returns the summed milliseconds and launch count of kernel `which`:
 * 0 blend, 1 blend backward, 2 preprocess backward together with the
 * gradient gather that follows it. */
hgs_status hgs_set_profiling(hgs_ctx *ctx, int32_t on);
hgs_status hgs_kernel_time(hgs_ctx *ctx, int32_t which, double *total_ms, int64_t *launches);

/* Counters of the last render and backward (synchronises): out[0..8] =
 * cut, visible, pairs, evaluated, blended, evaluated with t > 0,
 * backward evaluated, backward evaluated with t > 0, backward contributing
 * pairs.  At most n values are written. */
hgs_status hgs_counters(hgs_ctx *ctx, int64_t *out, int32_t n);

/* Read-only access to internal state of the last render/backward (device
 * pointers, valid until the next render on ctx), for tests and tools.
 * which: 0 cut node ids (int32, all views, view-major), 1 cut t (double),
 * 2 final transmittance per pixel (float, views concatenated, row-major),
 * 3 contributors processed per pixel (uint32: index within its tile's list
 * after the last blended splat, + 1; 0 if none), 4 blended splats per pixel
 * (uint32), 5 screen-space gradients of the last backward (double[visible]
 * [12], one row per visible splat: du, dv, dL/d(a, b, c) of the 2D
 * covariance through the conic, dA_n, dA_p, drgb(3), dt_alpha, unused), 6 cut
 * offsets per view (uint32[n_views + 1]), 7 per-tile ranges of the sorted
 * (tile, splat) pairs (uint32[tiles][2], tiles of all views), 8 row of buffer
 * 5 for each cut entry (uint32[cut], defined for visible entries).  *count
 * receives the element count. */
hgs_status hgs_get_buffer(hgs_ctx *ctx, int32_t which, const void **dev_ptr, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* HGS_H */
