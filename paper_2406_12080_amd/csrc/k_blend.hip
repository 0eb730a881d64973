// Per-tile alpha blending (forward) and its backward.
//
// One workgroup per tile of TW x TH pixels; each 64-lane wave owns an 8x8
// sub-tile, one lane per pixel.  The tile's splats (sorted front to back)
// are staged through LDS in batches of BATCH records; every lane walks the
// batch in order.  Per pixel and splat (Sec. 3 Eq. (alpha) with the
// projected Gaussian G; Eq. (alphap) generalised to K children, Sec. 5.2;
// the weight t of Eq. (t_interp) as the parent's weight; clamp of Sec. 7.3):
//   G     = exp(-q/2),  q = d^T conic d  (d = pixel centre - mean), evaluated
//           as exp2(-(u1^2 + u2^2)) with u_i = w_i . d on the conic's scaled
//           eigen-axes (see SplatRec)
//   a_n   = min(0.99, A_n G),  a_p = min(0.99, A_p G)
//   alpha = (1 - t) a_n + t (1 - (1 - a_p)^(1/K))     (= a_n when t = 0)
//   skip when alpha < 1/255; stop before T (1 - alpha) < 1e-4;
//   C += c alpha T;  T *= 1 - alpha.
// The backward walks each tile back to front from the final transmittance
// and the index of the last contributor of each pixel, recovering the
// transmittance in front of every splat by dividing by (1 - alpha) (no
// per-pixel lists), reduces each splat's gradient over rows of 16 lanes with
// DPP exchanges and over the rows and waves of the tile in LDS (FP32), and
// adds it once per tile, in FP64, to the splat's screen-space gradient.
#include <algorithm>
#include <map>
#include <mutex>

#include "hgs_internal.h"

namespace hgs {

namespace {

struct AlphaEval {
    float G, an, ap, apr, q, alpha, u1, u2;  // q = (1 - a_p)^(1/K), apr = 1 - q
    bool cn, cp;
};

// Staged splat, per 8x8 block of the tile: c = w . (block corner + 1/2 - mean)
// in FP64, so that a lane only adds w . (its offset inside the block): the
// result depends on the pixel alone, not on the tile size.
__device__ __forceinline__ void block_offsets(const SplatRec &r, const double4 &W, int bx, int by, float &c1,
                                              float &c2, float &dx0, float &dy0)
{
#pragma clang fp contract(off)
    const double dx = ((double)(bx - r.ax) + 0.5) - (double)r.fx;
    const double dy = ((double)(by - r.ay) + 0.5) - (double)r.fy;
    c1 = (float)(dx * W.x + dy * W.y);
    c2 = (float)(dx * W.z + dy * W.w);
    dx0 = (float)dx;
    dy0 = (float)dy;
}

// Identical instruction sequence in forward and backward (explicit FMAs, no
// other contraction), so that the backward reproduces the forward's
// decisions bit for bit.  `interp` (t > 0) is the same for every lane.
__device__ __forceinline__ void eval_alpha(const float4 &W, const float4 &O, float2 c, float lx, float ly,
                                           bool interp, AlphaEval &e)
{
#pragma clang fp contract(off)
    e.u1 = fmaf(ly, W.y, fmaf(lx, W.x, c.x));
    e.u2 = fmaf(ly, W.w, fmaf(lx, W.z, c.y));
    const float s = fmaf(e.u1, e.u1, e.u2 * e.u2);
    e.G = __builtin_amdgcn_exp2f(-s);
    const float an = O.x * e.G;
    e.cn = an > kAlphaMax;
    e.an = fminf(an, kAlphaMax);
    e.alpha = e.an;
    e.ap = 0.0f;
    e.apr = 0.0f;
    e.q = 1.0f;
    e.cp = false;
    if (interp) {
        const float ap = O.y * e.G;
        e.cp = ap > kAlphaMax;
        e.ap = fminf(ap, kAlphaMax);
        e.q = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(1.0f - e.ap) * O.w);
        e.apr = 1.0f - e.q;
        e.alpha = (1.0f - O.z) * e.an + O.z * e.apr;
    }
}

// True when no pixel of an 8x8 block can take the splat at alpha >= 1/255,
// so that the block may skip it.  On the conic's scaled eigen-axes the
// block's pixel centres lie in the box c + [0,7] a + [0,7] b (a = (w1x, w2x),
// b = (w1y, w2y), c = block corner offsets), and alpha <= Amax G with
// G = 2^-(u1^2 + u2^2) (Amax = A_n, or max(A_n, A_p) when t > 0: the pow
// of Eq. (alphap) never exceeds its argument).  The distance of the box from
// the origin is compared with log2(255 Amax) with a margin far above the
// FP32 rounding of either side; boxes wider than 64 (sub-pixel splats, whose
// offsets may cancel) are never skipped.
__device__ __forceinline__ bool block_dead(const float4 &W, float c1, float c2, float Amax)
{
    const float a1 = 7.0f * W.x, b1 = 7.0f * W.y, a2 = 7.0f * W.z, b2 = 7.0f * W.w;
    const float lo1 = c1 + fminf(a1, 0.0f) + fminf(b1, 0.0f), hi1 = c1 + fmaxf(a1, 0.0f) + fmaxf(b1, 0.0f);
    const float lo2 = c2 + fminf(a2, 0.0f) + fminf(b2, 0.0f), hi2 = c2 + fmaxf(a2, 0.0f) + fmaxf(b2, 0.0f);
    if (!(hi1 - lo1 <= 64.0f && hi2 - lo2 <= 64.0f)) return false;
    const float m1 = fmaxf(fmaxf(lo1, -hi1), 0.0f), m2 = fmaxf(fmaxf(lo2, -hi2), 0.0f);
    const float r2 = __builtin_amdgcn_logf(255.0f * Amax);  // log2
    return m1 * m1 + m2 * m2 > r2 * 1.001f + 1e-3f;
}

__device__ __forceinline__ int view_of_tile(const DevView *views, int nv, uint32_t tile)
{
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Staged copy of one splat for one tile.
struct Staged {
    float4 w, o, c;
    float2 u[8];
    uint32_t dead;  // bit bk: block bk skips the splat
};

template <int NB, int SX>
__device__ __forceinline__ void stage_one(const SplatRec &r, const double4 &W64, int ox, int oy, Staged &st)
{
    st.w = make_float4((float)W64.x, (float)W64.y, (float)W64.z, (float)W64.w);
    st.o = make_float4(r.An, r.Ap, r.t, r.invK);
    st.c = make_float4(r.r, r.g, r.b, 0.0f);
    const float amax = r.t > 0.0f ? fmaxf(r.An, r.Ap) : r.An;
    st.dead = 0u;
#pragma unroll
    for (int bk = 0; bk < NB; ++bk) {
        float c1, c2, d0, d1;
        block_offsets(r, W64, ox + (bk % SX) * 8, oy + (bk / SX) * 8, c1, c2, d0, d1);
        st.u[bk] = make_float2(c1, c2);
        st.dead |= block_dead(st.w, c1, c2, amax) ? 1u << bk : 0u;
    }
}

// Per-wave work counts (uint4 per wave, plain stores) are summed by
// k_stats_reduce into three consecutive counters: forward (evaluated,
// blended, evaluated with t > 0), backward (evaluated, evaluated with t > 0,
// contributing).  No contended atomics on the hot path.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Work distribution over tiles: either one workgroup per tile slot (grid =
// tile count, slot = workgroup index), or a persistent grid sized to the
// chip's resident workgroups, each taking runs of `chunk` consecutive slots
// from a device-side queue (a counter that the launch sequence clears first)
// until the slots run out.  Slots are handed out in the longest-first order
// either way; runs keep the one queue counter from serialising a million
// small tiles.
__device__ __forceinline__ uint32_t next_run(uint32_t *queue, uint32_t chunk, uint32_t *s_slot)
{
    if (threadIdx.x == 0) *s_slot = atomicAdd(queue, chunk);
    __syncthreads();
    const uint32_t slot = *s_slot;
    __syncthreads();  // every wave has its slot before lane 0 may overwrite it
    return slot;
}

template <int TW, int TH, int BATCH>
__device__ __forceinline__ void blend_tile(const DevView *__restrict__ views, int nv,
                                           const uint32_t *__restrict__ tile_order,
                                           const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_vals,
                                           const SplatRec *__restrict__ recs, const double4 *__restrict__ axes,
                                           float *__restrict__ T_final, uint32_t *__restrict__ n_last,
                                           uint32_t *__restrict__ n_blend, uint4 *__restrict__ wstats,
                                           uint32_t slot)
{
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int SX = TW / 8;
    constexpr int NB = (TW / 8) * (TH / 8);
    constexpr int PER = BATCH / NT;  // records staged per thread and batch
    static_assert(BATCH % NT == 0 && BATCH % 64 == 0 && NB <= 8, "tile/batch combination");
    __shared__ float4 s_w[BATCH], s_o[BATCH], s_c[BATCH];
    __shared__ float2 s_u[NB][BATCH];
    __shared__ uint64_t s_tm[BATCH / 64];  // bit j of word k: entry 64 k + j is interpolated (t > 0)
    __shared__ uint64_t s_dm[NB][BATCH / 64];  // likewise: block bk skips entry 64 k + j
    const uint32_t tile = tile_order[slot];  // longest lists first
    const int vi = view_of_tile(views, nv, tile);
    const DevView &V = views[vi];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ox = tx * TW, oy = ty * TH;
    const int px = ox + (w % SX) * 8 + (lane & 7), py = oy + (w / SX) * 8 + (lane >> 3);
    const bool inside = px < V.W && py < V.H;
    const float lx = (float)(lane & 7), ly = (float)(lane >> 3);
    const uint2 rg = ranges[tile];

    // T < 0 marks a finished pixel (or one outside the image); |T| is its
    // transmittance.  A pixel stops at the splat whose blend would take T
    // below kTMin; that splat was evaluated but not blended.
    float T = inside ? 1.0f : -1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    uint32_t last = 0, nb = 0;
    uint32_t n_eval = 0, n_eval_t = 0;  // wave totals (scalar): evaluated pairs, of them interpolated

    // records of the next batch, loaded while the current one is composited
    SplatRec nxt[PER];
    double4 nxw[PER];
    auto fetch = [&](uint32_t b0) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const uint32_t idx = b0 + p * NT + threadIdx.x;
            if (idx < rg.y) {
                const uint32_t sidx = pair_vals[idx];
                nxt[p] = recs[sidx];
                nxw[p] = axes[sidx];
            }
        }
    };
    if (rg.x < rg.y) fetch(rg.x);
    for (uint32_t b0 = rg.x; b0 < rg.y; b0 += BATCH) {
        if (__syncthreads_count(T > 0.0f) == 0) break;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int j = p * NT + threadIdx.x;
            const bool real = b0 + j < rg.y;
            Staged st;
            if (real) {
                stage_one<NB, SX>(nxt[p], nxw[p], ox, oy, st);
            } else {  // padding: alpha = 0 everywhere, skipped by every block
                st.w = st.o = st.c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) st.u[bk] = make_float2(0.0f, 0.0f);
                st.dead = (1u << NB) - 1u;
            }
            s_w[j] = st.w;
            s_o[j] = st.o;
            s_c[j] = st.c;
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) s_u[bk][j] = st.u[bk];
            const uint64_t m = __ballot(real && st.o.z > 0.0f);
            if (lane == 0) s_tm[j >> 6] = m;
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) {
                const uint64_t dm = __ballot((st.dead >> bk) & 1u);
                if (lane == 0) s_dm[bk][j >> 6] = dm;
            }
        }
        __syncthreads();
        if (b0 + BATCH < rg.y) fetch(b0 + BATCH);
        if (__ballot(T > 0.0f) == 0ull) continue;
        const int cnt = (int)min((uint32_t)BATCH, rg.y - b0), cnt4 = (cnt + 3) & ~3;
        const uint32_t jb = b0 - rg.x + 1u;  // 1-based list position of entry 0
        uint64_t tm = 0, dm = 0;
        for (int j0 = 0; j0 < cnt4; j0 += 4) {
            if ((j0 & 63) == 0) {
                tm = uniform_u64(s_tm[j0 >> 6]);
                dm = uniform_u64(s_dm[w][j0 >> 6]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u;
                if ((dm >> (j & 63)) & 1ull) continue;  // no pixel of this block reaches 1/255
                const uint32_t bit = (uint32_t)(tm >> (j & 63)) & 1u;
                // work counts from the wave's live mask (scalar unit only)
                const uint32_t n_live = (uint32_t)__popcll(__ballot(T > 0.0f));
                n_eval += n_live;
                n_eval_t += bit ? n_live : 0u;
                AlphaEval e;
                eval_alpha(s_w[j], s_o[j], s_u[w][j], lx, ly, bit != 0u, e);
                if (T > 0.0f && e.alpha >= kAlphaMin) {
                    const float Tn = T * (1.0f - e.alpha);
                    const bool stop = Tn < kTMin;
                    const float4 Cc = s_c[j];
                    const float wgt = stop ? 0.0f : e.alpha * T;
                    C0 += Cc.x * wgt;
                    C1 += Cc.y * wgt;
                    C2 += Cc.z * wgt;
                    nb += stop ? 0u : 1u;
                    last = stop ? last : jb + (uint32_t)j;
                    T = stop ? -T : Tn;
                }
            }
            if (__ballot(T > 0.0f) == 0ull) break;
        }
    }
    if (inside) {
        const size_t p = (size_t)py * V.W + px;
        float *o = V.out_rgb + 3 * p;
        o[0] = C0;
        o[1] = C1;
        o[2] = C2;
        const size_t g = (size_t)V.pix_base + p;
        T_final[g] = fabsf(T);
        n_last[g] = last;
        n_blend[g] = nb;
    }
    uint32_t nb_w = nb;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nb_w += (uint32_t)__shfl_xor((int)nb_w, d, 64);
    if (lane == 0) wstats[(size_t)slot * NW + w] = make_uint4(n_eval, nb_w, n_eval_t, 0u);
}

template <int TW, int TH, int BATCH, bool PERSIST>
__global__ __launch_bounds__(TW *TH) void k_blend(const DevView *__restrict__ views, int nv,
                                                  const uint32_t *__restrict__ tile_order,
                                                  const uint2 *__restrict__ ranges,
                                                  const uint32_t *__restrict__ pair_vals,
                                                  const SplatRec *__restrict__ recs,
                                                  const double4 *__restrict__ axes, float *__restrict__ T_final,
                                                  uint32_t *__restrict__ n_last, uint32_t *__restrict__ n_blend,
                                                  uint4 *__restrict__ wstats, uint32_t n_tiles,
                                                  uint32_t *__restrict__ queue, uint32_t chunk)
{
    if constexpr (!PERSIST) {
        blend_tile<TW, TH, BATCH>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final, n_last, n_blend,
                                  wstats, blockIdx.x);
    } else {
        __shared__ uint32_t s_slot;
        for (;;) {
            const uint32_t first = next_run(queue, chunk, &s_slot);
            if (first >= n_tiles) break;
            const uint32_t last = min(n_tiles, first + chunk);
            for (uint32_t slot = first; slot < last; ++slot) {
                blend_tile<TW, TH, BATCH>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final, n_last,
                                          n_blend, wstats, slot);
                __syncthreads();  // LDS of this tile read by every wave before the next stages
            }
        }
    }
}

// Cross-row halvings with the gfx950 lane swaps: permlane32_swap(x, y) moves
// the upper half of x and the lower half of y into each other's place, so
// x + y afterwards holds, on lanes 0-31, x summed over lanes l and l + 32
// and, on lanes 32-63, y summed likewise (permlane16_swap does the same for
// odd and even rows of 16): one swap and one add per pair of values.
__device__ __forceinline__ float swap_add32(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap_add16(float x, float y)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the 64 lanes of 12 per-lane values v[0..11] (v[11] only when DT):
// two swap steps (across halves, then across rows), two in-row halvings with
// DPP (partners l ^ 8, then l ^ 7, each keeping one of two values), and a sum
// over the quad (l ^ 2, l ^ 1).  Every lane of quad q = l >> 2 ends with the
// total of value wave_slot(l) (-1: nothing).
template <bool DT>
__device__ __forceinline__ float wave_reduce12(const float (&v)[12], int lane)
{
    const float S0 = swap_add32(v[0], v[1]), S1 = swap_add32(v[2], v[3]), S2 = swap_add32(v[4], v[5]);
    const float S3 = swap_add32(v[6], v[7]), S4 = swap_add32(v[8], v[9]);
    const float S5 = swap_add32(v[10], DT ? v[11] : 0.0f);  // slot 11 (dL/dt) only when asked for
    // rows 0..3 of Z0: v0 v2 v1 v3; Z1: v4 v6 v5 v7; Z2: v8 v10 v9 v11
    const float Z0 = swap_add16(S0, S1), Z1 = swap_add16(S2, S3), Z2 = swap_add16(S4, S5);
    const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
    const float R0 = (b3 ? Z1 : Z0) + dpp_move<0x128>(b3 ? Z0 : Z1);
    const float R1 = (b3 ? 0.0f : Z2) + dpp_move<0x128>(b3 ? Z2 : 0.0f);
    float F = (b2 ? R1 : R0) + dpp_move<0x141>(b2 ? R0 : R1);
    F += dpp_move<0x4E>(F);
    F += dpp_move<0xB1>(F);
    return F;
}

__device__ __forceinline__ int wave_slot(int lane)
{
    // by row (lane >> 4) and (b2, b3) = bits 2 and 3 of the lane
    constexpr int8_t kSlot[4][4] = {{0, 4, 8, -1}, {2, 6, 10, -1}, {1, 5, 9, -1}, {3, 7, 11, -1}};
    return kSlot[lane >> 4][((lane >> 2) & 1) * 2 + ((lane >> 3) & 1)];
}

constexpr int kG = 12;  // floats per splat in the screen-space gradient

// Per-lane gradient slots of one (pixel, splat) pair, summed over the tile:
//   0       S = h                         with h = G dL/dG (G the Gaussian)
//   1, 2    P'_i = h v_i
//   3..5    Q'_11, Q'_12, Q'_22 = h v_1 v_1, h v_1 v_2, h v_2 v_2
//   6, 7    dL/dA_n, dL/dA_p (A = kappa |o|)
//   8..10   dL/d colour
//   11      dL/dt through alpha (only when the caller asks for dL/dt)
// Here v = u - c is the pixel's position on the conic's scaled eigen-axes
// relative to the tile's corner pixel (c, formed in FP64 at staging): v is
// the pixel's offset inside the tile mapped by the axes.  The moments about
// the splat's centre follow in FP64 at the flush, P = P' + c S and
// Q = Q' + c P'^T + P' c^T + c c^T S.  Taken directly about the centre, the
// moments of a large splat whose centre lies far off screen are dominated
// by c S and c c^T S, and the mean and covariance gradients built from them
// cancel almost entirely in the chain through the projection: separately
// rounded FP32 sums of P and Q then leave errors far above the result.  With
// the moments about the corner both large parts carry the one rounded S, and
// the cancellation removes its error with it.
// The screen-space gradient follows from the tile sums by the splat's
// (per-tile constant) axes: with g = conic d = (u1 w1 + u2 w2) / kHalfLog2e
// and G = exp(-q/2), dL/dmean = sum h g and dL/dSigma2' = -sum (h / 2) g g^T
// (the covariance gradient through the conic), both linear in P and Q.
__device__ __forceinline__ void screen_grad(const float4 &W, const double P[2], const double Q[3], double out[5])
{
    const double k = 1.0 / kHalfLog2e;
    const double wx = W.x, wy = W.y, wz = W.z, ww = W.w;
    const double P1 = P[0], P2 = P[1], Q11 = Q[0], Q12 = Q[1], Q22 = Q[2];
    out[0] = k * (wx * P1 + wz * P2);
    out[1] = k * (wy * P1 + ww * P2);
    // (a, b, c) = (xx, 2 xy, yy) of sum (h / 2) g g^T, entering dL/dSigma2' with a minus
    // sign that the chain below takes as -dq = h / 2
    out[2] = 0.5 * k * k * (wx * wx * Q11 + 2.0 * wx * wz * Q12 + wz * wz * Q22);
    out[3] = k * k * (wx * wy * Q11 + (wx * ww + wz * wy) * Q12 + wz * ww * Q22);
    out[4] = 0.5 * k * k * (wy * wy * Q11 + 2.0 * wy * ww * Q12 + ww * ww * Q22);
}

// Offsets of the tile's corner pixel centre on the scaled eigen-axes, in FP64.
__device__ __forceinline__ double2 corner_offsets(const SplatRec &r, const double4 &W, int ox, int oy)
{
#pragma clang fp contract(off)
    const double dx = ((double)(ox - r.ax) + 0.5) - (double)r.fx;
    const double dy = ((double)(oy - r.ay) + 0.5) - (double)r.fy;
    return make_double2(dx * W.x + dy * W.y, dx * W.z + dy * W.w);
}

template <int TW, int TH, int BATCH, bool DT>
__device__ __forceinline__ void blend_bwd_tile(const DevView *__restrict__ views, int nv,
                                               const uint32_t *__restrict__ tile_order,
                                               const uint2 *__restrict__ ranges,
                                               const uint32_t *__restrict__ pair_vals,
                                               const SplatRec *__restrict__ recs, const double4 *__restrict__ axes,
                                               const float *__restrict__ T_final,
                                               const uint32_t *__restrict__ n_last,
                                               const uint32_t *__restrict__ vis_rank, double *__restrict__ sgrad,
                                               uint4 *__restrict__ wstats, uint32_t tslot)
{
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int SX = TW / 8;
    constexpr int NB = (TW / 8) * (TH / 8);
    __shared__ float4 s_w[BATCH], s_o[BATCH], s_c[BATCH];
    __shared__ float2 s_u[NB][BATCH];  // c1, c2
    __shared__ uint32_t s_id[BATCH];
    __shared__ __align__(16) float s_g[BATCH][kG];
    __shared__ double s_d[BATCH * 11];  // the flushed terms, splat-major
    __shared__ double2 s_ref[BATCH];    // the tile corner's offsets on the axes (FP64)
    __shared__ uint32_t s_max;
    const uint32_t tile = tile_order[tslot];  // longest lists first
    const int vi = view_of_tile(views, nv, tile);
    const DevView &V = views[vi];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ox = tx * TW, oy = ty * TH;
    const int px = ox + (w % SX) * 8 + (lane & 7), py = oy + (w / SX) * 8 + (lane >> 3);
    const bool inside = px < V.W && py < V.H;
    const float lx = (float)(lane & 7), ly = (float)(lane >> 3);
    // the pixel's offset from the tile corner (the moments' reference)
    const float lxt = (float)(px - ox), lyt = (float)(py - oy);
    const uint2 rg = ranges[tile];
    const int slot = wave_slot(lane);
    const bool writer = (lane & 3) == 0 && slot >= 0;

    float T = 1.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
    uint32_t last = 0;
    if (inside) {
        const size_t p = (size_t)py * V.W + px;
        const size_t g = (size_t)V.pix_base + p;
        T = T_final[g];
        last = n_last[g];
        g0 = V.dL[3 * p];
        g1 = V.dL[3 * p + 1];
        g2 = V.dL[3 * p + 2];
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    uint32_t wm = last;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wm = max(wm, (uint32_t)__shfl_xor((int)wm, d, 64));
    if (lane == 0) atomicMax(&s_max, wm);
    __syncthreads();
    const uint32_t end = rg.x + s_max;
    float R0 = 0.0f, R1 = 0.0f, R2 = 0.0f;  // colour composited behind the current splat
    uint32_t n_eval = 0, n_eval_t = 0, n_con = 0;  // wave totals (scalar)

    for (uint32_t hi = end; hi > rg.x;) {
        const uint32_t lo = hi - rg.x > (uint32_t)BATCH ? hi - BATCH : rg.x;
        const int cnt = (int)(hi - lo);
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const uint32_t sidx = pair_vals[lo + j];
            const SplatRec r = recs[sidx];
            const double4 W64 = axes[sidx];
            s_id[j] = vis_rank[sidx];  // gradient row
            s_w[j] = make_float4((float)W64.x, (float)W64.y, (float)W64.z, (float)W64.w);
            s_o[j] = make_float4(r.An, r.Ap, r.t, r.invK);
            s_c[j] = make_float4(r.r, r.g, r.b, 0.0f);
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) {
                float c1, c2, d0, d1;
                block_offsets(r, W64, ox + (bk % SX) * 8, oy + (bk / SX) * 8, c1, c2, d0, d1);
                s_u[bk][j] = make_float2(c1, c2);
            }
            s_ref[j] = corner_offsets(r, W64, ox, oy);
#pragma unroll
            for (int q = 0; q < kG; ++q) s_g[j][q] = 0.0f;
        }
        __syncthreads();
        for (int j = cnt - 1; j >= 0; --j) {
            const uint32_t li = lo - rg.x + (uint32_t)j;
            const bool in_range = li < last;
            const uint64_t live = __ballot(in_range);
            if (live == 0ull) continue;
            const float4 Wv = s_w[j], Ov = s_o[j];
            const float2 U = s_u[w][j];
            const bool interp = __builtin_amdgcn_readfirstlane(__float_as_int(Ov.z)) > 0;
            AlphaEval e;
            eval_alpha(Wv, Ov, U, lx, ly, interp, e);
            const bool contrib = in_range && e.alpha >= kAlphaMin;
            const uint64_t cm = __ballot(contrib);
            n_eval += (uint32_t)__popcll(live);
            n_eval_t += interp ? (uint32_t)__popcll(live) : 0u;
            if (cm == 0ull) continue;
            n_con += (uint32_t)__popcll(cm);
            // every lane runs the update; a non-contributing lane has a = 0 and
            // dL/dalpha = 0, which leaves T and R as they are and all slots 0
            const float4 Cc = s_c[j];
            const float a = contrib ? e.alpha : 0.0f;
            T = T * __builtin_amdgcn_rcpf(1.0f - a);
            const float dal_raw = T * ((Cc.x - R0) * g0 + (Cc.y - R1) * g1 + (Cc.z - R2) * g2);
            const float dal = contrib ? dal_raw : 0.0f;
            const float aT = a * T;
            float v[12];
            v[8] = aT * g0;
            v[9] = aT * g1;
            v[10] = aT * g2;
            R0 = a * Cc.x + (1.0f - a) * R0;
            R1 = a * Cc.y + (1.0f - a) * R1;
            R2 = a * Cc.z + (1.0f - a) * R2;
            float dan = dal, dap = 0.0f;
            v[11] = 0.0f;
            if (interp) {
                dan = (1.0f - Ov.z) * dal;
                const float dapr = Ov.z * dal;
                if constexpr (DT) v[11] = (e.apr - e.an) * dal;
                // d apr / d a_p = (1/K) (1 - a_p)^(1/K - 1) = (1/K) q / (1 - a_p)
                dap = dapr * Ov.w * (e.q * __builtin_amdgcn_rcpf(1.0f - e.ap));
            }
            const float dan_c = e.cn ? 0.0f : dan, dap_c = e.cp ? 0.0f : dap;
            v[6] = dan_c * e.G;
            v[7] = dap_c * e.G;
            const float h = e.G * (dan_c * Ov.x + dap_c * Ov.y);  // G dL/dG
            const float v1 = fmaf(lyt, Wv.y, lxt * Wv.x), v2 = fmaf(lyt, Wv.w, lxt * Wv.z);
            v[0] = h;
            v[1] = h * v1;
            v[2] = h * v2;
            v[3] = v[1] * v1;
            v[4] = v[1] * v2;
            v[5] = v[2] * v2;
            const float tot = wave_reduce12<DT>(v, lane);
            if (writer && tot != 0.0f) {
                if constexpr (NW == 1) s_g[j][slot] = tot;
                else atomicAdd(&s_g[j][slot], tot);
            }
        }
        __syncthreads();
        // flush: one lane per splat turns the tile's partial sums into the
        // 11 screen-space terms (FP64); then the terms of all splats go out
        // as consecutive atomics, row by row
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const float4 a = *reinterpret_cast<const float4 *>(&s_g[j][0]);
            const float4 b = *reinterpret_cast<const float4 *>(&s_g[j][4]);
            const float4 c = *reinterpret_cast<const float4 *>(&s_g[j][8]);
            // moments about the splat's centre from those about the tile corner
            const double2 cr = s_ref[j];
            const double S = a.x, P1 = a.y, P2 = a.z, Q11 = a.w, Q12 = b.x, Q22 = b.y;
            const double P[2] = {P1 + cr.x * S, P2 + cr.y * S};
            const double Q[3] = {Q11 + 2.0 * cr.x * P1 + cr.x * cr.x * S,
                                 Q12 + cr.x * P2 + cr.y * P1 + cr.x * cr.y * S,
                                 Q22 + 2.0 * cr.y * P2 + cr.y * cr.y * S};
            double sc[5];
            screen_grad(s_w[j], P, Q, sc);
            double *d = s_d + j * 11;
#pragma unroll
            for (int q = 0; q < 5; ++q) d[q] = sc[q];
            d[5] = (double)b.z;
            d[6] = (double)b.w;
            d[7] = (double)c.x;
            d[8] = (double)c.y;
            d[9] = (double)c.z;
            d[10] = (double)c.w;
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < cnt * 11; idx += NT) {
            const double val = s_d[idx];
            const int j = idx / 11, q = idx - 11 * j;
            if (val != 0.0) unsafeAtomicAdd(&sgrad[(size_t)s_id[j] * kG + q], val);
        }
        __syncthreads();
        hi = lo;
    }
    if (lane == 0) wstats[(size_t)tslot * NW + w] = make_uint4(n_eval, n_eval_t, n_con, 0u);
}

template <int TW, int TH, int BATCH, bool DT, bool PERSIST>
__global__ __launch_bounds__(TW *TH) void k_blend_bwd(const DevView *__restrict__ views, int nv,
                                                      const uint32_t *__restrict__ tile_order,
                                                      const uint2 *__restrict__ ranges,
                                                      const uint32_t *__restrict__ pair_vals,
                                                      const SplatRec *__restrict__ recs,
                                                      const double4 *__restrict__ axes,
                                                      const float *__restrict__ T_final,
                                                      const uint32_t *__restrict__ n_last,
                                                      const uint32_t *__restrict__ vis_rank,
                                                      double *__restrict__ sgrad, uint4 *__restrict__ wstats,
                                                      uint32_t n_tiles, uint32_t *__restrict__ queue,
                                                      uint32_t chunk)
{
    if constexpr (!PERSIST) {
        blend_bwd_tile<TW, TH, BATCH, DT>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final, n_last,
                                          vis_rank, sgrad, wstats, blockIdx.x);
    } else {
        __shared__ uint32_t s_slot;
        for (;;) {
            const uint32_t first = next_run(queue, chunk, &s_slot);
            if (first >= n_tiles) break;
            const uint32_t last = min(n_tiles, first + chunk);
            for (uint32_t slot = first; slot < last; ++slot) {
                blend_bwd_tile<TW, TH, BATCH, DT>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final,
                                                  n_last, vis_rank, sgrad, wstats, slot);
                __syncthreads();  // LDS of this tile read by every wave before the next stages
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_stats_reduce(const uint4 *__restrict__ s, uint32_t n,
                                                      unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long s_p[4][3];
    unsigned long long a = 0, b = 0, c = 0;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        const uint4 v = s[i];
        a += v.x;
        b += v.y;
        c += v.z;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        a += __shfl_xor(a, d, 64);
        b += __shfl_xor(b, d, 64);
        c += __shfl_xor(c, d, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_p[w][0] = a;
        s_p[w][1] = b;
        s_p[w][2] = c;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long t = s_p[0][threadIdx.x] + s_p[1][threadIdx.x] + s_p[2][threadIdx.x] +
                                     s_p[3][threadIdx.x];
        if (t) atomicAdd(&out[threadIdx.x], t);
    }
}

// Workgroups of `kernel` that the whole chip holds at once (CUs times the
// occupancy at `threads` per workgroup): the grid of a persistent launch.
// Looked up once per kernel.
template <typename K>
uint32_t resident_grid(K kernel, int threads)
{
    static std::mutex mu;
    static std::map<const void *, uint32_t> cache;
    std::lock_guard<std::mutex> lock(mu);
    const void *key = reinterpret_cast<const void *>(kernel);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0);
    const uint32_t g = (uint32_t)std::max(1, std::max(cus, 1) * std::max(per, 1));
    cache[key] = g;
    return g;
}

// Slots per queue ticket of a persistent launch of g workgroups over
// n_tiles slots: about a sixteenth of each workgroup's share, so that the
// last tickets still spread over the grid, and at most 32.
uint32_t queue_run(uint32_t n_tiles, uint32_t g)
{
    const uint32_t share = n_tiles / std::max(g, 1u);
    return std::min(32u, std::max(1u, share / 16u));
}

template <int TW, int TH, int BATCH>
void launch_blend_t(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                    const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, float *T_final,
                    uint32_t *n_last, uint32_t *n_blend, uint4 *wstats, bool persist, uint32_t *queue,
                    hipStream_t st)
{
    if (persist) {
        auto k = k_blend<TW, TH, BATCH, true>;
        const uint32_t g = std::min(n_tiles, resident_grid(k, TW * TH));
        launch_fill_u32(queue, 0u, 1, st);
        hipLaunchKernelGGL(k, dim3(g), dim3(TW * TH), 0, st, views, nv, order, ranges, pair_vals, recs, axes,
                           T_final, n_last, n_blend, wstats, n_tiles, queue, queue_run(n_tiles, g));
    } else {
        hipLaunchKernelGGL((k_blend<TW, TH, BATCH, false>), dim3(n_tiles), dim3(TW * TH), 0, st, views, nv, order,
                           ranges, pair_vals, recs, axes, T_final, n_last, n_blend, wstats, n_tiles, queue, 1u);
    }
}

template <int TW, int TH, int B, bool DT>
void launch_blend_bwd_dt(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                         const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, const float *T_final,
                         const uint32_t *n_last, const uint32_t *vis_rank, double *sgrad, uint4 *wstats, bool persist,
                         uint32_t *queue, hipStream_t st)
{
    if (persist) {
        auto k = k_blend_bwd<TW, TH, B, DT, true>;
        const uint32_t g = std::min(n_tiles, resident_grid(k, TW * TH));
        launch_fill_u32(queue, 0u, 1, st);
        hipLaunchKernelGGL(k, dim3(g), dim3(TW * TH), 0, st, views, nv, order, ranges, pair_vals, recs, axes, T_final,
                           n_last, vis_rank, sgrad, wstats, n_tiles, queue, queue_run(n_tiles, g));
    } else {
        hipLaunchKernelGGL((k_blend_bwd<TW, TH, B, DT, false>), dim3(n_tiles), dim3(TW * TH), 0, st, views, nv, order,
                           ranges, pair_vals, recs, axes, T_final, n_last, vis_rank, sgrad, wstats, n_tiles, queue,
                           1u);
    }
}

template <int TW, int TH, int BATCH>
void launch_blend_bwd_t(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                        const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, const float *T_final,
                        const uint32_t *n_last, const uint32_t *vis_rank, double *sgrad, uint4 *wstats,
                        bool want_dt, bool persist, uint32_t *queue, hipStream_t st)
{
    // the backward stages at most 32 splats per wave and step: its LDS holds
    // the FP32 partial sums and the FP64 flushed terms of every staged
    // splat, and a smaller footprint keeps more tiles resident per CU
    constexpr int BMAX = 32 * (TW * TH / 64);
    constexpr int B = BATCH < BMAX ? BATCH : BMAX;
    if (want_dt)
        launch_blend_bwd_dt<TW, TH, B, true>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final,
                                             n_last, vis_rank, sgrad, wstats, persist, queue, st);
    else
        launch_blend_bwd_dt<TW, TH, B, false>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final,
                                              n_last, vis_rank, sgrad, wstats, persist, queue, st);
}

}  // namespace

// Supported (tile, batch) combinations; batch 0 means one record per thread.
#define HGS_BLEND_CASES(X)                                                                                            \
    X(8, 8, 64) X(8, 8, 128) X(8, 8, 256) X(16, 8, 128) X(16, 8, 256) X(16, 16, 256) X(16, 16, 512) X(32, 16, 512)

template <int TW, int TH, int BATCH>
void prepare_t()
{
    constexpr int BMAX = 32 * (TW * TH / 64);
    constexpr int B = BATCH < BMAX ? BATCH : BMAX;
    (void)resident_grid(k_blend<TW, TH, BATCH, true>, TW * TH);
    (void)resident_grid(k_blend_bwd<TW, TH, B, true, true>, TW * TH);
    (void)resident_grid(k_blend_bwd<TW, TH, B, false, true>, TW * TH);
}

void blend_prepare(int tw, int th, int batch)
{
    if (batch == 0) batch = tw * th;
#define X(a, b, c) \
    if (tw == a && th == b && batch == c) return prepare_t<a, b, c>();
    HGS_BLEND_CASES(X)
#undef X
}

bool blend_supported(int tw, int th, int batch)
{
    if (batch == 0) batch = tw * th;
#define X(a, b, c) \
    if (tw == a && th == b && batch == c) return true;
    HGS_BLEND_CASES(X)
#undef X
    return false;
}

static void launch_blend_cfg(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order,
                             const uint2 *ranges, const uint32_t *pair_vals, const SplatRec *recs,
                             const double4 *axes, float *T_final, uint32_t *n_last, uint32_t *n_blend, uint4 *wstats,
                             int tw, int th, int batch, bool persist, uint32_t *queue, hipStream_t st)
{
#define X(a, b, c)                                                                                           \
    if (tw == a && th == b && batch == c)                                                                    \
        return launch_blend_t<a, b, c>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last, \
                                       n_blend, wstats, persist, queue, st);
    HGS_BLEND_CASES(X)
#undef X
}

void launch_blend(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                  const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, float *T_final,
                  uint32_t *n_last, uint32_t *n_blend, uint4 *wstats, Counters *ctr, int tw, int th, int batch,
                  bool persist, uint32_t *queue, hipStream_t st)
{
    if (batch == 0) batch = tw * th;
    if (!n_tiles) return;
    const uint32_t nst = n_tiles * (uint32_t)(tw * th / 64);
    launch_blend_cfg(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last, n_blend, wstats, tw,
                     th, batch, persist, queue, st);
    hipLaunchKernelGGL(k_stats_reduce, dim3(256), dim3(256), 0, st, wstats, nst, &ctr->evaluated);
}

void launch_blend_backward(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order,
                           const uint2 *ranges, const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes,
                           const float *T_final, const uint32_t *n_last, const uint32_t *vis_rank, double *sgrad,
                           uint4 *wstats, Counters *ctr, int tw, int th, int batch, bool want_dt, bool persist,
                           uint32_t *queue, hipStream_t st)
{
    if (batch == 0) batch = tw * th;
    if (!n_tiles) return;
#define X(a, b, c)                                                                                                 \
    if (tw == a && th == b && batch == c) {                                                                        \
        launch_blend_bwd_t<a, b, c>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last,    \
                                    vis_rank, sgrad, wstats, want_dt, persist, queue, st);                         \
        hipLaunchKernelGGL(k_stats_reduce, dim3(256), dim3(256), 0, st, wstats,                                    \
                           n_tiles * (uint32_t)(tw * th / 64), &ctr->bwd_evaluated);                               \
        return;                                                                                                    \
    }
    HGS_BLEND_CASES(X)
#undef X
}

}  // namespace hgs
