// Per-tile alpha blending (forward) and its backward.
//
// One workgroup per tile of TW x TH pixels; each 64-lane wave owns an 8x8
// sub-tile, one lane per pixel, and each row of 16 lanes one 4x4 quarter of
// it.  The tile's splats (sorted front to back) are staged through LDS in
// batches of BATCH records, each with one bit per quarter telling whether
// any pixel of the quarter can reach alpha = 1/255.  Every quarter walks the
// batch in order over the splats it may take only (a small splat touches
// one or two of them), so that the four quarters of a wave step through
// different splats together.  Per pixel and splat (Sec. 3 Eq. (alpha) with the
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
// DPP exchanges and over the rows and waves of the tile in LDS (FP64 atomics), and
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

// True when no pixel of a square of (E + 1) x (E + 1) pixels can take the
// splat at alpha >= 1/255, so that the square may skip it.  On the conic's
// scaled eigen-axes the square's pixel centres lie in the box
// c + [0,E] a + [0,E] b (a = (w1x, w2x), b = (w1y, w2y), c = the offsets of
// its corner pixel), and alpha <= Amax G with G = 2^-(u1^2 + u2^2)
// (Amax = A_n, or max(A_n, A_p) when t > 0: the pow of Eq. (alphap) never
// exceeds its argument).  The distance of the box from the origin is
// compared with log2(255 Amax) with a margin far above the FP32 rounding of
// either side; boxes wider than 64 (sub-pixel splats, whose offsets may
// cancel) are never skipped.
template <int E>
__device__ __forceinline__ bool square_dead(const float4 &W, float c1, float c2, float Amax)
{
    constexpr float e = (float)E;
    const float a1 = e * W.x, b1 = e * W.y, a2 = e * W.z, b2 = e * W.w;
    const float lo1 = c1 + fminf(a1, 0.0f) + fminf(b1, 0.0f), hi1 = c1 + fmaxf(a1, 0.0f) + fmaxf(b1, 0.0f);
    const float lo2 = c2 + fminf(a2, 0.0f) + fminf(b2, 0.0f), hi2 = c2 + fmaxf(a2, 0.0f) + fmaxf(b2, 0.0f);
    if (!(hi1 - lo1 <= 64.0f && hi2 - lo2 <= 64.0f)) return false;
    const float m1 = fmaxf(fmaxf(lo1, -hi1), 0.0f), m2 = fmaxf(fmaxf(lo2, -hi2), 0.0f);
    const float r2 = __builtin_amdgcn_logf(255.0f * Amax);  // log2
    return m1 * m1 + m2 * m2 > r2 * 1.001f + 1e-3f;
}

// Pixel of lane l inside its wave's 8x8 block: quarter l >> 4 is the 4x4
// square at ((q & 1) 4, (q >> 1) 4), rows of four lanes inside it.
__device__ __forceinline__ int quarter_x(int lane) { return ((lane >> 4) & 1) * 4 + (lane & 3); }
__device__ __forceinline__ int quarter_y(int lane) { return (lane >> 5) * 4 + ((lane >> 2) & 3); }

// Quarter mask of a staged splat: bit 4 bk + q set when some pixel of
// quarter q of block bk may take the splat (square_dead on the quarter).
template <int NB>
__device__ __forceinline__ uint32_t quarter_live(const float4 &W, const float2 (&u)[8], float amax)
{
    uint32_t live = 0u;
#pragma unroll
    for (int bk = 0; bk < NB; ++bk)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float sx = (float)((q & 1) * 4), sy = (float)((q >> 1) * 4);
            const float c1 = fmaf(sy, W.y, fmaf(sx, W.x, u[bk].x)), c2 = fmaf(sy, W.w, fmaf(sx, W.z, u[bk].y));
            live |= square_dead<3>(W, c1, c2, amax) ? 0u : 1u << (4 * bk + q);
        }
    return live;
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
    uint32_t live;  // bit 4 bk + q: quarter q of block bk may take the splat
};

template <int NB, int SX>
__device__ __forceinline__ void stage_one(const SplatRec &r, const double4 &W64, int ox, int oy, Staged &st)
{
    st.w = make_float4((float)W64.x, (float)W64.y, (float)W64.z, (float)W64.w);
    st.o = make_float4(r.An, r.Ap, r.t, r.invK);
    st.c = make_float4(r.r, r.g, r.b, 0.0f);
#pragma unroll
    for (int bk = 0; bk < NB; ++bk) {
        float c1, c2, d0, d1;
        block_offsets(r, W64, ox + (bk % SX) * 8, oy + (bk / SX) * 8, c1, c2, d0, d1);
        st.u[bk] = make_float2(c1, c2);
    }
    st.live = quarter_live<NB>(st.w, st.u, r.t > 0.0f ? fmaxf(r.An, r.Ap) : r.An);
}

// Per-wave work counts (uint4 per wave, plain stores) are summed by
// k_stats_reduce into three consecutive counters: forward (evaluated,
// blended, evaluated with t > 0), backward (evaluated, evaluated with t > 0,
// contributing).  No contended atomics on the hot path.

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

// Stores the quarter records of one 32-entry word of the batch: `cw` holds,
// per lane, the entries of the word the lane's pixel blended (or stopped
// at); OR over each
// row of 16 lanes (DPP partners l ^ 8, l ^ 7, l ^ 2, l ^ 1) gives the
// quarter's entries, and lane i writes the byte of entry i (bit q: quarter q
// blended it) for the n entries of the word, at qbits[p0 + i] (the wave's
// block's plane of the records).  All lanes take part.
__device__ __forceinline__ void record_word(uint8_t *__restrict__ qbits, uint32_t cw, uint32_t p0, int n,
                                            int lane)
{
    cw |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cw, 0x128, 0xF, 0xF, true);
    cw |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cw, 0x141, 0xF, 0xF, true);
    cw |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cw, 0x4E, 0xF, 0xF, true);
    cw |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)cw, 0xB1, 0xF, 0xF, true);
    const uint32_t r0 = __builtin_amdgcn_readlane(cw, 0), r1 = __builtin_amdgcn_readlane(cw, 16);
    const uint32_t r2 = __builtin_amdgcn_readlane(cw, 32), r3 = __builtin_amdgcn_readlane(cw, 48);
    if (lane < n) {
        const uint32_t b = ((r0 >> lane) & 1u) | (((r1 >> lane) & 1u) << 1) | (((r2 >> lane) & 1u) << 2) |
                           (((r3 >> lane) & 1u) << 3);
        qbits[p0 + (uint32_t)lane] = (uint8_t)b;
    }
}

template <int TW, int TH, int BATCH>
__device__ __forceinline__ void blend_tile(const DevView *__restrict__ views, int nv,
                                           const uint32_t *__restrict__ tile_order,
                                           const uint2 *__restrict__ ranges, const uint32_t *__restrict__ pair_vals,
                                           const SplatRec *__restrict__ recs, const double4 *__restrict__ axes,
                                           float *__restrict__ T_final, uint32_t *__restrict__ n_last,
                                           uint32_t *__restrict__ n_blend, uint8_t *__restrict__ qbits,
                                           uint32_t qstride, uint4 *__restrict__ wstats, uint32_t slot)
{
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int SX = TW / 8;
    constexpr int NB = (TW / 8) * (TH / 8);
    constexpr int PER = BATCH / NT;  // records staged per thread and batch
    static_assert(BATCH % NT == 0 && BATCH % 64 == 0 && NB <= 8, "tile/batch combination");
    __shared__ float4 s_w[BATCH], s_o[BATCH], s_c[BATCH];
    __shared__ float2 s_u[NB][BATCH];
    __shared__ uint32_t s_qm[NB][4][BATCH / 32];  // bit b of word k: quarter q of block bk may take entry 32 k + b
    const uint32_t tile = tile_order[slot];  // longest lists first
    const int vi = view_of_tile(views, nv, tile);
    const DevView &V = views[vi];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4;
    const int ox = tx * TW, oy = ty * TH;
    const int bx = quarter_x(lane), by = quarter_y(lane);
    const int px = ox + (w % SX) * 8 + bx, py = oy + (w / SX) * 8 + by;
    const bool inside = px < V.W && py < V.H;
    const float lx = (float)bx, ly = (float)by;
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
            } else {  // padding: alpha = 0 everywhere, taken by no quarter
                st.w = st.o = st.c = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) st.u[bk] = make_float2(0.0f, 0.0f);
                st.live = 0u;
            }
            s_w[j] = st.w;
            s_o[j] = st.o;
            s_c[j] = st.c;
#pragma unroll
            for (int bk = 0; bk < NB; ++bk) s_u[bk][j] = st.u[bk];
            const int e0 = p * NT + 64 * w;  // first entry of this wave's 64
#pragma unroll
            for (int bq = 0; bq < 4 * NB; ++bq) {
                const uint64_t m = __ballot((st.live >> bq) & 1u);
                if (lane == 0) {
                    s_qm[bq >> 2][bq & 3][e0 >> 5] = (uint32_t)m;
                    s_qm[bq >> 2][bq & 3][(e0 >> 5) + 1] = (uint32_t)(m >> 32);
                }
            }
        }
        __syncthreads();
        if (b0 + BATCH < rg.y) fetch(b0 + BATCH);
        uint64_t alive = __ballot(T > 0.0f);
        if (alive == 0ull) continue;
        const int cnt = (int)min((uint32_t)BATCH, rg.y - b0);
        const uint32_t jb = b0 - rg.x + 1u;  // 1-based list position of entry 0
        // each quarter walks, front to back, the entries it may take, until
        // its pixels are all finished; the four quarters of a wave step together
        for (int k = 0; 32 * k < cnt; ++k) {
            uint32_t m = s_qm[w][q][k];
            uint32_t cw = 0u;  // entries of this word the lane's pixel blended (or stopped at)
            for (;;) {
                m = ((alive >> (lane & 48)) & 0xFFFFull) ? m : 0u;  // nothing left for a finished quarter
                const uint64_t hm = __ballot(m != 0u);
                if (hm == 0ull) break;
                const bool has = m != 0u;
                const int j = 32 * k + __builtin_ctz(m | 0x80000000u);  // entry 32 k + 31 when nothing is left
                m &= m - 1u;
                const bool go = has && T > 0.0f;
                const float4 Ov = s_o[j];
                const bool interp = Ov.z > 0.0f;
                // work counts from the wave's masks (scalar unit only)
                const uint64_t gm = hm & alive;
                n_eval += (uint32_t)__popcll(gm);
                n_eval_t += (uint32_t)__popcll(gm & __ballot(Ov.z > 0.0f));
                AlphaEval e;
                eval_alpha(s_w[j], Ov, s_u[w][j], lx, ly, interp, e);
                if (go && e.alpha >= kAlphaMin) {
                    const float Tn = T * (1.0f - e.alpha);
                    const bool stop = Tn < kTMin;
                    const float4 Cc = s_c[j];
                    const float wgt = stop ? 0.0f : e.alpha * T;
                    C0 += Cc.x * wgt;
                    C1 += Cc.y * wgt;
                    C2 += Cc.z * wgt;
                    nb += stop ? 0u : 1u;
                    last = stop ? last : jb + (uint32_t)j;
                    cw |= 1u << (j & 31);  // the splat a pixel stops at too: the backward's range test drops it
                    T = stop ? -T : Tn;
                }
                alive = __ballot(T > 0.0f);
            }
            // the backward takes, per quarter, only the entries it blended here
            // (entries after the last word walked lie after every pixel's last
            // contributor, where the backward never looks)
            record_word(qbits + (size_t)w * qstride, cw, b0 + 32u * (uint32_t)k, min(32, cnt - 32 * k), lane);
            if (alive == 0ull) break;
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
                                                  uint8_t *__restrict__ qbits, uint32_t qstride,
                                                  uint4 *__restrict__ wstats, uint32_t n_tiles,
                                                  uint32_t *__restrict__ queue, uint32_t chunk)
{
    if constexpr (!PERSIST) {
        blend_tile<TW, TH, BATCH>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final, n_last, n_blend,
                                  qbits, qstride, wstats, blockIdx.x);
    } else {
        __shared__ uint32_t s_slot;
        for (;;) {
            const uint32_t first = next_run(queue, chunk, &s_slot);
            if (first >= n_tiles) break;
            const uint32_t last = min(n_tiles, first + chunk);
            for (uint32_t slot = first; slot < last; ++slot) {
                blend_tile<TW, TH, BATCH>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final, n_last,
                                          n_blend, qbits, qstride, wstats, slot);
                __syncthreads();  // LDS of this tile read by every wave before the next stages
            }
        }
    }
}

// Sum over each row of 16 lanes (one 4x4 quarter of the wave's block) of 12
// per-lane values, taken as six pairs (first, second): four halvings with
// DPP inside the row (partners l ^ 8, l ^ 7, l ^ 2 and l ^ 1), each keeping
// one of the two values of a pair per lane.  The caller gives the first
// halving's operands, chosen per lane by bit 3 of the lane: S1[k] = second
// if set, else first; S2[k] = the other one.  Lane l of the row ends with the
// row's total of value row_slot(l) (value 2 k + 1 is the second of pair k;
// -1: a copy of another lane's total).
__device__ __forceinline__ float row_reduce12(const float (&S1)[6], const float (&S2)[6], int lane)
{
    const bool b2 = (lane & 4) != 0, b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
    float A[6], B[3];
#pragma unroll
    for (int k = 0; k < 6; ++k) A[k] = S1[k] + dpp_move<0x128>(S2[k]);  // row_ror:8
#pragma unroll
    for (int m = 0; m < 3; ++m)
        B[m] = (b2 ? A[2 * m + 1] : A[2 * m]) + dpp_move<0x141>(b2 ? A[2 * m] : A[2 * m + 1]);  // half mirror
    const float C0 = (b1 ? B[1] : B[0]) + dpp_move<0x4E>(b1 ? B[0] : B[1]);
    const float C1 = B[2] + dpp_move<0x4E>(B[2]);
    return (b0 ? C1 : C0) + dpp_move<0xB1>(b0 ? C0 : C1);
}

__device__ __forceinline__ int row_slot(int lane)
{
    const int b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1, b1 = (lane >> 1) & 1, b0 = lane & 1;
    return b0 == 0 ? 4 * b1 + 2 * b2 + b3 : (b1 == 0 ? 8 + 2 * b2 + b3 : -1);
}

constexpr int kG = 12;  // floats per splat in the screen-space gradient

// Per-lane gradient slots of one (pixel, splat) pair, summed over the tile:
//   0, 1    P'_i = h v_i                  with h = G dL/dG (G the Gaussian)
//   2, 3    Q'_11, Q'_22 = h v_1 v_1, h v_2 v_2
//   4       Q'_12 = h v_1 v_2
//   5       S = h
//   6, 7    dL/dA_n, dL/dA_p (A = kappa |o|)
//   8..10   dL/d colour
//   11      dL/dt through alpha (only when the caller asks for dL/dt)
// Here v = u - c is the pixel's position on the conic's scaled eigen-axes
// relative to the tile's centre (c, formed in FP64 at staging): v is the
// pixel's offset from the tile centre mapped by the axes.  The moments
// about the splat's centre follow in FP64 at the flush, P = P' + c S and
// Q = Q' + c P'^T + P' c^T + c c^T S.  Taken directly about the splat's
// centre, the moments of a large splat whose centre lies far off screen are
// dominated by c S and c c^T S, and the mean and covariance gradients built
// from them cancel almost entirely in the chain through the projection:
// separately rounded FP32 sums of P and Q then leave errors far above the
// result.  With the moments about the tile both large parts carry the one
// rounded S, and the cancellation removes its error with it.  What remains
// is the FP32 rounding of P' and Q', which grows with |v|^2: hence the
// tile's centre (|v| at most half the tile's diagonal) rather than a
// corner, and S summed from the same per-pixel h as P' and Q' (forming it
// from slots 5 and 6 instead, equal in exact arithmetic, leaves per-pixel
// differences that c c^T amplifies).
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

// Offsets of the centre of the TW x TH tile at (ox, oy) on the scaled
// eigen-axes, in FP64.
template <int TW, int TH>
__device__ __forceinline__ double2 centre_offsets(const SplatRec &r, const double4 &W, int ox, int oy)
{
#pragma clang fp contract(off)
    const double dx = ((double)(ox - r.ax) + 0.5 * TW) - (double)r.fx;
    const double dy = ((double)(oy - r.ay) + 0.5 * TH) - (double)r.fy;
    return make_double2(dx * W.x + dy * W.y, dx * W.z + dy * W.w);
}

// DET (the deterministic mode): no floating-point atomics.  Each row of 16
// lanes stores its FP32 partial sums in a slot of its own, the flush adds the
// rows in a fixed order (FP64), and the tile's 11 terms for a splat go with
// plain stores to det.part at the pair's position in the list k_duplicate
// emitted (the splat's first pair plus the tile's row-major index in its
// tile rectangle); launch_det_sum then adds each splat's rows in order.
template <int TW, int TH, int BATCH, bool DT, bool DET>
__device__ __forceinline__ void blend_bwd_tile(const DevView *__restrict__ views, int nv,
                                               const uint32_t *__restrict__ tile_order,
                                               const uint2 *__restrict__ ranges,
                                               const uint32_t *__restrict__ pair_vals,
                                               const SplatRec *__restrict__ recs, const double4 *__restrict__ axes,
                                               const float *__restrict__ T_final,
                                               const uint32_t *__restrict__ n_last,
                                               const uint8_t *__restrict__ qbits, uint32_t qstride,
                                               const uint32_t *__restrict__ vis_rank, double *__restrict__ sgrad,
                                               const DetArgs det, uint4 *__restrict__ wstats, uint32_t tslot)
{
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int SX = TW / 8;
    constexpr int NB = (TW / 8) * (TH / 8);
    constexpr int NQW = BATCH / 32;  // 32-entry words of a quarter's mask
    static_assert(BATCH % 32 == 0 && BATCH <= 32 * NW && NB <= 8, "tile/batch combination");
    __shared__ float4 s_w[BATCH], s_o[BATCH], s_c[BATCH];
    __shared__ float2 s_u[NB][BATCH];  // c1, c2
    __shared__ uint32_t s_id[BATCH];
    __shared__ __align__(16) double s_g[DET ? 1 : BATCH][kG];  // the quarters' partial sums, added in FP64
    __shared__ double s_d[DET ? 1 : BATCH * 11];  // the flushed terms, splat-major
    __shared__ float s_gr[DET ? 4 * NW : 1][DET ? BATCH : 1][kG];  // DET: each row's partial sums
    __shared__ uint32_t s_pq[DET ? BATCH : 1];  // DET: the pair's position in the emitted list
    __shared__ double2 s_ref[BATCH];    // the tile centre's offsets on the axes (FP64)
    // bit b of word k: quarter q of block bk may take entry 32 k + 31 - b
    // (reversed, so that the lowest set bit is the next entry back to front)
    __shared__ uint32_t s_qm[NB][4][NQW];
    __shared__ uint32_t s_max;
    const uint32_t tile = tile_order[tslot];  // longest lists first
    const int vi = view_of_tile(views, nv, tile);
    const DevView &V = views[vi];
    const uint32_t lt = tile - V.tile_base;
    const int tx = (int)(lt % (uint32_t)V.tiles_x), ty = (int)(lt / (uint32_t)V.tiles_x);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, q = lane >> 4;
    const int ox = tx * TW, oy = ty * TH;
    const int bx = quarter_x(lane), by = quarter_y(lane);
    const int px = ox + (w % SX) * 8 + bx, py = oy + (w / SX) * 8 + by;
    const bool inside = px < V.W && py < V.H;
    const float lx = (float)bx, ly = (float)by;
    // the pixel's offset from the tile centre (the moments' reference; exact)
    const float lxt = (float)(px - ox) - 0.5f * (TW - 1), lyt = (float)(py - oy) - 0.5f * (TH - 1);
    const uint2 rg = ranges[tile];
    const int slot = row_slot(lane);
    const bool b3 = (lane & 8) != 0;  // which value of each pair this lane keeps in the first halving

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
    // the colour cotangents as the first halving takes them (pairs (0, 1), (2, -))
    const float ga = b3 ? g1 : g0, gb = b3 ? g0 : g1, g2a = b3 ? 0.0f : g2, g2b = b3 ? g2 : 0.0f;
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    // the quarter's last contributor (rows of 16 lanes), then the tile's
    uint32_t qm = last;
#pragma unroll
    for (int d = 8; d >= 1; d >>= 1) qm = max(qm, (uint32_t)__shfl_xor((int)qm, d, 64));
    uint32_t wm = max(qm, (uint32_t)__shfl_xor((int)qm, 16, 64));
    wm = max(wm, (uint32_t)__shfl_xor((int)wm, 32, 64));
    if (lane == 0) atomicMax(&s_max, wm);
    __syncthreads();
    const uint32_t end = rg.x + s_max;
    float R0 = 0.0f, R1 = 0.0f, R2 = 0.0f;  // colour composited behind the current splat
    uint32_t n_eval = 0, n_eval_t = 0, n_con = 0;  // wave totals (scalar)

    for (uint32_t hi = end; hi > rg.x;) {
        const uint32_t lo = hi - rg.x > (uint32_t)BATCH ? hi - BATCH : rg.x;
        const int cnt = (int)(hi - lo);
        {
            // wave w stages entries 32 w .. 32 w + 31 on its lanes 0-31 (the
            // batch holds at most 32 entries per wave), so that the staging
            // work is spread over the waves of the tile
            const int j = 32 * w + lane;
            uint32_t live = 0u;
            if (lane < 32 && j < cnt) {
                const uint32_t sidx = pair_vals[lo + j];
                const SplatRec r = recs[sidx];
                const double4 W64 = axes[sidx];
                const float4 W = make_float4((float)W64.x, (float)W64.y, (float)W64.z, (float)W64.w);
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) {
                    float c1, c2, d0, d1;
                    block_offsets(r, W64, ox + (bk % SX) * 8, oy + (bk / SX) * 8, c1, c2, d0, d1);
                    s_u[bk][j] = make_float2(c1, c2);
                    // the quarters of this block that blended the splat in the forward
                    live |= (uint32_t)qbits[(size_t)bk * qstride + lo + (uint32_t)j] << (4 * bk);
                }
                s_id[j] = vis_rank[sidx];  // gradient row
                s_w[j] = W;
                s_o[j] = make_float4(r.An, r.Ap, r.t, r.invK);
                s_c[j] = make_float4(r.r, r.g, r.b, 0.0f);
                s_ref[j] = centre_offsets<TW, TH>(r, W64, ox, oy);
                if constexpr (DET) {
                    for (int row = 0; row < 4 * NW; ++row)
#pragma unroll
                        for (int k = 0; k < kG; ++k) s_gr[row][j][k] = 0.0f;
                    const uint32_t jr = det.jrank[sidx];
                    const uint2 rc = det.rect[jr];
                    const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu;
                    s_pq[j] = det.pair_offsets[jr] + ((uint32_t)ty - ty0) * (tx1 - tx0 + 1u) + ((uint32_t)tx - tx0);
                } else {
#pragma unroll
                    for (int k = 0; k < kG; ++k) s_g[j][k] = 0.0;
                }
            } else if (lane < 32 && j < BATCH) {  // padding read by quarters with nothing left: alpha = 0
                s_w[j] = s_o[j] = s_c[j] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) s_u[bk][j] = make_float2(0.0f, 0.0f);
            }
            if (32 * w < BATCH) {  // this wave's word of the quarter masks
#pragma unroll
                for (int bq = 0; bq < 4 * NB; ++bq) {
                    const uint64_t m = __ballot((live >> bq) & 1u);
                    if (lane == 0) s_qm[bq >> 2][bq & 3][w] = __builtin_bitreverse32((uint32_t)m);
                }
            }
        }
        __syncthreads();
        // each quarter walks, back to front, the entries some pixel of it blended
        // in the forward (those before its last contributor: later records are
        // not written); the four quarters of a wave step together
        const uint32_t base = lo - rg.x;  // list position of entry 0
        const int lim = qm > base ? (int)min(qm - base, (uint32_t)cnt) : 0;
        for (int k = (cnt - 1) >> 5; k >= 0; --k) {
            uint32_t m = s_qm[w][q][k];
            const int lk = lim - 32 * k;  // entries 32 k + i, i < lk, come before the last contributor
            m &= lk >= 32 ? ~0u : (lk <= 0 ? 0u : ~((1u << (32 - lk)) - 1u));
            for (;;) {
                // lane masks straight from the compares (no per-lane booleans
                // carried across the branches)
                const uint64_t hm = __ballot(m != 0u);
                if (hm == 0ull) break;
                const bool has = m != 0u;
                const int j = 32 * k + 31 - __builtin_ctz(m | 0x80000000u);  // entry 32 k when nothing is left
                m &= m - 1u;
                const uint64_t rm = __ballot(base + (uint32_t)j < last);
                const float4 Wv = s_w[j], Ov = s_o[j];
                const float2 U = s_u[w][j];
                const uint64_t tm = __ballot(Ov.z > 0.0f);
                const bool interp = Ov.z > 0.0f;
                AlphaEval e;
                eval_alpha(Wv, Ov, U, lx, ly, interp, e);
                const uint64_t irm = hm & rm;
                const uint64_t cm = irm & __ballot(e.alpha >= kAlphaMin);
                n_eval += (uint32_t)__popcll(irm);
                n_eval_t += (uint32_t)__popcll(irm & tm);
                if (cm == 0ull) continue;
                const bool contrib = has && base + (uint32_t)j < last && e.alpha >= kAlphaMin;
                n_con += (uint32_t)__popcll(cm);
                // every lane runs the update; a non-contributing lane has a = 0 and
                // dL/dalpha = 0, which leaves T and R as they are and all slots 0
                const float4 Cc = s_c[j];
                const float a = contrib ? e.alpha : 0.0f;
                T = T * __builtin_amdgcn_rcpf(1.0f - a);
                const float dal_raw = T * ((Cc.x - R0) * g0 + (Cc.y - R1) * g1 + (Cc.z - R2) * g2);
                const float dal = contrib ? dal_raw : 0.0f;
                const float aT = a * T;
                R0 = fmaf(a, Cc.x - R0, R0);
                R1 = fmaf(a, Cc.y - R1, R1);
                R2 = fmaf(a, Cc.z - R2, R2);
                float dan = dal, dap = 0.0f, dtv = 0.0f;
                if (interp) {
                    dan = (1.0f - Ov.z) * dal;
                    const float dapr = Ov.z * dal;
                    if constexpr (DT) dtv = (e.apr - e.an) * dal;
                    // d apr / d a_p = (1/K) (1 - a_p)^(1/K - 1) = (1/K) q / (1 - a_p)
                    dap = dapr * Ov.w * (e.q * __builtin_amdgcn_rcpf(1.0f - e.ap));
                }
                const float dan_c = e.cn ? 0.0f : dan, dap_c = e.cp ? 0.0f : dap;
                const float h = e.G * (dan_c * Ov.x + dap_c * Ov.y);  // G dL/dG
                const float v1 = fmaf(lyt, Wv.y, lxt * Wv.x), v2 = fmaf(lyt, Wv.w, lxt * Wv.z);
                // the six pairs of the slots, as the first halving takes them
                const float pa = b3 ? v2 : v1, pb = b3 ? v1 : v2;
                const float ha = h * pa, hb = h * pb, hab = ha * pb;
                float S1[6], S2[6];
                S1[0] = ha;                      // P'_1, P'_2
                S2[0] = hb;
                S1[1] = ha * pa;                 // Q'_11, Q'_22
                S2[1] = hb * pb;
                S1[2] = b3 ? h : hab;            // Q'_12, S
                S2[2] = b3 ? hab : h;
                S1[3] = e.G * (b3 ? dap_c : dan_c);  // dL/dA_n, dL/dA_p
                S2[3] = e.G * (b3 ? dan_c : dap_c);
                S1[4] = aT * ga;                 // colour 0, 1
                S2[4] = aT * gb;
                if constexpr (DT) {              // colour 2, dL/dt
                    const float c2 = aT * g2;
                    S1[5] = b3 ? dtv : c2;
                    S2[5] = b3 ? c2 : dtv;
                } else {
                    S1[5] = aT * g2a;
                    S2[5] = aT * g2b;
                }
                const float tot = row_reduce12(S1, S2, lane);
                if constexpr (DET) {
                    if (has && slot >= 0) s_gr[4 * w + q][j][slot] = tot;
                } else {
                    if (has && slot >= 0 && tot != 0.0f) unsafeAtomicAdd(&s_g[j][slot], (double)tot);
                }
            }
        }
        __syncthreads();
        // flush: one lane per splat turns the tile's partial sums into the
        // 11 screen-space terms (FP64); then the terms of all splats go out
        // as consecutive atomics, row by row
        if (const int j = 32 * w + lane; lane < 32 && j < cnt) {  // wave w: entries 32 w .. 32 w + 31
            double gd[kG];
            if constexpr (DET) {
#pragma unroll
                for (int k = 0; k < kG; ++k) gd[k] = 0.0;
                for (int row = 0; row < 4 * NW; ++row)  // rows in a fixed order
#pragma unroll
                    for (int k = 0; k < kG; ++k) gd[k] += (double)s_gr[row][j][k];
            } else {
#pragma unroll
                for (int k = 0; k < kG; ++k) gd[k] = s_g[j][k];
            }
            const double *g = gd;
            // moments about the splat's centre from those about the tile's
            const double2 cr = s_ref[j];
            const double S = g[5];
            const double P1 = g[0], P2 = g[1], Q11 = g[2], Q22 = g[3], Q12 = g[4];
            const double P[2] = {P1 + cr.x * S, P2 + cr.y * S};
            const double Q[3] = {Q11 + 2.0 * cr.x * P1 + cr.x * cr.x * S,
                                 Q12 + cr.x * P2 + cr.y * P1 + cr.x * cr.y * S,
                                 Q22 + 2.0 * cr.y * P2 + cr.y * cr.y * S};
            double sc[5];
            screen_grad(s_w[j], P, Q, sc);
            double dd[11];
#pragma unroll
            for (int k = 0; k < 5; ++k) dd[k] = sc[k];
#pragma unroll
            for (int k = 5; k < 11; ++k) dd[k] = g[k + 1];
            if constexpr (DET) {
                double *o = det.part + (size_t)s_pq[j] * 11;
#pragma unroll
                for (int k = 0; k < 11; ++k) o[k] = dd[k];
            } else {
#pragma unroll
                for (int k = 0; k < 11; ++k) s_d[j * 11 + k] = dd[k];
            }
        }
        __syncthreads();
        if constexpr (!DET) {
            for (int idx = threadIdx.x; idx < cnt * 11; idx += NT) {
                const double val = s_d[idx];
                const int j = idx / 11, k = idx - 11 * j;
                if (val != 0.0) unsafeAtomicAdd(&sgrad[(size_t)s_id[j] * kG + k], val);
            }
            __syncthreads();
        }
        hi = lo;
    }
    if (lane == 0) wstats[(size_t)tslot * NW + w] = make_uint4(n_eval, n_eval_t, n_con, 0u);
}
template <int TW, int TH, int BATCH, bool DT, bool PERSIST, bool DET>
__global__ __launch_bounds__(TW *TH) void k_blend_bwd(const DevView *__restrict__ views, int nv,
                                                      const uint32_t *__restrict__ tile_order,
                                                      const uint2 *__restrict__ ranges,
                                                      const uint32_t *__restrict__ pair_vals,
                                                      const SplatRec *__restrict__ recs,
                                                      const double4 *__restrict__ axes,
                                                      const float *__restrict__ T_final,
                                                      const uint32_t *__restrict__ n_last,
                                                      const uint8_t *__restrict__ qbits, uint32_t qstride,
                                                      const uint32_t *__restrict__ vis_rank,
                                                      double *__restrict__ sgrad, const DetArgs det,
                                                      uint4 *__restrict__ wstats, uint32_t n_tiles,
                                                      uint32_t *__restrict__ queue, uint32_t chunk)
{
    if constexpr (!PERSIST) {
        blend_bwd_tile<TW, TH, BATCH, DT, DET>(views, nv, tile_order, ranges, pair_vals, recs, axes, T_final,
                                               n_last, qbits, qstride, vis_rank, sgrad, det, wstats, blockIdx.x);
    } else {
        __shared__ uint32_t s_slot;
        for (;;) {
            const uint32_t first = next_run(queue, chunk, &s_slot);
            if (first >= n_tiles) break;
            const uint32_t last = min(n_tiles, first + chunk);
            for (uint32_t slot = first; slot < last; ++slot) {
                blend_bwd_tile<TW, TH, BATCH, DT, DET>(views, nv, tile_order, ranges, pair_vals, recs, axes,
                                                       T_final, n_last, qbits, qstride, vis_rank, sgrad, det, wstats,
                                                       slot);
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
                    uint32_t *n_last, uint32_t *n_blend, uint8_t *qbits, uint32_t qstride, uint4 *wstats,
                    bool persist, uint32_t *queue, hipStream_t st)
{
    if (persist) {
        auto k = k_blend<TW, TH, BATCH, true>;
        const uint32_t g = std::min(n_tiles, resident_grid(k, TW * TH));
        launch_fill_u32(queue, 0u, 1, st);
        hipLaunchKernelGGL(k, dim3(g), dim3(TW * TH), 0, st, views, nv, order, ranges, pair_vals, recs, axes,
                           T_final, n_last, n_blend, qbits, qstride, wstats, n_tiles, queue, queue_run(n_tiles, g));
    } else {
        hipLaunchKernelGGL((k_blend<TW, TH, BATCH, false>), dim3(n_tiles), dim3(TW * TH), 0, st, views, nv, order,
                           ranges, pair_vals, recs, axes, T_final, n_last, n_blend, qbits, qstride, wstats, n_tiles,
                           queue, 1u);
    }
}

template <int TW, int TH, int B, bool DT>
void launch_blend_bwd_dt(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                         const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, const float *T_final,
                         const uint32_t *n_last, const uint8_t *qbits, uint32_t qstride, const uint32_t *vis_rank,
                         double *sgrad, const DetArgs *det, uint4 *wstats, bool persist, uint32_t *queue,
                         hipStream_t st)
{
    if (det) {  // the deterministic mode: one workgroup per tile, 32 splats staged per batch
        hipLaunchKernelGGL((k_blend_bwd<TW, TH, 32, DT, false, true>), dim3(n_tiles), dim3(TW * TH), 0, st, views, nv,
                           order, ranges, pair_vals, recs, axes, T_final, n_last, qbits, qstride, vis_rank, sgrad,
                           *det, wstats, n_tiles, queue, 1u);
    } else if (persist) {
        auto k = k_blend_bwd<TW, TH, B, DT, true, false>;
        const uint32_t g = std::min(n_tiles, resident_grid(k, TW * TH));
        launch_fill_u32(queue, 0u, 1, st);
        hipLaunchKernelGGL(k, dim3(g), dim3(TW * TH), 0, st, views, nv, order, ranges, pair_vals, recs, axes, T_final,
                           n_last, qbits, qstride, vis_rank, sgrad, DetArgs{}, wstats, n_tiles, queue,
                           queue_run(n_tiles, g));
    } else {
        hipLaunchKernelGGL((k_blend_bwd<TW, TH, B, DT, false, false>), dim3(n_tiles), dim3(TW * TH), 0, st, views, nv,
                           order, ranges, pair_vals, recs, axes, T_final, n_last, qbits, qstride, vis_rank, sgrad,
                           DetArgs{}, wstats, n_tiles, queue, 1u);
    }
}

template <int TW, int TH, int BATCH>
void launch_blend_bwd_t(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                        const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, const float *T_final,
                        const uint32_t *n_last, const uint8_t *qbits, uint32_t qstride, const uint32_t *vis_rank,
                        double *sgrad, const DetArgs *det, uint4 *wstats, bool want_dt, bool persist,
                        uint32_t *queue, hipStream_t st)
{
    // the backward stages at most 32 splats per wave and step: its LDS holds
    // the FP32 partial sums and the FP64 flushed terms of every staged
    // splat, and a smaller footprint keeps more tiles resident per CU
    constexpr int BMAX = 32 * (TW * TH / 64);
    constexpr int B = BATCH < BMAX ? BATCH : BMAX;
    if (want_dt)
        launch_blend_bwd_dt<TW, TH, B, true>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final,
                                             n_last, qbits, qstride, vis_rank, sgrad, det, wstats, persist, queue, st);
    else
        launch_blend_bwd_dt<TW, TH, B, false>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final,
                                              n_last, qbits, qstride, vis_rank, sgrad, det, wstats, persist, queue, st);
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
    (void)resident_grid(k_blend_bwd<TW, TH, B, true, true, false>, TW * TH);
    (void)resident_grid(k_blend_bwd<TW, TH, B, false, true, false>, TW * TH);
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
                             const double4 *axes, float *T_final, uint32_t *n_last, uint32_t *n_blend,
                             uint8_t *qbits, uint32_t qstride, uint4 *wstats, int tw, int th, int batch, bool persist,
                             uint32_t *queue, hipStream_t st)
{
#define X(a, b, c)                                                                                           \
    if (tw == a && th == b && batch == c)                                                                    \
        return launch_blend_t<a, b, c>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last, \
                                       n_blend, qbits, qstride, wstats, persist, queue, st);
    HGS_BLEND_CASES(X)
#undef X
}

void launch_blend(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order, const uint2 *ranges,
                  const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes, float *T_final,
                  uint32_t *n_last, uint32_t *n_blend, uint8_t *qbits, uint32_t qstride, uint4 *wstats,
                  Counters *ctr, int tw, int th, int batch, bool persist, uint32_t *queue, hipStream_t st)
{
    if (batch == 0) batch = tw * th;
    if (!n_tiles) return;
    const uint32_t nst = n_tiles * (uint32_t)(tw * th / 64);
    launch_blend_cfg(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last, n_blend, qbits,
                     qstride, wstats, tw, th, batch, persist, queue, st);
    hipLaunchKernelGGL(k_stats_reduce, dim3(256), dim3(256), 0, st, wstats, nst, &ctr->evaluated);
}

void launch_blend_backward(const DevView *views, int nv, uint32_t n_tiles, const uint32_t *order,
                           const uint2 *ranges, const uint32_t *pair_vals, const SplatRec *recs, const double4 *axes,
                           const float *T_final, const uint32_t *n_last, const uint8_t *qbits, uint32_t qstride,
                           const uint32_t *vis_rank, double *sgrad, const DetArgs *det, uint4 *wstats, Counters *ctr,
                           int tw, int th, int batch, bool want_dt, bool persist, uint32_t *queue, hipStream_t st)
{
    if (batch == 0) batch = tw * th;
    if (!n_tiles) return;
#define X(a, b, c)                                                                                                 \
    if (tw == a && th == b && batch == c) {                                                                        \
        launch_blend_bwd_t<a, b, c>(views, nv, n_tiles, order, ranges, pair_vals, recs, axes, T_final, n_last,    \
                                    qbits, qstride, vis_rank, sgrad, det, wstats, want_dt, persist, queue, st);    \
        hipLaunchKernelGGL(k_stats_reduce, dim3(256), dim3(256), 0, st, wstats,                                    \
                           n_tiles * (uint32_t)(tw * th / 64), &ctr->bwd_evaluated);                               \
        return;                                                                                                    \
    }
    HGS_BLEND_CASES(X)
#undef X
}

}  // namespace hgs
