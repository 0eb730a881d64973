// Hierarchy generation on the GPU (Sec. 4.1 "Hierarchy Generation", with the
// orientation matching of Sec. 4.2): the octree over the leaves' Morton
// cells, the bottom-up merge of Eq. (merge) with the weights o_i S_i, the SH
// merge with the same weights and the falloff sum(w') / S_p, the top-down
// orientation matching over the 24 proper axis re-assignments, and the
// nodes' boxes.
//
// The tree is built one level at a time over the leaves sorted by Morton
// code: every leaf position knows the node of the current level that holds
// it; a position starts a node of the next level when it starts its node, or
// when the code prefix of the next level changes there (the first level at
// which two neighbouring codes differ is computed once per position), or,
// for leaves that share one cell, at the group boundaries j m / k (k =
// min(8, m) groups of m leaves).  A scan of those starts numbers the new
// nodes in breadth-first order.  The merges then run level by level from
// the deepest up (one thread per node, FP64), and the matching level by
// level from the root down.
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;
constexpr int kMortonBits = 21;

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, (n + kT - 1) / kT); }

// ------------------------------------------------------------- grid, codes
// Per-block minimum and maximum of the leaf positions (node-major [n][3]).
__global__ __launch_bounds__(kT) void k_bounds(const float *__restrict__ pos, int64_t n, float *__restrict__ part)
{
    __shared__ float s[6][kT];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
        for (int k = 0; k < 3; ++k) {
            const float v = pos[3 * i + k];
            lo[k] = fminf(lo[k], v);
            hi[k] = fmaxf(hi[k], v);
        }
    for (int k = 0; k < 3; ++k) {
        s[k][threadIdx.x] = lo[k];
        s[3 + k][threadIdx.x] = hi[k];
    }
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = fminf(s[k][threadIdx.x], s[k][threadIdx.x + w]);
                s[3 + k][threadIdx.x] = fmaxf(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

// Spreads the low 21 bits of v so that bit b lands at bit 3 b.
__device__ __forceinline__ uint64_t spread3(uint64_t v)
{
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Morton code of every leaf on the grid lo + cell / s, split into its low
// and high 32 bits (the sort keys), and the identity permutation.
__global__ __launch_bounds__(kT) void k_morton(const float *__restrict__ pos, int64_t n, double lo0, double lo1,
                                               double lo2, double s, uint32_t *__restrict__ key_lo,
                                               uint32_t *__restrict__ key_hi, uint32_t *__restrict__ idx)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lo0, lo1, lo2};
    uint64_t c = 0;
    for (int k = 0; k < 3; ++k) {
        const double t = ((double)pos[3 * i + k] - lo[k]) * s;
        const uint64_t q = (uint64_t)floor(t + 0.5);
        c |= spread3(q) << k;
    }
    key_lo[i] = (uint32_t)c;
    key_hi[i] = (uint32_t)(c >> 32);
    idx[i] = (uint32_t)i;
}

__global__ __launch_bounds__(kT) void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx,
                                                   int64_t n, uint32_t *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// First tree level at which the codes of sorted positions i - 1 and i lie in
// different cells (1..21), 22 when they share the finest cell; 0 at i = 0.
__global__ __launch_bounds__(kT) void k_split_level(const uint32_t *__restrict__ lo, const uint32_t *__restrict__ hi,
                                                    int64_t n, uint8_t *__restrict__ sl)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    if (i == 0) {
        sl[0] = 0;
        return;
    }
    const uint64_t a = ((uint64_t)hi[i - 1] << 32) | lo[i - 1], b = ((uint64_t)hi[i] << 32) | lo[i];
    const uint64_t x = a ^ b;
    if (x == 0) {
        sl[i] = kMortonBits + 1;
        return;
    }
    const int top = 63 - __clzll((long long)x);  // highest differing bit
    sl[i] = (uint8_t)(kMortonBits - top / 3);
}

// ------------------------------------------------------------- topology
// Node arrays of the tree under construction (breadth-first ids).
struct Tree {
    int32_t *start, *size;          // first sorted leaf position and leaf count
    int32_t *parent, *child_begin, *child_count;
};

// Starts of the nodes of level d + 1 (flag = 1): positions held by a node of
// level d with two or more leaves where that node starts, where the cell of
// level d + 1 changes (d + 1 <= 21), or at a group boundary of leaves that
// share the finest cell (d + 1 > 21).
__global__ __launch_bounds__(kT) void k_level_starts(const int32_t *__restrict__ node_of, const uint8_t *__restrict__ sl,
                                                     Tree t, int64_t n, int next_level, uint32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int32_t p = node_of[i];
    uint32_t f = 0;
    if (p >= 0) {
        const int64_t a = t.start[p], m = t.size[p];
        if (m >= 2) {
            if (i == a) {
                f = 1;
            } else if (next_level <= kMortonBits) {
                f = sl[i] <= next_level ? 1u : 0u;
            } else {
                const int64_t k = m < 8 ? m : 8, r = i - a;
                const int64_t j = (r * k + m - 1) / m;  // smallest j with j m / k >= r
                f = (j < k && (j * m) / k == r) ? 1u : 0u;
            }
        }
    }
    flag[i] = f;
}

// The new level's nodes: id = base + rank; start, parent, the parent's first
// child; and every position's node of the new level (-1 once its leaf is
// done).  rank = exclusive scan of flag.
__global__ __launch_bounds__(kT) void k_level_nodes(const int32_t *__restrict__ node_of,
                                                    const uint32_t *__restrict__ flag,
                                                    const uint32_t *__restrict__ rank, Tree t, int64_t n,
                                                    int32_t base, int32_t *__restrict__ node_of_next)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int32_t p = node_of[i];
    if (p < 0 || t.size[p] < 2) {
        node_of_next[i] = -1;
        return;
    }
    // positions of a multi-leaf node: its first position is always a start,
    // so the inclusive count of starts names the new node
    const int32_t id = base + (int32_t)(rank[i] + flag[i]) - 1;
    node_of_next[i] = id;
    if (flag[i]) {
        t.start[id] = (int32_t)i;
        t.parent[id] = p;
        if (i == t.start[p]) t.child_begin[p] = id;
    }
}

// Sizes of the new level's nodes (they tile their parents in order) and the
// child count of every parent, written by its last child.
__global__ __launch_bounds__(kT) void k_level_sizes(Tree t, int32_t base, int32_t count, int64_t n,
                                                    const uint32_t *__restrict__ sorted_idx,
                                                    int32_t *__restrict__ leaf_src)
{
    const int32_t k = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (k >= count) return;
    const int32_t id = base + k;
    const int32_t p = t.parent[id];
    const int64_t pend = (int64_t)t.start[p] + t.size[p];
    const int64_t next = k + 1 < count ? (int64_t)t.start[id + 1] : n;
    const int64_t end = next < pend ? next : pend;
    t.size[id] = (int32_t)(end - t.start[id]);
    t.child_begin[id] = 0;
    t.child_count[id] = 0;
    leaf_src[id] = end - t.start[id] == 1 ? (int32_t)sorted_idx[t.start[id]] : -1;
    if (end == pend) t.child_count[p] = id - t.child_begin[p] + 1;
}

__global__ __launch_bounds__(kT) void k_interior_flags(const int32_t *__restrict__ child_count, int64_t N,
                                                       uint32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < N) flag[i] = child_count[i] > 0 ? 1u : 0u;
}

__global__ __launch_bounds__(kT) void k_interior_list(const int32_t *__restrict__ child_count,
                                                      const uint32_t *__restrict__ irank, int64_t N,
                                                      int32_t *__restrict__ interior)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < N && child_count[i] > 0) interior[irank[i]] = (int32_t)i;
}

__global__ __launch_bounds__(kT) void k_build_finish(const int32_t *__restrict__ parent,
                                                     const int32_t *__restrict__ child_count, int64_t N,
                                                     const float *__restrict__ bmin, const float *__restrict__ bmax,
                                                     uint32_t *__restrict__ pinfo, float *__restrict__ box)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N) return;
    pinfo[i] = (parent[i] < 0 ? kRootParent : (uint32_t)parent[i]) | (child_count[i] == 0 ? kLeafBit : 0u);
    for (int k = 0; k < 3; ++k) {
        box[k * N + i] = bmin[3 * i + k];
        box[(3 + k) * N + i] = bmax[3 * i + k];
    }
}

__global__ __launch_bounds__(kT) void k_unpack_nodes(const uint32_t *__restrict__ pinfo, const float *__restrict__ box,
                                                     int64_t N, int32_t *__restrict__ parent,
                                                     float *__restrict__ bmin, float *__restrict__ bmax)
{
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= N) return;
    const uint32_t p = pinfo[i] & ~kLeafBit;
    if (parent) parent[i] = p == kRootParent ? -1 : (int32_t)p;
    for (int k = 0; k < 3; ++k) {
        if (bmin) bmin[3 * i + k] = box[k * N + i];
        if (bmax) bmax[3 * i + k] = box[(3 + k) * N + i];
    }
}

// ------------------------------------------------------------- geometry
__device__ void rot_of_quat(const double q[4], double R[9])
{
#pragma clang fp contract(off)
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z;
    const double wx = w * x, wy = w * y, wz = w * z;
    R[0] = 1.0 - 2.0 * (yy + zz);
    R[1] = 2.0 * (xy - wz);
    R[2] = 2.0 * (xz + wy);
    R[3] = 2.0 * (xy + wz);
    R[4] = 1.0 - 2.0 * (xx + zz);
    R[5] = 2.0 * (yz - wx);
    R[6] = 2.0 * (xz - wy);
    R[7] = 2.0 * (yz + wx);
    R[8] = 1.0 - 2.0 * (xx + yy);
}

// Thomsen's approximation of an ellipsoid's surface from its semi-axes.
__device__ double ellipsoid_area(const double s[3])
{
#pragma clang fp contract(off)
    constexpr double p = 1.6075;
    const double a = pow(s[0], p), b = pow(s[1], p), c = pow(s[2], p);
    return 4.0 * 3.14159265358979323846 * pow((a * b + b * c + c * a) * (1.0 / 3.0), 1.0 / p);
}

// Symmetric 3x3 eigen-decomposition by Jacobi sweeps over the three
// off-diagonal entries (A given as xx, xy, xz, yy, yz, zz); columns of V
// are the eigenvectors of the eigenvalues ev.
__device__ void jacobi3(const double a6[6], double ev[3], double V[9])
{
#pragma clang fp contract(off)
    double A[3][3] = {{a6[0], a6[1], a6[2]}, {a6[1], a6[3], a6[4]}, {a6[2], a6[4], a6[5]}};
    double U[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        const double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off == 0.0 || off <= 1e-18 * scale) break;
        for (int r = 0; r < 3; ++r) {
            const int p = r == 2 ? 1 : 0, q = r == 0 ? 1 : 2;  // (0,1), (0,2), (1,2)
            if (A[p][q] == 0.0) continue;
            const double h = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
            const double t = copysign(1.0, h) / (fabs(h) + sqrt(1.0 + h * h));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            for (int k = 0; k < 3; ++k) {  // columns p, q
                const double x = A[k][p], y = A[k][q];
                A[k][p] = c * x - s * y;
                A[k][q] = s * x + c * y;
            }
            for (int k = 0; k < 3; ++k) {  // rows p, q
                const double x = A[p][k], y = A[q][k];
                A[p][k] = c * x - s * y;
                A[q][k] = s * x + c * y;
            }
            for (int k = 0; k < 3; ++k) {
                const double x = U[k][p], y = U[k][q];
                U[k][p] = c * x - s * y;
                U[k][q] = s * x + c * y;
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        ev[k] = A[k][k];
        for (int j = 0; j < 3; ++j) V[3 * k + j] = U[k][j];
    }
}

// Working values of the nodes (FP64): mean, covariance (xx xy xz yy yz zz),
// opacity or falloff, ellipsoid surface, unmatched axes (columns) and their
// scales; SH of interior nodes by interior rank.
struct Work {
    double *mean, *cov, *op, *surf, *axes, *sc;
    double *sh;        // [interior][48]
    int32_t *irank;    // interior rank of every interior node
    double *R, *q;     // matched rotation [9] and quaternion [4]
};

struct LeafIn {
    const float *pos, *scale, *rot, *opacity, *sh;  // node-major inputs
};

// Nodes of one level, bottom up: a leaf takes its input Gaussian; an
// interior node merges its children (Eq. merge, w'_i = o_i S_i).
__global__ __launch_bounds__(kT) void k_merge_level(Tree t, const int32_t *__restrict__ leaf_src, LeafIn in, Work w,
                                                    int32_t base, int32_t count)
{
#pragma clang fp contract(off)
    const int32_t k = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (k >= count) return;
    const int32_t id = base + k;
    const int32_t cc = t.child_count[id];
    if (cc == 0) {
        const int64_t i = leaf_src[id];
        double q[4], qn = 0.0;
        for (int j = 0; j < 4; ++j) {
            q[j] = (double)in.rot[4 * i + j];
            qn += q[j] * q[j];
        }
        qn = sqrt(qn);
        for (int j = 0; j < 4; ++j) q[j] /= qn;
        double R[9], s[3];
        rot_of_quat(q, R);
        for (int j = 0; j < 3; ++j) {
            s[j] = (double)in.scale[3 * i + j];
            w.mean[3 * (int64_t)id + j] = (double)in.pos[3 * i + j];
            w.sc[3 * (int64_t)id + j] = s[j];
        }
        const double s2[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
        double *C = w.cov + 6 * (int64_t)id;
        int e = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) {
                C[e++] = R[3 * a] * s2[0] * R[3 * b] + R[3 * a + 1] * s2[1] * R[3 * b + 1] +
                         R[3 * a + 2] * s2[2] * R[3 * b + 2];
            }
        for (int j = 0; j < 9; ++j) w.axes[9 * (int64_t)id + j] = R[j];
        w.op[id] = (double)in.opacity[i];
        w.surf[id] = ellipsoid_area(s);
        return;
    }
    const int32_t c0 = t.child_begin[id];
    double W = 0.0;
    for (int32_t c = c0; c < c0 + cc; ++c) W += w.op[c] * w.surf[c];
    double mu[3] = {0.0, 0.0, 0.0};
    for (int32_t c = c0; c < c0 + cc; ++c) {
        const double wc = w.op[c] * w.surf[c] / W;
        for (int j = 0; j < 3; ++j) mu[j] += wc * w.mean[3 * (int64_t)c + j];
    }
    double C[6] = {0, 0, 0, 0, 0, 0};
    double *sh = w.sh + 48 * (int64_t)w.irank[id];
    for (int j = 0; j < 48; ++j) sh[j] = 0.0;
    for (int32_t c = c0; c < c0 + cc; ++c) {
        const double wc = w.op[c] * w.surf[c] / W;
        double d[3];
        for (int j = 0; j < 3; ++j) d[j] = w.mean[3 * (int64_t)c + j] - mu[j];
        const double *Cc = w.cov + 6 * (int64_t)c;
        int e = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b, ++e) C[e] += wc * (Cc[e] + d[a] * d[b]);
        if (t.child_count[c] == 0) {
            const float *src = in.sh + 48 * (int64_t)leaf_src[c];
            for (int j = 0; j < 48; ++j) sh[j] += wc * (double)src[j];
        } else {
            const double *src = w.sh + 48 * (int64_t)w.irank[c];
            for (int j = 0; j < 48; ++j) sh[j] += wc * src[j];
        }
    }
    double ev[3], V[9], s[3];
    jacobi3(C, ev, V);
    for (int j = 0; j < 3; ++j) s[j] = sqrt(fmax(ev[j], 1e-20));
    for (int j = 0; j < 3; ++j) {
        w.mean[3 * (int64_t)id + j] = mu[j];
        w.sc[3 * (int64_t)id + j] = s[j];
    }
    for (int j = 0; j < 6; ++j) w.cov[6 * (int64_t)id + j] = C[j];
    for (int j = 0; j < 9; ++j) w.axes[9 * (int64_t)id + j] = V[j];
    const double S = ellipsoid_area(s);
    w.surf[id] = S;
    w.op[id] = W / S;
}

// The 24 proper signed axis re-assignments in a fixed order (axis
// permutations in lexicographic order, then sign patterns + + +, + + -, ...,
// keeping those of determinant +1): new axis j = sign_j * old axis perm_j.
struct AxisMaps {
    int8_t perm[24][3], sign[24][3];
};

__constant__ AxisMaps c_maps;

// Matching of one level, top down: each node's axes re-assigned to be
// closest to its parent's (the world axes at the root), scales following,
// the quaternion taken with a non-negative dot product with the parent's
// (w >= 0 at the root); FP32 outputs, and a leaf's box from them.
__global__ __launch_bounds__(kT) void k_match_level(Tree t, Work w, int32_t base, int32_t count,
                                                    float *__restrict__ out_mean, float *__restrict__ out_scale,
                                                    float *__restrict__ out_rot, float *__restrict__ out_op,
                                                    float *__restrict__ out_sh, const int32_t *__restrict__ leaf_src,
                                                    const float *__restrict__ in_sh, float *__restrict__ bmin,
                                                    float *__restrict__ bmax)
{
#pragma clang fp contract(off)
    const int32_t k = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (k >= count) return;
    const int32_t id = base + k;
    const int32_t p = t.parent[id];
    double Rp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (p >= 0)
        for (int j = 0; j < 9; ++j) Rp[j] = w.R[9 * (int64_t)p + j];
    double V[9];
    for (int j = 0; j < 9; ++j) V[j] = w.axes[9 * (int64_t)id + j];
    const double det = V[0] * (V[4] * V[8] - V[5] * V[7]) - V[1] * (V[3] * V[8] - V[5] * V[6]) +
                       V[2] * (V[3] * V[7] - V[4] * V[6]);
    if (det < 0.0)
        for (int r = 0; r < 3; ++r) V[3 * r + 2] = -V[3 * r + 2];
    // D[a][b] = column a of Rp . column b of V
    double D[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) D[a][b] = Rp[a] * V[b] + Rp[3 + a] * V[3 + b] + Rp[6 + a] * V[6 + b];
    int best = 0;
    double bt = -1e300;
    for (int m = 0; m < 24; ++m) {
        const double tr = c_maps.sign[m][0] * D[0][c_maps.perm[m][0]] + c_maps.sign[m][1] * D[1][c_maps.perm[m][1]] +
                          c_maps.sign[m][2] * D[2][c_maps.perm[m][2]];
        if (tr > bt) {
            bt = tr;
            best = m;
        }
    }
    double R[9], s[3];
    for (int j = 0; j < 3; ++j) {
        const int o = c_maps.perm[best][j];
        const double sg = c_maps.sign[best][j];
        for (int r = 0; r < 3; ++r) R[3 * r + j] = sg * V[3 * r + o];
        s[j] = w.sc[3 * (int64_t)id + o];
    }
    // quaternion from the largest of 1 + trace and the diagonal terms
    const double tr = R[0] + R[4] + R[8];
    const double cand[4] = {1.0 + tr, 1.0 + R[0] - R[4] - R[8], 1.0 - R[0] + R[4] - R[8], 1.0 - R[0] - R[4] + R[8]};
    int big = 0;
    for (int j = 1; j < 4; ++j)
        if (cand[j] > cand[big]) big = j;
    const double f = 0.5 * sqrt(cand[big]), g = 0.25 / f;
    double q[4];
    if (big == 0) {
        q[0] = f; q[1] = (R[7] - R[5]) * g; q[2] = (R[2] - R[6]) * g; q[3] = (R[3] - R[1]) * g;
    } else if (big == 1) {
        q[1] = f; q[0] = (R[7] - R[5]) * g; q[2] = (R[1] + R[3]) * g; q[3] = (R[2] + R[6]) * g;
    } else if (big == 2) {
        q[2] = f; q[0] = (R[2] - R[6]) * g; q[1] = (R[1] + R[3]) * g; q[3] = (R[5] + R[7]) * g;
    } else {
        q[3] = f; q[0] = (R[3] - R[1]) * g; q[1] = (R[2] + R[6]) * g; q[2] = (R[5] + R[7]) * g;
    }
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int j = 0; j < 4; ++j) q[j] /= qn;
    double dot = q[0];
    if (p >= 0) {
        dot = 0.0;
        for (int j = 0; j < 4; ++j) dot += q[j] * w.q[4 * (int64_t)p + j];
    }
    if (dot < 0.0)
        for (int j = 0; j < 4; ++j) q[j] = -q[j];
    for (int j = 0; j < 9; ++j) w.R[9 * (int64_t)id + j] = R[j];
    for (int j = 0; j < 4; ++j) {
        w.q[4 * (int64_t)id + j] = q[j];
        out_rot[4 * (int64_t)id + j] = (float)q[j];
    }
    for (int j = 0; j < 3; ++j) {
        out_scale[3 * (int64_t)id + j] = (float)s[j];
        out_mean[3 * (int64_t)id + j] = (float)w.mean[3 * (int64_t)id + j];
    }
    out_op[id] = (float)w.op[id];
    if (t.child_count[id] > 0) {
        const double *src = w.sh + 48 * (int64_t)w.irank[id];
        for (int j = 0; j < 48; ++j) out_sh[48 * (int64_t)id + j] = (float)src[j];
        return;
    }
    const float *src = in_sh + 48 * (int64_t)leaf_src[id];
    for (int j = 0; j < 48; ++j) out_sh[48 * (int64_t)id + j] = src[j];
    // the leaf's box from its stored (FP32) scale and normalised quaternion,
    // rounded outward to FP32
    double q32[4], n2 = 0.0, s32[3], R32[9];
    for (int j = 0; j < 4; ++j) {
        q32[j] = (double)out_rot[4 * (int64_t)id + j];
        n2 += q32[j] * q32[j];
    }
    n2 = sqrt(n2);
    for (int j = 0; j < 4; ++j) q32[j] /= n2;
    for (int j = 0; j < 3; ++j) s32[j] = (double)out_scale[3 * (int64_t)id + j];
    rot_of_quat(q32, R32);
    for (int a = 0; a < 3; ++a) {
        const double e = 3.0 * sqrt(R32[3 * a] * R32[3 * a] * s32[0] * s32[0] +
                                    R32[3 * a + 1] * R32[3 * a + 1] * s32[1] * s32[1] +
                                    R32[3 * a + 2] * R32[3 * a + 2] * s32[2] * s32[2]);
        const double m = (double)out_mean[3 * (int64_t)id + a];
        bmin[3 * (int64_t)id + a] = __double2float_rd(m - e);
        bmax[3 * (int64_t)id + a] = __double2float_ru(m + e);
    }
}

// Interior boxes of one level (bottom up): the union of the children's.
__global__ __launch_bounds__(kT) void k_box_level(Tree t, int32_t base, int32_t count, float *__restrict__ bmin,
                                                  float *__restrict__ bmax)
{
    const int32_t k = (int32_t)(blockIdx.x * kT + threadIdx.x);
    if (k >= count) return;
    const int32_t id = base + k;
    const int32_t cc = t.child_count[id];
    if (cc == 0) return;
    const int32_t c0 = t.child_begin[id];
    for (int a = 0; a < 3; ++a) {
        float lo = bmin[3 * (int64_t)c0 + a], hi = bmax[3 * (int64_t)c0 + a];
        for (int32_t c = c0 + 1; c < c0 + cc; ++c) {
            lo = fminf(lo, bmin[3 * (int64_t)c + a]);
            hi = fmaxf(hi, bmax[3 * (int64_t)c + a]);
        }
        bmin[3 * (int64_t)id + a] = lo;
        bmax[3 * (int64_t)id + a] = hi;
    }
}

__global__ __launch_bounds__(kT) void k_fill_i32(int32_t *__restrict__ p, int32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) p[i] = v;
}

}  // namespace

// ------------------------------------------------------------------ host
void build_axis_maps_upload(hipStream_t st)
{
    AxisMaps m{};
    static const int P6[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int parity[6] = {1, -1, -1, 1, 1, -1};  // sign of each permutation
    int c = 0;
    for (int p = 0; p < 6; ++p)
        for (int sb = 0; sb < 8; ++sb) {
            int sg[3], prod = 1;
            for (int j = 0; j < 3; ++j) {
                sg[j] = ((sb >> (2 - j)) & 1) ? -1 : 1;
                prod *= sg[j];
            }
            if (prod * parity[p] > 0) {  // determinant +1
                for (int j = 0; j < 3; ++j) {
                    m.perm[c][j] = (int8_t)P6[p][j];
                    m.sign[c][j] = (int8_t)sg[j];
                }
                ++c;
            }
        }
    (void)st;
    (void)hipMemcpyToSymbol(HIP_SYMBOL(c_maps), &m, sizeof m, 0, hipMemcpyHostToDevice);
}

void launch_build_bounds(const float *pos, int64_t n, float *part, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_bounds, dim3(nblocks), dim3(kT), 0, st, pos, n, part);
}

void launch_build_morton(const float *pos, int64_t n, const double lo[3], double s, uint32_t *key_lo,
                         uint32_t *key_hi, uint32_t *idx, hipStream_t st)
{
    hipLaunchKernelGGL(k_morton, dim3(blocks_for(n)), dim3(kT), 0, st, pos, n, lo[0], lo[1], lo[2], s, key_lo, key_hi,
                       idx);
}

void launch_gather_u32(const uint32_t *src, const uint32_t *idx, int64_t n, uint32_t *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather_u32, dim3(blocks_for(n)), dim3(kT), 0, st, src, idx, n, dst);
}

void launch_split_level(const uint32_t *lo, const uint32_t *hi, int64_t n, uint8_t *sl, hipStream_t st)
{
    hipLaunchKernelGGL(k_split_level, dim3(blocks_for(n)), dim3(kT), 0, st, lo, hi, n, sl);
}

void launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_i32, dim3(std::min<uint32_t>(blocks_for(n), 8192)), dim3(kT), 0, st, p, v, n);
}

void launch_level_starts(const int32_t *node_of, const uint8_t *sl, const BuildTree &t, int64_t n, int next_level,
                         uint32_t *flag, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    hipLaunchKernelGGL(k_level_starts, dim3(blocks_for(n)), dim3(kT), 0, st, node_of, sl, tt, n, next_level, flag);
}

void launch_level_nodes(const int32_t *node_of, const uint32_t *flag, const uint32_t *rank, const BuildTree &t,
                        int64_t n, int32_t base, int32_t *node_of_next, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    hipLaunchKernelGGL(k_level_nodes, dim3(blocks_for(n)), dim3(kT), 0, st, node_of, flag, rank, tt, n, base,
                       node_of_next);
}

void launch_level_sizes(const BuildTree &t, int32_t base, int32_t count, int64_t n, const uint32_t *sorted_idx,
                        int32_t *leaf_src, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    hipLaunchKernelGGL(k_level_sizes, dim3(blocks_for((uint64_t)count)), dim3(kT), 0, st, tt, base, count, n,
                       sorted_idx, leaf_src);
}

void launch_interior_ranks(const int32_t *child_count, int64_t N, uint32_t *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_interior_flags, dim3(blocks_for(N)), dim3(kT), 0, st, child_count, N, flag);
}

void launch_interior_list(const int32_t *child_count, const uint32_t *irank, int64_t N, int32_t *interior,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_interior_list, dim3(blocks_for(N)), dim3(kT), 0, st, child_count, irank, N, interior);
}

void launch_build_finish(const BuildTree &t, int64_t N, const float *bmin, const float *bmax, uint32_t *pinfo,
                         float *box, hipStream_t st)
{
    hipLaunchKernelGGL(k_build_finish, dim3(blocks_for(N)), dim3(kT), 0, st, t.parent, t.child_count, N, bmin, bmax,
                       pinfo, box);
}

void launch_unpack_nodes(const uint32_t *pinfo, const float *box, int64_t N, int32_t *parent, float *bmin,
                         float *bmax, hipStream_t st)
{
    hipLaunchKernelGGL(k_unpack_nodes, dim3(blocks_for(N)), dim3(kT), 0, st, pinfo, box, N, parent, bmin, bmax);
}

void launch_merge_level(const BuildTree &t, const int32_t *leaf_src, const BuildLeaves &in, const BuildWork &w,
                        int32_t base, int32_t count, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    const LeafIn li{in.pos, in.scale, in.rot, in.opacity, in.sh};
    const Work ww{w.mean, w.cov, w.op, w.surf, w.axes, w.sc, w.sh, w.irank, w.R, w.q};
    hipLaunchKernelGGL(k_merge_level, dim3(blocks_for((uint64_t)count)), dim3(kT), 0, st, tt, leaf_src, li, ww, base,
                       count);
}

void launch_match_level(const BuildTree &t, const BuildWork &w, int32_t base, int32_t count, const BuildOut &o,
                        const int32_t *leaf_src, const float *in_sh, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    const Work ww{w.mean, w.cov, w.op, w.surf, w.axes, w.sc, w.sh, w.irank, w.R, w.q};
    hipLaunchKernelGGL(k_match_level, dim3(blocks_for((uint64_t)count)), dim3(kT), 0, st, tt, ww, base, count, o.mean,
                       o.scale, o.rot, o.opacity, o.sh, leaf_src, in_sh, o.bmin, o.bmax);
}

void launch_box_level(const BuildTree &t, int32_t base, int32_t count, float *bmin, float *bmax, hipStream_t st)
{
    const Tree tt{t.start, t.size, t.parent, t.child_begin, t.child_count};
    hipLaunchKernelGGL(k_box_level, dim3(blocks_for((uint64_t)count)), dim3(kT), 0, st, tt, base, count, bmin, bmax);
}

}  // namespace hgs
