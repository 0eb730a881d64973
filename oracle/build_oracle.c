/*
 * FP64 CPU oracle of the hierarchy generation of "A Hierarchical 3D Gaussian
 * Representation for Real-Time Rendering of Very Large Datasets" (Kerbl et
 * al., ACM TOG 43(4), 2024), Sec. 4.1 "Hierarchy Generation" and the
 * orientation matching of Sec. 4.2 (the paragraph before Fig. simple-hier).
 *
 * TEST INFRASTRUCTURE ONLY.  The plain definition the GPU hierarchy builder
 * is checked against; it shares no code with the HIP path and is called only
 * by the tests.  Everything is computed in double precision from the FP32
 * leaf values the caller stores (the Python wrapper widens them).
 *
 * Definition (the tree follows the workloads' octree rule; the merge, the
 * weights, the SH merge, the falloff and the matching follow the paper):
 *   grid      lo = per-axis minimum of the leaf means, e = the largest
 *             extent (1 if zero), s = (2^21 - 1) / e; a leaf's cell
 *             coordinate on axis k is floor((x_k - lo_k) s + 1/2); its
 *             Morton code interleaves the 21 bits of x, y, z (x lowest).
 *   order     leaves sorted by (Morton code, leaf index).
 *   tree      breadth first from the root, which holds every leaf; a node
 *             holding m >= 2 leaves at depth d < 21 gets one child per
 *             distinct code prefix of 3 (d + 1) bits among its leaves, in
 *             code order (a single child when they all share it); at depth
 *             21 and beyond (leaves in one cell) it gets k = min(8, m)
 *             children, child j holding its leaves [j m / k, (j + 1) m / k);
 *             a node holding one leaf is that leaf.
 *   merge     (Eq. merge) bottom up: w'_i = o_i S_i with o_i the child's
 *             opacity (a leaf) or falloff (an interior node) and S_i the
 *             surface of its ellipsoid (Thomsen's formula, p = 1.6075, for
 *             the semi-axes given by its scales), w_i = w'_i / sum w';
 *             mu = sum w_i mu_i; Sigma = sum w_i (Sigma_i + (mu_i - mu)
 *             (mu_i - mu)^T); SH = sum w_i SH_i; scales = square roots of
 *             the eigenvalues of Sigma (at least 1e-20 before the root);
 *             falloff = sum w' / S_p.  A leaf's Sigma = R(q) diag(s^2)
 *             R(q)^T with q normalised.
 *   matching  top down, each node's axes (the eigenvectors, or a leaf's
 *             rotation columns, made right-handed) are re-assigned by the
 *             proper signed axis permutation P (24 of them, enumerated in a
 *             fixed order, first maximum kept) that maximises
 *             trace(R_parent^T V P), i.e. minimises the rotation between the
 *             node and its parent; the root is matched against the world
 *             axes.  Scales follow their axes.  The quaternion of the
 *             result is taken with w >= 0 at the root and q . q_parent >= 0
 *             below it.
 *   boxes     a leaf's box is mean +- 3 sqrt(diag Sigma) evaluated from its
 *             stored (FP32-rounded) scale and normalised quaternion, rounded
 *             outward to FP32; an interior node's box is the union of its
 *             children's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OB_BITS 21

typedef struct {
    int64_t n;
    const double *pos, *scale, *rot, *opacity, *sh; /* [3][n] [3][n] [4][n] [n] [48][n] */
} ob_leaves;

/* ------------------------------------------------------------------ tree */
typedef struct {
    uint64_t code;
    int64_t idx;
} ob_key;

static int cmp_key(const void *a, const void *b)
{
    const ob_key *x = (const ob_key *)a, *y = (const ob_key *)b;
    if (x->code != y->code) return x->code < y->code ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static uint64_t morton(uint32_t x, uint32_t y, uint32_t z)
{
    uint64_t c = 0;
    for (int b = 0; b < OB_BITS; ++b) {
        c |= (uint64_t)((x >> b) & 1u) << (3 * b);
        c |= (uint64_t)((y >> b) & 1u) << (3 * b + 1);
        c |= (uint64_t)((z >> b) & 1u) << (3 * b + 2);
    }
    return c;
}

/* Leaves in tree order and their codes. */
static ob_key *sorted_leaves(const ob_leaves *L)
{
    const int64_t n = L->n;
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = hi[k] = L->pos[k * n];
        for (int64_t i = 1; i < n; ++i) {
            const double v = L->pos[k * n + i];
            if (v < lo[k]) lo[k] = v;
            if (v > hi[k]) hi[k] = v;
        }
    }
    double e = 0.0;
    for (int k = 0; k < 3; ++k)
        if (hi[k] - lo[k] > e) e = hi[k] - lo[k];
    if (e == 0.0) e = 1.0;
    const double s = (double)((1u << OB_BITS) - 1u) / e;
    ob_key *key = (ob_key *)malloc(sizeof(ob_key) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k) {
            const double t = (L->pos[k * n + i] - lo[k]) * s;
            c[k] = (uint32_t)floor(t + 0.5);
        }
        key[i].code = morton(c[0], c[1], c[2]);
        key[i].idx = i;
    }
    qsort(key, (size_t)n, sizeof(ob_key), cmp_key);
    return key;
}

typedef struct {
    int64_t a, b;  /* leaves [a, b) in tree order */
    int depth;
} ob_range;

/* Children of the node holding leaves [a, b) at `depth` (m >= 2): their
 * first leaves, written to starts; returns the count. */
static int child_starts(const ob_key *key, int64_t a, int64_t b, int depth, int64_t *starts)
{
    const int64_t m = b - a;
    if (depth < OB_BITS) {
        const int shift = 3 * (OB_BITS - (depth + 1));
        int c = 0;
        starts[c++] = a;
        for (int64_t i = a + 1; i < b; ++i)
            if ((key[i].code >> shift) != (key[i - 1].code >> shift)) starts[c++] = i;
        return c;
    }
    const int64_t k = m < 8 ? m : 8;
    for (int64_t j = 0; j < k; ++j) starts[j] = a + (j * m) / k;
    return (int)k;
}

/* Breadth-first walk; writes the tree when the output arrays are given.
 * Returns the node count. */
static int64_t walk(const ob_key *key, int64_t n, int32_t *parent, int32_t *child_begin, int32_t *child_count,
                    int32_t *leaf_src, int64_t cap)
{
    int64_t qcap = 1024, head = 0, tail = 0;
    ob_range *q = (ob_range *)malloc(sizeof(ob_range) * (size_t)qcap);
    q[tail++] = (ob_range){0, n, 0};
    if (parent && cap > 0) parent[0] = -1;
    int64_t starts[8];
    while (head < tail) {
        const ob_range r = q[head];
        const int64_t id = head++;
        const int64_t m = r.b - r.a;
        if (m == 1) {
            if (child_count && id < cap) {
                child_count[id] = 0;
                child_begin[id] = 0;
                leaf_src[id] = (int32_t)key[r.a].idx;
            }
            continue;
        }
        int64_t *st = starts;  /* a cell has at most 8 non-empty octants; grouping makes at most 8 */
        const int c = child_starts(key, r.a, r.b, r.depth, st);
        if (tail + c > qcap) {
            while (tail + c > qcap) qcap *= 2;
            q = (ob_range *)realloc(q, sizeof(ob_range) * (size_t)qcap);
        }
        if (child_count && id < cap) {
            child_count[id] = c;
            child_begin[id] = (int32_t)tail;
            leaf_src[id] = -1;
        }
        for (int j = 0; j < c; ++j) {
            const int64_t e = j + 1 < c ? st[j + 1] : r.b;
            if (parent && tail < cap) parent[tail] = (int32_t)id;
            q[tail++] = (ob_range){st[j], e, r.depth + 1};
        }
    }
    free(q);
    return tail;
}

int64_t ob_count(const ob_leaves *L)
{
    if (L->n <= 0) return 0;
    ob_key *key = sorted_leaves(L);
    const int64_t N = walk(key, L->n, NULL, NULL, NULL, NULL, 0);
    free(key);
    return N;
}

/* ------------------------------------------------------------ geometry */
static void quat_to_mat(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Quaternion (w, x, y, z) of a proper rotation, from whichever of w, x, y, z
 * is largest in magnitude (the numerically stable choice), unit length. */
static void mat_to_quat(const double R[9], double q[4])
{
    const double t = R[0] + R[4] + R[8];
    const double c[4] = {1.0 + t, 1.0 + R[0] - R[4] - R[8], 1.0 - R[0] + R[4] - R[8], 1.0 - R[0] - R[4] + R[8]};
    int k = 0;
    for (int i = 1; i < 4; ++i)
        if (c[i] > c[k]) k = i;
    const double r = 2.0 * sqrt(c[k]);  /* 4 |q_k| */
    switch (k) {
    case 0: q[0] = r / 4; q[1] = (R[7] - R[5]) / r; q[2] = (R[2] - R[6]) / r; q[3] = (R[3] - R[1]) / r; break;
    case 1: q[1] = r / 4; q[0] = (R[7] - R[5]) / r; q[2] = (R[1] + R[3]) / r; q[3] = (R[2] + R[6]) / r; break;
    case 2: q[2] = r / 4; q[0] = (R[2] - R[6]) / r; q[1] = (R[1] + R[3]) / r; q[3] = (R[5] + R[7]) / r; break;
    default: q[3] = r / 4; q[0] = (R[3] - R[1]) / r; q[1] = (R[2] + R[6]) / r; q[2] = (R[5] + R[7]) / r; break;
    }
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; ++i) q[i] /= nq;
}

/* Thomsen's approximation of the surface of an ellipsoid with semi-axes
 * s[0..2]. */
static double surface(const double s[3])
{
    const double p = 1.6075;
    const double a = pow(s[0], p), b = pow(s[1], p), c = pow(s[2], p);
    return 4.0 * M_PI * pow((a * b + a * c + b * c) / 3.0, 1.0 / p);
}

/* Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations:
 * A = V diag(lam) V^T, V's columns the eigenvectors. */
static void eigen_sym3(const double A_in[9], double lam[3], double V[9])
{
    double A[9];
    memcpy(A, A_in, sizeof A);
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-36 * dia || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[3 * p + q];
                if (apq == 0.0) continue;
                const double app = A[3 * p + p], aqq = A[3 * q + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J, J the rotation in the (p, q) plane */
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[3 * k + p], akq = A[3 * k + q];
                    A[3 * k + p] = c * akp - s * akq;
                    A[3 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[3 * p + k], aqk = A[3 * q + k];
                    A[3 * p + k] = c * apk - s * aqk;
                    A[3 * q + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[3 * k + p], vkq = V[3 * k + q];
                    V[3 * k + p] = c * vkp - s * vkq;
                    V[3 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int k = 0; k < 3; ++k) lam[k] = A[4 * k];
}

static double det3(const double M[9])
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* The 24 proper signed axis permutations, in the order: permutations of
 * (0, 1, 2) lexicographically, then signs (+ + +), (+ + -), ... ; P maps new
 * axis j to old axis perm[j] with sign sg[j]: (V P)_{:, j} = sg[j] V_{:, perm[j]}. */
static int g_perm[24][3], g_sign[24][3];
static int g_nperm = 0;

static void perms_init(void)
{
    if (g_nperm) return;
    static const int P6[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int c = 0;
    for (int p = 0; p < 6; ++p)
        for (int sb = 0; sb < 8; ++sb) {
            double M[9] = {0};
            int sg[3];
            for (int j = 0; j < 3; ++j) {
                sg[j] = (sb >> (2 - j)) & 1 ? -1 : 1;
                M[3 * P6[p][j] + j] = sg[j];
            }
            if (det3(M) > 0) {
                for (int j = 0; j < 3; ++j) {
                    g_perm[c][j] = P6[p][j];
                    g_sign[c][j] = sg[j];
                }
                c++;
            }
        }
    g_nperm = c;
}

/* The proper rotation V P (axes of V re-assigned) closest to Rp, and the
 * scales following their axes. */
static void match(const double Rp[9], const double V_in[9], const double s_in[3], double R[9], double s[3])
{
    double V[9];
    memcpy(V, V_in, sizeof V);
    if (det3(V) < 0)
        for (int k = 0; k < 3; ++k) V[3 * k + 2] = -V[3 * k + 2];
    /* C = Rp^T V: trace(Rp^T V P) = sum_j sg[j] C[j][perm[j]] */
    double C[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C[3 * i + j] = Rp[i] * V[j] + Rp[3 + i] * V[3 + j] + Rp[6 + i] * V[6 + j];
    int best = 0;
    double bt = -1e300;
    for (int p = 0; p < g_nperm; ++p) {
        double tr = 0.0;
        for (int j = 0; j < 3; ++j) tr += g_sign[p][j] * C[3 * j + g_perm[p][j]];
        if (tr > bt) {
            bt = tr;
            best = p;
        }
    }
    for (int j = 0; j < 3; ++j) {
        const int o = g_perm[best][j];
        for (int k = 0; k < 3; ++k) R[3 * k + j] = g_sign[best][j] * V[3 * k + o];
        s[j] = s_in[o];
    }
}

static double round_down_f32(double x)
{
    float y = (float)x;
    if ((double)y > x) y = nextafterf(y, -INFINITY);
    return y;
}

static double round_up_f32(double x)
{
    float y = (float)x;
    if ((double)y < x) y = nextafterf(y, INFINITY);
    return y;
}

/* The hierarchy over the leaves (N = ob_count(L) nodes, breadth first).
 * Out (each [N] or [k][N], component-major): parent (-1 at the root),
 * child_begin (0 for a leaf), child_count, leaf_src (input index of a leaf
 * node, -1 for an interior node), mean, scale, rot (w, x, y, z), opacity
 * (a leaf's opacity, an interior node's falloff), sh, in FP64 (the caller
 * rounds them to FP32 to the nearest), and the boxes bmin, bmax already
 * rounded outward to FP32. */
void ob_build(const ob_leaves *L, int64_t N, int32_t *parent, int32_t *child_begin, int32_t *child_count,
              int32_t *leaf_src, double *mean, double *scale, double *rot, double *opacity, double *sh,
              float *bmin, float *bmax)
{
    perms_init();
    const int64_t n = L->n;
    ob_key *key = sorted_leaves(L);
    walk(key, n, parent, child_begin, child_count, leaf_src, N);
    free(key);

    double *cov = (double *)malloc(sizeof(double) * 9 * (size_t)N);
    double *axes = (double *)malloc(sizeof(double) * 9 * (size_t)N); /* unmatched axes (columns) */
    double *surf = (double *)malloc(sizeof(double) * (size_t)N);
    /* bottom up: children have larger ids than their parent */
    for (int64_t id = N - 1; id >= 0; --id) {
        double *S = cov + 9 * id, *V = axes + 9 * id;
        if (child_count[id] == 0) {
            const int64_t i = leaf_src[id];
            double q[4], qn = 0.0;
            for (int k = 0; k < 4; ++k) {
                q[k] = L->rot[k * n + i];
                qn += q[k] * q[k];
            }
            qn = sqrt(qn);
            for (int k = 0; k < 4; ++k) q[k] /= qn;
            double s[3];
            for (int k = 0; k < 3; ++k) {
                s[k] = L->scale[k * n + i];
                mean[k * N + id] = L->pos[k * n + i];
                scale[k * N + id] = s[k];
            }
            quat_to_mat(q, V);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += V[3 * a + k] * s[k] * s[k] * V[3 * b + k];
                    S[3 * a + b] = acc;
                }
            opacity[id] = L->opacity[i];
            for (int k = 0; k < 48; ++k) sh[k * N + id] = L->sh[k * n + i];
            surf[id] = surface(s);
            continue;
        }
        const int64_t c0 = child_begin[id], cc = child_count[id];
        double W = 0.0;
        for (int64_t c = c0; c < c0 + cc; ++c) W += opacity[c] * surf[c];
        double mu[3] = {0, 0, 0};
        for (int64_t c = c0; c < c0 + cc; ++c) {
            const double w = opacity[c] * surf[c] / W;
            for (int k = 0; k < 3; ++k) mu[k] += w * mean[k * N + c];
        }
        for (int k = 0; k < 9; ++k) S[k] = 0.0;
        for (int k = 0; k < 48; ++k) sh[k * N + id] = 0.0;
        for (int64_t c = c0; c < c0 + cc; ++c) {
            const double w = opacity[c] * surf[c] / W;
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = mean[k * N + c] - mu[k];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) S[3 * a + b] += w * (cov[9 * c + 3 * a + b] + d[a] * d[b]);
            for (int k = 0; k < 48; ++k) sh[k * N + id] += w * sh[k * N + c];
        }
        for (int k = 0; k < 3; ++k) mean[k * N + id] = mu[k];
        double lam[3], s[3];
        eigen_sym3(S, lam, V);
        for (int k = 0; k < 3; ++k) s[k] = sqrt(lam[k] > 1e-20 ? lam[k] : 1e-20);
        for (int k = 0; k < 3; ++k) scale[k * N + id] = s[k];
        surf[id] = surface(s);
        opacity[id] = W / surf[id];
    }
    /* top down: orientation matching and quaternions */
    double *Rm = (double *)malloc(sizeof(double) * 9 * (size_t)N);
    for (int64_t id = 0; id < N; ++id) {
        static const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        const double *Rp = parent[id] < 0 ? I3 : Rm + 9 * parent[id];
        double s_in[3], s[3];
        for (int k = 0; k < 3; ++k) s_in[k] = scale[k * N + id];
        match(Rp, axes + 9 * id, s_in, Rm + 9 * id, s);
        for (int k = 0; k < 3; ++k) scale[k * N + id] = s[k];
        double q[4];
        mat_to_quat(Rm + 9 * id, q);
        double dot;
        if (parent[id] < 0) {
            dot = q[0];
        } else {
            dot = 0.0;
            for (int k = 0; k < 4; ++k) dot += q[k] * rot[k * N + parent[id]];
        }
        if (dot < 0)
            for (int k = 0; k < 4; ++k) q[k] = -q[k];
        for (int k = 0; k < 4; ++k) rot[k * N + id] = q[k];
    }
    /* boxes: leaves from their stored values, interior nodes bottom up */
    for (int64_t id = N - 1; id >= 0; --id) {
        if (child_count[id] == 0) {
            double q[4], qn = 0.0, s[3], R[9];
            for (int k = 0; k < 4; ++k) {
                q[k] = (double)(float)rot[k * N + id];
                qn += q[k] * q[k];
            }
            qn = sqrt(qn);
            for (int k = 0; k < 4; ++k) q[k] /= qn;
            for (int k = 0; k < 3; ++k) s[k] = (double)(float)scale[k * N + id];
            quat_to_mat(q, R);
            for (int a = 0; a < 3; ++a) {
                const double e =
                    3.0 * sqrt(R[3 * a] * R[3 * a] * s[0] * s[0] + R[3 * a + 1] * R[3 * a + 1] * s[1] * s[1] +
                               R[3 * a + 2] * R[3 * a + 2] * s[2] * s[2]);
                const double m = (double)(float)mean[a * N + id];
                bmin[a * N + id] = (float)round_down_f32(m - e);
                bmax[a * N + id] = (float)round_up_f32(m + e);
            }
            continue;
        }
        const int64_t c0 = child_begin[id], cc = child_count[id];
        for (int a = 0; a < 3; ++a) {
            float lo = bmin[a * N + c0], hi = bmax[a * N + c0];
            for (int64_t c = c0 + 1; c < c0 + cc; ++c) {
                if (bmin[a * N + c] < lo) lo = bmin[a * N + c];
                if (bmax[a * N + c] > hi) hi = bmax[a * N + c];
            }
            bmin[a * N + id] = lo;
            bmax[a * N + id] = hi;
        }
    }
    free(Rm);
    free(cov);
    free(axes);
    free(surf);
}

/* Exposed pieces for the pins: the surface formula, the eigen-solver and
 * the matching of one node against a given parent frame. */
double ob_surface(const double s[3]) { return surface(s); }
void ob_eigen(const double A[9], double lam[3], double V[9]) { eigen_sym3(A, lam, V); }
void ob_match(const double Rp[9], const double V[9], const double s_in[3], double R[9], double s[3])
{
    perms_init();
    match(Rp, V, s_in, R, s);
}
