/*
 * FP64 CPU oracle for the per-view hierarchy cut and splatting path of
 * "A Hierarchical 3D Gaussian Representation for Real-Time Rendering of Very
 * Large Datasets" (Kerbl et al., ACM TOG 43(4), 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition the GPU
 * library is checked against.  It shares no code with the HIP path and is
 * called only by the tests, the smoke check and the benchmark's CPU-baseline
 * leg.  Every quantity is computed in double precision from the FP32 values a
 * caller stores (the Python wrapper widens them).
 *
 * What each function follows:
 *   or_granularity  Sec. 4.2 "Hierarchy Cut Selection": projected size of the
 *                   largest dimension of a node's leaf bounding box.
 *   or_cut          Sec. 4.2: a node is in the cut when it meets the target
 *                   granularity and its parent does not; found here by a
 *                   top-down descent (the first node on each root-to-leaf path
 *                   that meets it), a different algorithm from the GPU's
 *                   per-node predicate.  Weights t from Eq. (t_interp).
 *   or_project      Sec. 4.2 interpolation of position, scale, rotation (lerp,
 *                   then normalise) and SH; Sec. 3 background, Eq. (alpha)
 *                   and the projected Gaussian G; the EWA low-pass of
 *                   Sec. 5.1 (last paragraph) as a screen-space dilation with
 *                   opacity compensation.
 *   or_render       Eq. (alpha), the opacity transition of Eq. (alphap)
 *                   generalised to K children (Sec. 5.2) and blended with the
 *                   weight of Sec. 4.2, the 0.99 clamp of Sec. 7.3, and
 *                   front-to-back compositing.
 *   or_backward     The adjoint of all of the above with respect to every
 *                   node's parameters (Sec. 5.1, 7.1 "Implementation"):
 *                   gradients reach node and parent through the
 *                   interpolation, and through the pow of Eq. (alphap);
 *                   opacity uses an absolute-value activation and its
 *                   gradient is zero where the clamp is active (Sec. 7.3).
 *                   Leaf masking is applied by the caller.
 *
 * Readings of points the paper leaves open (fixed constants, named below):
 *   t is the PARENT's weight: x~ = (1-t) x_n + t x_p and
 *   alpha = (1-t) a_n + t (1 - (1 - a_p)^(1/K)), both continuous at the ends
 *   of a transition; a_p is evaluated per pixel with the interpolated
 *   footprint; K = number of children of the parent; t = 0 for the root,
 *   for a parent inside the eye's box, or when eps(p) <= eps(n);
 *   t is clamped to [0, 1].  Skip a splat whose alpha < 1/255, stop before a
 *   splat that would take transmittance below 1e-4, black background,
 *   dilation 0.3 px^2, near plane 0.2, colour = max(0, SH.Y + 1/2) with the
 *   real orthonormal SH basis (no Condon-Shortley phase), pixel (i, j)
 *   sampled at (i + 1/2, j + 1/2), splats ordered per pixel by (FP32 depth,
 *   node id).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_ALPHA_MIN (1.0 / 255.0)
#define OR_T_MIN 1e-4
#define OR_ALPHA_MAX 0.99
#define OR_DILATION 0.3
#define OR_GUARD 1e-4
#define OR_MAX_ALT 4

typedef struct {
    int64_t n;
    const int32_t *parent, *child_begin, *child_count;
    const double *bmin, *bmax;                       /* [3][n] */
    const double *mean, *scale, *rot, *opacity, *sh; /* [3][n] [3][n] [4][n] [n] [48][n] */
} or_hier;

typedef struct {
    double R[9];   /* rows: right, down, forward (world -> camera) */
    double eye[3];
    double fx, fy, cx, cy;
    int32_t width, height;
    double z_near, tau;
} or_view;

/* One projected splat (a cut node after interpolation). */
typedef struct {
    int32_t node, parent, K, valid;
    double t;
    double mu_rel[3];        /* interpolated mean minus eye */
    double s[3], qraw[4], q[4], qnorm;
    double sh[48];
    double o_n, o_p;
    double pc[3];            /* camera-space position */
    double Tm[6];            /* J R, 2x3 row-major */
    double cov3[9];
    double a, b, c;          /* Sigma2 before dilation */
    double kappa, conic[3];  /* conic: quadratic form ca dx^2 + 2 cb dx dy + cc dy^2 */
    double u, v, depth;
    float depth32;
    double dir[3], Y[16], raw[3], rgb[3];
    double A_n, A_p;
    int32_t x0, x1, y0, y1;  /* footprint pixel range, inclusive; empty if x1 < x0 */
} or_splat;

/* ---------------------------------------------------------------------- */
/* granularity and cut (Sec. 4.2)                                          */
/* ---------------------------------------------------------------------- */

/* Projected size of the largest box dimension: f * L / d with d the distance
 * from the eye to the box (zero inside the box, where eps = +inf). */
double or_granularity(const or_hier *h, const or_view *v, int64_t i)
{
    const int64_t n = h->n;
    double L = 0.0, d2 = 0.0;
    double dk[3];
    for (int k = 0; k < 3; ++k) {
        double lo = h->bmin[k * n + i], hi = h->bmax[k * n + i];
        double ext = hi - lo;
        if (ext > L) L = ext;
        double e = v->eye[k];
        double c = e < lo ? lo : (e > hi ? hi : e);
        dk[k] = e - c;
    }
    d2 = (dk[0] * dk[0] + dk[1] * dk[1]) + dk[2] * dk[2];
    double d = sqrt(d2);
    if (d == 0.0) return INFINITY;
    double f = v->fx > v->fy ? v->fx : v->fy;
    return (f * L) / d;
}

void or_granularity_all(const or_hier *h, const or_view *v, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < h->n; ++i) out[i] = or_granularity(h, v, i);
}

static int meets(const or_hier *h, const or_view *v, int64_t i)
{
    if (h->child_count[i] == 0) return 1;  /* leaves always qualify */
    return or_granularity(h, v, i) <= v->tau;
}

/* Weight of the parent in the interpolation, Eq. (t_interp). */
double or_weight(const or_hier *h, const or_view *v, int64_t i)
{
    int32_t p = h->parent[i];
    if (p < 0) return 0.0;
    double en = or_granularity(h, v, i);
    double ep = or_granularity(h, v, p);
    if (isinf(ep) || !(ep > en)) return 0.0;
    double t = (v->tau - en) / (ep - en);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return t;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Top-down descent.  Returns the cut size; writes at most cap ids (ascending)
 * and weights. */
int64_t or_cut(const or_hier *h, const or_view *v, int32_t *out_ids, double *out_t, int64_t cap)
{
    int64_t count = 0;
    int64_t *stack = (int64_t *)malloc(sizeof(int64_t) * 4096);
    int64_t sp = 0, scap = 4096;
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (h->n > 0 ? h->n : 1));
    if (h->n > 0) stack[sp++] = 0;
    while (sp > 0) {
        int64_t i = stack[--sp];
        if (meets(h, v, i)) {
            tmp[count++] = (int32_t)i;
            continue;
        }
        int32_t cb = h->child_begin[i], cc = h->child_count[i];
        if (sp + cc > scap) {
            scap = 2 * (sp + cc);
            stack = (int64_t *)realloc(stack, sizeof(int64_t) * scap);
        }
        for (int32_t k = cc - 1; k >= 0; --k) stack[sp++] = cb + k;
    }
    qsort(tmp, (size_t)count, sizeof(int32_t), cmp_i32);
    for (int64_t k = 0; k < count && k < cap; ++k) {
        out_ids[k] = tmp[k];
        if (out_t) out_t[k] = or_weight(h, v, tmp[k]);
    }
    free(tmp);
    free(stack);
    return count;
}

/* ---------------------------------------------------------------------- */
/* SH basis (real, orthonormal, degree 3), and its gradient                */
/* ---------------------------------------------------------------------- */
static void sh_basis(const double d[3], double Y[16])
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    Y[0] = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    Y[1] = c1 * y;
    Y[2] = c1 * z;
    Y[3] = c1 * x;
    const double c2 = 0.5 * sqrt(15.0 / pi);
    Y[4] = c2 * x * y;
    Y[5] = c2 * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = c2 * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    Y[9] = 0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = 0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    Y[13] = 0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = 0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

/* dY[k][0..2] = gradient of the polynomial Y_k with respect to (x, y, z). */
static void sh_basis_grad(const double d[3], double dY[16][3])
{
    const double x = d[0], y = d[1], z = d[2];
    const double pi = M_PI;
    memset(dY, 0, sizeof(double) * 48);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    dY[1][1] = c1;
    dY[2][2] = c1;
    dY[3][0] = c1;
    const double c2 = 0.5 * sqrt(15.0 / pi);
    dY[4][0] = c2 * y; dY[4][1] = c2 * x;
    dY[5][1] = c2 * z; dY[5][2] = c2 * y;
    dY[6][2] = 0.25 * sqrt(5.0 / pi) * 6.0 * z;
    dY[7][0] = c2 * z; dY[7][2] = c2 * x;
    const double c22 = 0.25 * sqrt(15.0 / pi);
    dY[8][0] = c22 * 2.0 * x; dY[8][1] = -c22 * 2.0 * y;
    const double c33 = 0.25 * sqrt(35.0 / (2.0 * pi));
    dY[9][0] = c33 * 6.0 * x * y; dY[9][1] = c33 * (3.0 * x * x - 3.0 * y * y);
    const double c32 = 0.5 * sqrt(105.0 / pi);
    dY[10][0] = c32 * y * z; dY[10][1] = c32 * x * z; dY[10][2] = c32 * x * y;
    const double c31 = 0.25 * sqrt(21.0 / (2.0 * pi));
    dY[11][1] = c31 * (5.0 * z * z - 1.0); dY[11][2] = c31 * y * 10.0 * z;
    const double c30 = 0.25 * sqrt(7.0 / pi);
    dY[12][2] = c30 * (15.0 * z * z - 3.0);
    dY[13][0] = c31 * (5.0 * z * z - 1.0); dY[13][2] = c31 * x * 10.0 * z;
    const double c3m = 0.25 * sqrt(105.0 / pi);
    dY[14][0] = c3m * 2.0 * x * z; dY[14][1] = -c3m * 2.0 * y * z; dY[14][2] = c3m * (x * x - y * y);
    dY[15][0] = c33 * (3.0 * x * x - 3.0 * y * y); dY[15][1] = -c33 * 6.0 * x * y;
}

void or_sh_basis(const double d[3], double Y[16]) { sh_basis(d, Y); }

/* ---------------------------------------------------------------------- */
/* projection (Sec. 3, 4.2, 5.1)                                            */
/* ---------------------------------------------------------------------- */
static void quat_to_mat(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static void project_one(const or_hier *h, const or_view *v, int32_t node, double t, or_splat *S)
{
    const int64_t n = h->n;
    memset(S, 0, sizeof(*S));
    S->node = node;
    int32_t p = h->parent[node];
    S->parent = p;
    if (p < 0) t = 0.0;
    S->t = t;
    S->K = p >= 0 ? h->child_count[p] : 1;
    const int32_t pp = p >= 0 ? p : node;
    const double w0 = 1.0 - t, w1 = t;

    for (int k = 0; k < 3; ++k) {
        double mn = h->mean[k * n + node], mp = h->mean[k * n + pp];
        S->mu_rel[k] = (mn - v->eye[k]) + t * (mp - mn);
        S->s[k] = w0 * h->scale[k * n + node] + w1 * h->scale[k * n + pp];
    }
    double qq = 0.0;
    for (int k = 0; k < 4; ++k) {
        S->qraw[k] = w0 * h->rot[k * n + node] + w1 * h->rot[k * n + pp];
        qq += S->qraw[k] * S->qraw[k];
    }
    S->qnorm = sqrt(qq);
    for (int k = 0; k < 4; ++k) S->q[k] = S->qraw[k] / S->qnorm;
    for (int k = 0; k < 48; ++k) S->sh[k] = w0 * h->sh[k * n + node] + w1 * h->sh[k * n + pp];
    S->o_n = fabs(h->opacity[node]);
    S->o_p = p >= 0 ? fabs(h->opacity[p]) : 0.0;

    for (int i = 0; i < 3; ++i)
        S->pc[i] = v->R[3 * i] * S->mu_rel[0] + v->R[3 * i + 1] * S->mu_rel[1] + v->R[3 * i + 2] * S->mu_rel[2];
    S->depth = S->pc[2];
    S->depth32 = (float)S->pc[2];
    S->x0 = 0; S->x1 = -1; S->y0 = 0; S->y1 = -1;
    if (!(S->pc[2] > v->z_near)) return;  /* near-plane cull */

    const double x = S->pc[0], y = S->pc[1], z = S->pc[2];
    double Rq[9];
    quat_to_mat(S->q, Rq);
    double M[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * S->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += M[3 * i + k] * M[3 * j + k];
            S->cov3[3 * i + j] = acc;
        }
    const double J[6] = {v->fx / z, 0.0, -v->fx * x / (z * z), 0.0, v->fy / z, -v->fy * y / (z * z)};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[3 * i + k] * v->R[3 * k + j];
            S->Tm[3 * i + j] = acc;
        }
    double TS[6];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += S->Tm[3 * i + k] * S->cov3[3 * k + j];
            TS[3 * i + j] = acc;
        }
    double c2[4];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += TS[3 * i + k] * S->Tm[3 * j + k];
            c2[2 * i + j] = acc;
        }
    S->a = c2[0];
    S->b = 0.5 * (c2[1] + c2[2]);
    S->c = c2[3];
    const double ad = S->a + OR_DILATION, cd = S->c + OR_DILATION;
    const double D = S->a * S->c - S->b * S->b;
    const double Dd = ad * cd - S->b * S->b;
    if (!(Dd > 0.0)) return;
    S->kappa = D > 0.0 ? sqrt(D / Dd) : 0.0;
    S->conic[0] = cd / Dd;
    S->conic[1] = -S->b / Dd;
    S->conic[2] = ad / Dd;
    S->u = v->fx * x / z + v->cx;
    S->v = v->fy * y / z + v->cy;

    double r = sqrt(S->mu_rel[0] * S->mu_rel[0] + S->mu_rel[1] * S->mu_rel[1] + S->mu_rel[2] * S->mu_rel[2]);
    for (int k = 0; k < 3; ++k) S->dir[k] = S->mu_rel[k] / r;
    sh_basis(S->dir, S->Y);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < 16; ++k) acc += S->sh[3 * k + ch] * S->Y[k];
        S->raw[ch] = acc + 0.5;
        S->rgb[ch] = S->raw[ch] > 0.0 ? S->raw[ch] : 0.0;
    }
    S->A_n = S->kappa * S->o_n;
    S->A_p = S->kappa * S->o_p;
    S->valid = 1;

    /* Footprint: alpha <= min(0.99, A G) with A = kappa((1-t)o_n + t o_p),
     * so a pixel can reach alpha_min only inside the ellipse
     * d^T Sigma'^-1 d <= 2 ln(A / alpha_min).  The per-pixel test decides. */
    const double A = S->kappa * (w0 * S->o_n + w1 * S->o_p);
    if (!(A >= OR_ALPHA_MIN)) return;
    const double r2 = 2.0 * log(A / OR_ALPHA_MIN);
    const double hx = sqrt(r2 * ad), hy = sqrt(r2 * cd);
    double fx0 = ceil(S->u - hx - 0.5), fx1 = floor(S->u + hx - 0.5);
    double fy0 = ceil(S->v - hy - 0.5), fy1 = floor(S->v + hy - 0.5);
    if (fx0 < 0) fx0 = 0;
    if (fy0 < 0) fy0 = 0;
    if (fx1 > v->width - 1) fx1 = v->width - 1;
    if (fy1 > v->height - 1) fy1 = v->height - 1;
    if (fx1 < fx0 || fy1 < fy0) return;
    S->x0 = (int32_t)fx0; S->x1 = (int32_t)fx1;
    S->y0 = (int32_t)fy0; S->y1 = (int32_t)fy1;
}

/* Splat parameters for a list of cut nodes (flat export for tests):
 * out[k*OR_NSPLAT + ...] = valid, u, v, depth, conic(3), kappa, A_n, A_p, t, K,
 * rgb(3), x0, x1, y0, y1. */
#define OR_NSPLAT 20
void or_project(const or_hier *h, const or_view *v, const int32_t *ids, const double *t,
                int64_t count, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        or_splat S;
        project_one(h, v, ids[k], t[k], &S);
        double *o = out + k * OR_NSPLAT;
        o[0] = S.valid; o[1] = S.u; o[2] = S.v; o[3] = S.depth;
        o[4] = S.conic[0]; o[5] = S.conic[1]; o[6] = S.conic[2];
        o[7] = S.kappa; o[8] = S.A_n; o[9] = S.A_p; o[10] = S.t; o[11] = S.K;
        o[12] = S.rgb[0]; o[13] = S.rgb[1]; o[14] = S.rgb[2];
        o[15] = S.x0; o[16] = S.x1; o[17] = S.y0; o[18] = S.y1;
        o[19] = S.depth32;
    }
}

/* ---------------------------------------------------------------------- */
/* per-pixel alpha and compositing (Eq. alpha, Eq. alphap, Sec. 7.3)        */
/* ---------------------------------------------------------------------- */
typedef struct {
    double G, an, ap, apr, alpha;  /* apr = 1 - (1 - a_p)^(1/K) */
    int clamp_n, clamp_p;
    double dx, dy;
} or_alpha_t;

static void splat_alpha(const or_splat *S, int px, int py, or_alpha_t *o)
{
    o->dx = (px + 0.5) - S->u;
    o->dy = (py + 0.5) - S->v;
    const double Q = S->conic[0] * o->dx * o->dx + 2.0 * S->conic[1] * o->dx * o->dy + S->conic[2] * o->dy * o->dy;
    o->G = exp(-0.5 * Q);
    double an = S->A_n * o->G;
    o->clamp_n = an > OR_ALPHA_MAX;
    o->an = o->clamp_n ? OR_ALPHA_MAX : an;
    o->ap = 0.0; o->apr = 0.0; o->clamp_p = 0;
    if (S->t > 0.0) {
        double ap = S->A_p * o->G;
        o->clamp_p = ap > OR_ALPHA_MAX;
        o->ap = o->clamp_p ? OR_ALPHA_MAX : ap;
        o->apr = 1.0 - pow(1.0 - o->ap, 1.0 / S->K);
        o->alpha = (1.0 - S->t) * o->an + S->t * o->apr;
    } else {
        o->alpha = o->an;
    }
}

typedef struct {
    int64_t nsplat;
    or_splat *splats;
    int32_t *order;        /* splat indices sorted by (depth32, node) */
} or_frame;

static const or_splat *g_sort_splats;
static int cmp_order(const void *a, const void *b)
{
    const or_splat *x = g_sort_splats + *(const int32_t *)a;
    const or_splat *y = g_sort_splats + *(const int32_t *)b;
    if (x->depth32 < y->depth32) return -1;
    if (x->depth32 > y->depth32) return 1;
    return (x->node > y->node) - (x->node < y->node);
}

static void frame_build(const or_hier *h, const or_view *v, const int32_t *ids, const double *t,
                        int64_t count, or_frame *F)
{
    F->nsplat = count;
    F->splats = (or_splat *)malloc(sizeof(or_splat) * (count > 0 ? count : 1));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) project_one(h, v, ids[k], t[k], &F->splats[k]);
    F->order = (int32_t *)malloc(sizeof(int32_t) * (count > 0 ? count : 1));
    for (int64_t k = 0; k < count; ++k) F->order[k] = (int32_t)k;
    g_sort_splats = F->splats;
    qsort(F->order, (size_t)count, sizeof(int32_t), cmp_order);
}

static void frame_free(or_frame *F)
{
    free(F->splats);
    free(F->order);
}

/* Per-pixel candidate lists (CSR) for the requested pixels: every splat whose
 * footprint range contains the pixel, in (depth32, node) order. */
typedef struct {
    int64_t npix;
    int64_t *start;   /* npix + 1 */
    int32_t *items;
} or_lists;

static void lists_build(const or_frame *F, const or_view *v, const int64_t *pix, int64_t npix, or_lists *Lst)
{
    const int64_t W = v->width, H = v->height;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * W * H);
    for (int64_t i = 0; i < W * H; ++i) slot[i] = -1;
    /* the requested pixels' bounding box: footprint ranges are visited only
     * inside it (pixels outside it are not requested) */
    int bx0 = (int)W, bx1 = -1, by0 = (int)H, by1 = -1;
    for (int64_t k = 0; k < npix; ++k) {
        slot[pix[k]] = k;
        const int x = (int)(pix[k] % W), y = (int)(pix[k] / W);
        if (x < bx0) bx0 = x;
        if (x > bx1) bx1 = x;
        if (y < by0) by0 = y;
        if (y > by1) by1 = y;
    }
    int64_t *cnt = (int64_t *)calloc((size_t)npix + 1, sizeof(int64_t));
    for (int64_t oi = 0; oi < F->nsplat; ++oi) {
        const or_splat *S = &F->splats[F->order[oi]];
        if (!S->valid) continue;
        const int y0 = S->y0 > by0 ? S->y0 : by0, y1 = S->y1 < by1 ? S->y1 : by1;
        const int x0 = S->x0 > bx0 ? S->x0 : bx0, x1 = S->x1 < bx1 ? S->x1 : bx1;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                int64_t s = slot[(int64_t)y * W + x];
                if (s >= 0) cnt[s + 1]++;
            }
    }
    for (int64_t k = 0; k < npix; ++k) cnt[k + 1] += cnt[k];
    int32_t *items = (int32_t *)malloc(sizeof(int32_t) * (cnt[npix] > 0 ? cnt[npix] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (npix > 0 ? npix : 1));
    for (int64_t k = 0; k < npix; ++k) fill[k] = cnt[k];
    for (int64_t oi = 0; oi < F->nsplat; ++oi) {
        int32_t si = F->order[oi];
        const or_splat *S = &F->splats[si];
        if (!S->valid) continue;
        const int y0 = S->y0 > by0 ? S->y0 : by0, y1 = S->y1 < by1 ? S->y1 : by1;
        const int x0 = S->x0 > bx0 ? S->x0 : bx0, x1 = S->x1 < bx1 ? S->x1 : bx1;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) {
                int64_t s = slot[(int64_t)y * W + x];
                if (s >= 0) items[fill[s]++] = si;
            }
    }
    free(fill);
    free(slot);
    Lst->npix = npix;
    Lst->start = cnt;
    Lst->items = items;
}

static void lists_free(or_lists *L)
{
    free(L->start);
    free(L->items);
}

/* Composite one pixel front to back.  flip >= 0 inverts the flip-th
 * near-threshold decision (see or_render).  Returns the number of blended
 * splats; near-threshold decisions are counted in *n_near, and blended
 * splats whose unclamped a_n or a_p lies within the same relative guard of
 * the 0.99 clamp in *n_clamp (there the value is continuous but its
 * derivative is not: either side's gradient is a correct one). */
static int composite(const or_frame *F, const int32_t *items, int64_t m, int px, int py, int flip,
                     double rgb[3], double *T_out, int *n_near, int *n_clamp, uint64_t *sig)
{
    double T = 1.0, C[3] = {0, 0, 0};
    int nb = 0, near = 0, nclamp = 0;
    uint64_t hsh = 1469598103934665603ULL;
    for (int64_t k = 0; k < m; ++k) {
        const or_splat *S = &F->splats[items[k]];
        or_alpha_t a;
        splat_alpha(S, px, py, &a);
        /* skip decision */
        int skip = a.alpha < OR_ALPHA_MIN;
        if (fabs(a.alpha / OR_ALPHA_MIN - 1.0) < OR_GUARD) {
            if (near == flip) skip = !skip;
            near++;
        }
        if (skip) continue;
        const double Tn = T * (1.0 - a.alpha);
        int stop = Tn < OR_T_MIN;
        if (fabs(Tn / OR_T_MIN - 1.0) < OR_GUARD) {
            if (near == flip) stop = !stop;
            near++;
        }
        if (stop) break;
        for (int ch = 0; ch < 3; ++ch) C[ch] += S->rgb[ch] * a.alpha * T;
        T = Tn;
        nb++;
        if (fabs(S->A_n * a.G / OR_ALPHA_MAX - 1.0) < OR_GUARD ||
            (S->t > 0.0 && fabs(S->A_p * a.G / OR_ALPHA_MAX - 1.0) < OR_GUARD))
            nclamp++;
        if (sig) {
            uint64_t token = (uint64_t)(uint32_t)S->node * 8u + (uint64_t)(a.clamp_n * 4 + a.clamp_p * 2) +
                             ((uint64_t)((S->raw[0] > 0) | ((S->raw[1] > 0) << 1) | ((S->raw[2] > 0) << 2)) << 40);
            hsh = (hsh ^ token) * 1099511628211ULL;
        }
    }
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = C[ch];
    *T_out = T;
    if (n_near) *n_near = near;
    if (n_clamp) *n_clamp = nclamp;
    if (sig) *sig = hsh;
    return nb;
}

/* Render the requested pixels of one view.
 *   pix[npix]          linear pixel indices y*W + x
 *   rgb[npix*3], T[npix], nblend[npix]      nominal result
 *   nalt[npix], alt_rgb[npix*OR_MAX_ALT*3], alt_T[npix*OR_MAX_ALT]
 *       results with one near-threshold decision inverted (decisions whose
 *       quantity lies within a relative 1e-4 of its threshold), at most 4.
 *   nclamp[npix] (optional) blended splats of the pixel whose unclamped
 *       opacity term lies within a relative 1e-4 of the 0.99 clamp.
 * Returns the total number of blended (pixel, splat) pairs. */
int64_t or_render(const or_hier *h, const or_view *v, const int32_t *ids, const double *t, int64_t count,
                  const int64_t *pix, int64_t npix, double *rgb, double *T, int32_t *nblend,
                  int32_t *nalt, double *alt_rgb, double *alt_T, int32_t *nclamp)
{
    or_frame F;
    frame_build(h, v, ids, t, count, &F);
    or_lists L;
    lists_build(&F, v, pix, npix, &L);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t k = 0; k < npix; ++k) {
        const int px = (int)(pix[k] % v->width), py = (int)(pix[k] / v->width);
        const int32_t *items = L.items + L.start[k];
        const int64_t m = L.start[k + 1] - L.start[k];
        int nn = 0, nc = 0;
        nblend[k] = composite(&F, items, m, px, py, -1, rgb + 3 * k, T + k, &nn, &nc, NULL);
        if (nclamp) nclamp[k] = nc;
        total += nblend[k];
        int na = nn < OR_MAX_ALT ? nn : OR_MAX_ALT;
        if (nalt) {
            nalt[k] = na;
            for (int f = 0; f < na; ++f)
                composite(&F, items, m, px, py, f, alt_rgb + (k * OR_MAX_ALT + f) * 3, alt_T + k * OR_MAX_ALT + f,
                          NULL, NULL, NULL);
        }
    }
    lists_free(&L);
    frame_free(&F);
    return total;
}

/* Hash of every decision the listed pixels pix[npix] depend on (contributing
 * set and order, clamp states, colour clamps), used to reject
 * finite-difference steps that cross a discontinuity. */
uint64_t or_signature_pix(const or_hier *h, const or_view *v, const int32_t *ids, const double *t, int64_t count,
                          const int64_t *pix, int64_t npix)
{
    or_frame F;
    frame_build(h, v, ids, t, count, &F);
    or_lists L;
    lists_build(&F, v, pix, npix, &L);
    uint64_t acc = 0;
    for (int64_t k = 0; k < npix; ++k) {
        double rgb[3], T;
        uint64_t s;
        composite(&F, L.items + L.start[k], L.start[k + 1] - L.start[k], (int)(pix[k] % v->width),
                  (int)(pix[k] / v->width), -1, rgb, &T, NULL, NULL, &s);
        acc = (acc ^ (s + (uint64_t)pix[k] * 0x9E3779B97F4A7C15ULL)) * 1099511628211ULL;
    }
    lists_free(&L);
    frame_free(&F);
    return acc;
}

/* The same over every pixel of the view. */
uint64_t or_signature(const or_hier *h, const or_view *v, const int32_t *ids, const double *t, int64_t count)
{
    const int64_t npix = (int64_t)v->width * v->height;
    int64_t *pix = (int64_t *)malloc(sizeof(int64_t) * (npix > 0 ? npix : 1));
    for (int64_t k = 0; k < npix; ++k) pix[k] = k;
    const uint64_t acc = or_signature_pix(h, v, ids, t, count, pix, npix);
    free(pix);
    return acc;
}

/* ---------------------------------------------------------------------- */
/* backward                                                                 */
/* ---------------------------------------------------------------------- */
/* Per-splat adjoints of the screen-space quantities. */
typedef struct {
    double du, dv, dconic[3], dAn, dAp, drgb[3], dt_alpha;
} or_sgrad;

/* Parameter slots of the gradient array, each [n] long:
 * 0..2 mean, 3..5 scale, 6..9 rot, 10 opacity, 11..58 sh. */
#define OR_NPARAM 59

static void splat_backward(const or_hier *h, const or_view *v, const or_splat *S, const or_sgrad *g,
                           double *grad, double *dt_out)
{
    const int64_t n = h->n;
    if (!S->valid) return;
    const double t = S->t, w0 = 1.0 - t, w1 = t;
    const int32_t node = S->node, p = S->parent;
    const int32_t pp = p >= 0 ? p : node;

    /* colour: rgb = max(0, sh . Y(dir) + 1/2) */
    double dsh[48];
    double ddir[3] = {0, 0, 0};
    double dY[16][3];
    sh_basis_grad(S->dir, dY);
    for (int ch = 0; ch < 3; ++ch) {
        const double gr = S->raw[ch] > 0.0 ? g->drgb[ch] : 0.0;
        for (int k = 0; k < 16; ++k) {
            dsh[3 * k + ch] = gr * S->Y[k];
            for (int m = 0; m < 3; ++m) ddir[m] += gr * S->sh[3 * k + ch] * dY[k][m];
        }
    }
    double dmu[3];
    {
        double r = sqrt(S->mu_rel[0] * S->mu_rel[0] + S->mu_rel[1] * S->mu_rel[1] + S->mu_rel[2] * S->mu_rel[2]);
        double dd = S->dir[0] * ddir[0] + S->dir[1] * ddir[1] + S->dir[2] * ddir[2];
        for (int m = 0; m < 3; ++m) dmu[m] = (ddir[m] - S->dir[m] * dd) / r;
    }

    /* opacity and kappa: A_n = kappa o_n, A_p = kappa o_p */
    const double dkappa = g->dAn * S->o_n + g->dAp * S->o_p;
    const double don = g->dAn * S->kappa, dop = g->dAp * S->kappa;

    /* conic and kappa from Sigma2 = (a, b, c) with dilation h */
    const double a = S->a, b = S->b, c = S->c;
    const double ad = a + OR_DILATION, cd = c + OR_DILATION;
    const double Dd = ad * cd - b * b, D = a * c - b * b;
    const double Dd2 = Dd * Dd;
    double da = 0, db = 0, dc = 0;
    /* ca = cd/Dd, cb = -b/Dd, cc = ad/Dd */
    const double gca = g->dconic[0], gcb = g->dconic[1], gcc = g->dconic[2];
    da += gca * (-cd * cd / Dd2) + gcb * (b * cd / Dd2) + gcc * (1.0 / Dd - ad * cd / Dd2);
    dc += gca * (1.0 / Dd - cd * ad / Dd2) + gcb * (b * ad / Dd2) + gcc * (-ad * ad / Dd2);
    db += gca * (2.0 * b * cd / Dd2) + gcb * (-1.0 / Dd - 2.0 * b * b / Dd2) + gcc * (2.0 * b * ad / Dd2);
    if (D > 0.0 && S->kappa > 0.0) {
        const double k2 = 0.5 * S->kappa;
        da += dkappa * k2 * (c / D - cd / Dd);
        dc += dkappa * k2 * (a / D - ad / Dd);
        db += dkappa * k2 * (-2.0 * b / D + 2.0 * b / Dd);
    }

    /* Sigma2 = Tm Sigma3 Tm^T: a = T0 S T0^T, b = T0 S T1^T, c = T1 S T1^T */
    const double *T0 = S->Tm, *T1 = S->Tm + 3;
    double T0S[3], T1S[3];
    for (int j = 0; j < 3; ++j) {
        T0S[j] = T0[0] * S->cov3[j] + T0[1] * S->cov3[3 + j] + T0[2] * S->cov3[6 + j];
        T1S[j] = T1[0] * S->cov3[j] + T1[1] * S->cov3[3 + j] + T1[2] * S->cov3[6 + j];
    }
    double dS3[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            dS3[3 * i + j] = da * T0[i] * T0[j] + db * T0[i] * T1[j] + dc * T1[i] * T1[j];
    double dT[6];
    for (int j = 0; j < 3; ++j) {
        dT[j] = 2.0 * da * T0S[j] + db * T1S[j];
        dT[3 + j] = db * T0S[j] + 2.0 * dc * T1S[j];
    }
    /* Tm = J R: dJ = dT R^T */
    double dJ[6];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int j = 0; j < 3; ++j) acc += dT[3 * i + j] * v->R[3 * k + j];
            dJ[3 * i + k] = acc;
        }
    const double x = S->pc[0], y = S->pc[1], z = S->pc[2];
    const double z2 = z * z, z3 = z2 * z;
    double dp[3] = {0, 0, 0};
    dp[0] += dJ[2] * (-v->fx / z2);
    dp[1] += dJ[5] * (-v->fy / z2);
    dp[2] += dJ[0] * (-v->fx / z2) + dJ[2] * (2.0 * v->fx * x / z3) + dJ[4] * (-v->fy / z2) +
             dJ[5] * (2.0 * v->fy * y / z3);
    /* pixel centre u = fx x/z + cx, v = fy y/z + cy */
    dp[0] += g->du * v->fx / z;
    dp[2] += -g->du * v->fx * x / z2;
    dp[1] += g->dv * v->fy / z;
    dp[2] += -g->dv * v->fy * y / z2;
    /* pc = R mu_rel */
    for (int k = 0; k < 3; ++k) dmu[k] += v->R[k] * dp[0] + v->R[3 + k] * dp[1] + v->R[6 + k] * dp[2];

    /* Sigma3 = M M^T, M = Rq diag(s): dM = (dS3 + dS3^T) M */
    double Rq[9], M[9], dM[9];
    quat_to_mat(S->q, Rq);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * S->s[j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += (dS3[3 * i + k] + dS3[3 * k + i]) * M[3 * k + j];
            dM[3 * i + j] = acc;
        }
    double ds[3], dR[9];
    for (int j = 0; j < 3; ++j) {
        ds[j] = 0.0;
        for (int i = 0; i < 3; ++i) {
            ds[j] += dM[3 * i + j] * Rq[3 * i + j];
            dR[3 * i + j] = dM[3 * i + j] * S->s[j];
        }
    }
    const double qw = S->q[0], qx = S->q[1], qy = S->q[2], qz = S->q[3];
    double dq[4];
    dq[0] = dR[1] * (-2 * qz) + dR[2] * (2 * qy) + dR[3] * (2 * qz) + dR[5] * (-2 * qx) + dR[6] * (-2 * qy) +
            dR[7] * (2 * qx);
    dq[1] = dR[1] * (2 * qy) + dR[2] * (2 * qz) + dR[3] * (2 * qy) + dR[4] * (-4 * qx) + dR[5] * (-2 * qw) +
            dR[6] * (2 * qz) + dR[7] * (2 * qw) + dR[8] * (-4 * qx);
    dq[2] = dR[0] * (-4 * qy) + dR[1] * (2 * qx) + dR[2] * (2 * qw) + dR[3] * (2 * qx) + dR[5] * (2 * qz) +
            dR[6] * (-2 * qw) + dR[7] * (2 * qz) + dR[8] * (-4 * qy);
    dq[3] = dR[0] * (-4 * qz) + dR[1] * (-2 * qw) + dR[2] * (2 * qx) + dR[3] * (2 * qw) + dR[4] * (-4 * qz) +
            dR[5] * (2 * qy) + dR[6] * (2 * qx) + dR[7] * (2 * qy);
    /* q = qraw / |qraw| */
    double dqraw[4];
    {
        double qd = qw * dq[0] + qx * dq[1] + qy * dq[2] + qz * dq[3];
        for (int k = 0; k < 4; ++k) dqraw[k] = (dq[k] - S->q[k] * qd) / S->qnorm;
    }

    /* interpolation: node gets (1-t), parent gets t; dL/dt collected */
    double dt = g->dt_alpha;
    for (int k = 0; k < 3; ++k) {
        double mn = h->mean[k * n + node], mp = h->mean[k * n + pp];
        grad[(0 + k) * n + node] += w0 * dmu[k];
        if (p >= 0) grad[(0 + k) * n + p] += w1 * dmu[k];
        dt += dmu[k] * (mp - mn);
        double sn = h->scale[k * n + node], sp = h->scale[k * n + pp];
        grad[(3 + k) * n + node] += w0 * ds[k];
        if (p >= 0) grad[(3 + k) * n + p] += w1 * ds[k];
        dt += ds[k] * (sp - sn);
    }
    for (int k = 0; k < 4; ++k) {
        double qn = h->rot[k * n + node], qp = h->rot[k * n + pp];
        grad[(6 + k) * n + node] += w0 * dqraw[k];
        if (p >= 0) grad[(6 + k) * n + p] += w1 * dqraw[k];
        dt += dqraw[k] * (qp - qn);
    }
    for (int k = 0; k < 48; ++k) {
        double sn = h->sh[k * n + node], sp = h->sh[k * n + pp];
        grad[(11 + k) * n + node] += w0 * dsh[k];
        if (p >= 0) grad[(11 + k) * n + p] += w1 * dsh[k];
        dt += dsh[k] * (sp - sn);
    }
    /* o = |o_raw| */
    {
        double on = h->opacity[node];
        grad[10 * n + node] += (on > 0 ? 1.0 : (on < 0 ? -1.0 : 0.0)) * don;
        if (p >= 0) {
            double op = h->opacity[p];
            grad[10 * n + p] += (op > 0 ? 1.0 : (op < 0 ? -1.0 : 0.0)) * dop;
        }
    }
    if (dt_out) *dt_out = (p >= 0) ? dt : 0.0;
}

/* Gradient of L = sum over the listed pixels pix[npix] (linear indices
 * y*W + x) and channels of dL_drgb[k*3 + c] * rgb, i.e. the vector-Jacobian
 * product with a cotangent that is zero on every other pixel.
 * grad[OR_NPARAM * n] accumulates; dt[count] (optional) receives dL/dt for
 * each cut node; screen[count*11] (optional) receives the screen-space
 * adjoints du, dv, dconic(3), dA_n, dA_p, drgb(3), dt_alpha of each cut node
 * (A_n = kappa o_n, A_p = kappa o_p, dt_alpha = the part of dL/dt that flows
 * through alpha alone). */
void or_backward(const or_hier *h, const or_view *v, const int32_t *ids, const double *t, int64_t count,
                 const int64_t *pix, int64_t npix, const double *dL_drgb, double *grad, double *dt, double *screen)
{
    or_frame F;
    frame_build(h, v, ids, t, count, &F);
    or_lists L;
    lists_build(&F, v, pix, npix, &L);
    or_sgrad *sg = (or_sgrad *)calloc((size_t)(count > 0 ? count : 1), sizeof(or_sgrad));

    int32_t *inc = NULL;
    double *alph = NULL, *Tb = NULL;
    int64_t cap = 0;
    for (int64_t k = 0; k < npix; ++k) {
        const int px = (int)(pix[k] % v->width), py = (int)(pix[k] / v->width);
        const int32_t *items = L.items + L.start[k];
        const int64_t m = L.start[k + 1] - L.start[k];
        const double *gC = dL_drgb + 3 * k;
        if (m > cap) {
            cap = 2 * m;
            inc = (int32_t *)realloc(inc, sizeof(int32_t) * cap);
            alph = (double *)realloc(alph, sizeof(double) * cap);
            Tb = (double *)realloc(Tb, sizeof(double) * cap);
        }
        /* forward: record contributors, their alpha and the transmittance
         * in front of them */
        double T = 1.0;
        int64_t nc = 0;
        for (int64_t j = 0; j < m; ++j) {
            or_alpha_t a;
            splat_alpha(&F.splats[items[j]], px, py, &a);
            if (a.alpha < OR_ALPHA_MIN) continue;
            const double Tn = T * (1.0 - a.alpha);
            if (Tn < OR_T_MIN) break;
            inc[nc] = items[j];
            alph[nc] = a.alpha;
            Tb[nc] = T;
            nc++;
            T = Tn;
        }
        /* C = sum_i c_i alpha_i T_i,  T_{i+1} = T_i (1 - alpha_i):
         * dC/dc_i = alpha_i T_i,
         * dC/dalpha_i = T_i c_i - (sum_{j>i} c_j alpha_j T_j) / (1 - alpha_i) */
        double after[3] = {0, 0, 0};
        for (int64_t j = nc - 1; j >= 0; --j) {
            const or_splat *S = &F.splats[inc[j]];
            or_sgrad *G = &sg[inc[j]];
            const double al = alph[j], Ti = Tb[j];
            double dal = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                G->drgb[ch] += al * Ti * gC[ch];
                dal += (Ti * S->rgb[ch] - after[ch] / (1.0 - al)) * gC[ch];
            }
            for (int ch = 0; ch < 3; ++ch) after[ch] += S->rgb[ch] * al * Ti;
            /* alpha = (1-t) a_n + t (1 - (1 - a_p)^(1/K))  or a_n when t = 0 */
            or_alpha_t a;
            splat_alpha(S, px, py, &a);
            double dan, dap = 0.0;
            if (S->t > 0.0) {
                dan = (1.0 - S->t) * dal;
                const double dapr = S->t * dal;
                G->dt_alpha += (a.apr - a.an) * dal;
                dap = dapr * (1.0 / S->K) * pow(1.0 - a.ap, 1.0 / S->K - 1.0);
            } else {
                dan = dal;
            }
            /* a = min(0.99, A G): zero derivative where clamped */
            double dG = 0.0;
            if (!a.clamp_n) {
                G->dAn += dan * a.G;
                dG += dan * S->A_n;
            }
            if (S->t > 0.0 && !a.clamp_p) {
                G->dAp += dap * a.G;
                dG += dap * S->A_p;
            }
            /* G = exp(-Q/2), Q = ca dx^2 + 2 cb dx dy + cc dy^2, dx = px - u */
            const double dQ = -0.5 * a.G * dG;
            const double ddx = dQ * (2.0 * S->conic[0] * a.dx + 2.0 * S->conic[1] * a.dy);
            const double ddy = dQ * (2.0 * S->conic[1] * a.dx + 2.0 * S->conic[2] * a.dy);
            G->du -= ddx;
            G->dv -= ddy;
            G->dconic[0] += dQ * a.dx * a.dx;
            G->dconic[1] += dQ * 2.0 * a.dx * a.dy;
            G->dconic[2] += dQ * a.dy * a.dy;
        }
    }
    free(inc);
    free(alph);
    free(Tb);
    for (int64_t k = 0; k < count; ++k) splat_backward(h, v, &F.splats[k], &sg[k], grad, dt ? dt + k : NULL);
    if (screen)
        for (int64_t k = 0; k < count; ++k) {
            double *o = screen + 11 * k;
            o[0] = sg[k].du; o[1] = sg[k].dv;
            o[2] = sg[k].dconic[0]; o[3] = sg[k].dconic[1]; o[4] = sg[k].dconic[2];
            o[5] = sg[k].dAn; o[6] = sg[k].dAp;
            o[7] = sg[k].drgb[0]; o[8] = sg[k].drgb[1]; o[9] = sg[k].drgb[2];
            o[10] = sg[k].dt_alpha;
        }
    free(sg);
    lists_free(&L);
    frame_free(&F);
}


/* ---------------------------------------------------------------------- */
/* rounding budget of the gradient (test helper)                            */
/* ---------------------------------------------------------------------- */
/* A renderer that composites in FP32 (as the paper's rasteriser does) gets
 * every per-pixel term of the gradient with an error of a few units in the
 * last place of the quantities it is formed from, and the transmittance in
 * front of a splat, recovered over the pixel's list, with an error that
 * grows with the list: about one rounding per contributor in the forward
 * product and one in each backward division.  A gradient element that sums
 * many such terms of both signs can therefore be far smaller than the error
 * those terms carry.  or_backward_budget returns, per parameter element,
 *     B_e = sum over (pixel, splat) terms of (nc + 16) |term reaching e|,
 * nc = the pixel's contributor count: every factor of the chain of
 * or_backward taken in absolute value (a difference such as c - R counted
 * as |c| + |R|), and the per-splat map from screen-space adjoints to the
 * node and parent parameters taken column by column in absolute value
 * (splat_backward applied to each unit screen adjoint).  An FP32 result
 * then lies within about u B_e of the exact one (u = 2^-24 per rounding and
 * a small constant per step); the caller chooses the constant.  Same
 * arguments as or_backward; budget[OR_NPARAM * n] accumulates. */
static void unit_param_adjoint(const or_hier *h, const or_view *v, const or_splat *S, int k, double out[2][OR_NPARAM])
{
    /* the splat's node (slot 1) and parent (slot 0) copied into a two-node
     * hierarchy, so that splat_backward writes into a 2-column array */
    double mean[6], scale[6], rot[8], op[2], sh[96];
    int32_t par[2] = {-1, 0}, cb[2] = {1, 0}, cc[2] = {1, 0};
    double bmn[6] = {0}, bmx[6] = {0};
    const int64_t n = h->n;
    const int32_t node = S->node, p = S->parent, pp = p >= 0 ? p : node;
    for (int c = 0; c < 3; ++c) {
        mean[2 * c] = h->mean[c * n + pp]; mean[2 * c + 1] = h->mean[c * n + node];
        scale[2 * c] = h->scale[c * n + pp]; scale[2 * c + 1] = h->scale[c * n + node];
    }
    for (int c = 0; c < 4; ++c) { rot[2 * c] = h->rot[c * n + pp]; rot[2 * c + 1] = h->rot[c * n + node]; }
    op[0] = h->opacity[pp]; op[1] = h->opacity[node];
    for (int c = 0; c < 48; ++c) { sh[2 * c] = h->sh[c * n + pp]; sh[2 * c + 1] = h->sh[c * n + node]; }
    or_hier h2 = {2, par, cb, cc, bmn, bmx, mean, scale, rot, op, sh};
    or_splat S2 = *S;
    S2.node = 1;
    S2.parent = p >= 0 ? 0 : -1;
    or_sgrad g;
    memset(&g, 0, sizeof g);
    switch (k) {  /* the 11 adjoints in the order du, dv, dconic, dA_n, dA_p, drgb, dt_alpha */
    case 0: g.du = 1.0; break;
    case 1: g.dv = 1.0; break;
    case 2: case 3: case 4: g.dconic[k - 2] = 1.0; break;
    case 5: g.dAn = 1.0; break;
    case 6: g.dAp = 1.0; break;
    case 7: case 8: case 9: g.drgb[k - 7] = 1.0; break;
    default: g.dt_alpha = 1.0; break;
    }
    double tmp[OR_NPARAM * 2];
    memset(tmp, 0, sizeof tmp);
    splat_backward(&h2, v, &S2, &g, tmp, NULL);
    for (int q = 0; q < OR_NPARAM; ++q) {
        out[0][q] = tmp[q * 2 + 1];  /* node */
        out[1][q] = p >= 0 ? tmp[q * 2] : 0.0;
    }
}

void or_backward_budget(const or_hier *h, const or_view *v, const int32_t *ids, const double *t, int64_t count,
                        const int64_t *pix, int64_t npix, const double *dL_drgb, double *budget)
{
    or_frame F;
    frame_build(h, v, ids, t, count, &F);
    or_lists L;
    lists_build(&F, v, pix, npix, &L);
    double *m = (double *)calloc((size_t)(count > 0 ? count : 1) * 11, sizeof(double));
    int32_t *inc = NULL;
    double *alph = NULL, *Tb = NULL;
    int64_t cap = 0;
    for (int64_t k = 0; k < npix; ++k) {
        const int px = (int)(pix[k] % v->width), py = (int)(pix[k] / v->width);
        const int32_t *items = L.items + L.start[k];
        const int64_t mm = L.start[k + 1] - L.start[k];
        const double *gC = dL_drgb + 3 * k;
        if (mm > cap) {
            cap = 2 * mm;
            inc = (int32_t *)realloc(inc, sizeof(int32_t) * cap);
            alph = (double *)realloc(alph, sizeof(double) * cap);
            Tb = (double *)realloc(Tb, sizeof(double) * cap);
        }
        double T = 1.0;
        int64_t nc = 0;
        for (int64_t j = 0; j < mm; ++j) {
            or_alpha_t a;
            splat_alpha(&F.splats[items[j]], px, py, &a);
            if (a.alpha < OR_ALPHA_MIN) continue;
            const double Tn = T * (1.0 - a.alpha);
            if (Tn < OR_T_MIN) break;
            inc[nc] = items[j];
            alph[nc] = a.alpha;
            Tb[nc] = T;
            nc++;
            T = Tn;
        }
        const double wgt = (double)(nc + 16);
        double after[3] = {0, 0, 0};
        for (int64_t j = nc - 1; j >= 0; --j) {
            const or_splat *S = &F.splats[inc[j]];
            double *M = m + 11 * (int64_t)inc[j];
            const double al = alph[j], Ti = Tb[j];
            double dal = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                M[7 + ch] += wgt * fabs(al * Ti * gC[ch]);
                dal += (Ti * S->rgb[ch] + fabs(after[ch]) / (1.0 - al)) * fabs(gC[ch]);
            }
            for (int ch = 0; ch < 3; ++ch) after[ch] += S->rgb[ch] * al * Ti;
            or_alpha_t a;
            splat_alpha(S, px, py, &a);
            double dan, dap = 0.0;
            if (S->t > 0.0) {
                dan = (1.0 - S->t) * dal;
                M[10] += wgt * (fabs(a.apr) + fabs(a.an)) * dal;
                dap = S->t * dal * (1.0 / S->K) * pow(1.0 - a.ap, 1.0 / S->K - 1.0);
            } else {
                dan = dal;
            }
            double dG = 0.0;
            if (!a.clamp_n) {
                M[5] += wgt * dan * a.G;
                dG += dan * S->A_n;
            }
            if (S->t > 0.0 && !a.clamp_p) {
                M[6] += wgt * dap * a.G;
                dG += dap * S->A_p;
            }
            const double dQ = 0.5 * a.G * dG;
            M[0] += wgt * dQ * (2.0 * fabs(S->conic[0] * a.dx) + 2.0 * fabs(S->conic[1] * a.dy));
            M[1] += wgt * dQ * (2.0 * fabs(S->conic[1] * a.dx) + 2.0 * fabs(S->conic[2] * a.dy));
            M[2] += wgt * dQ * a.dx * a.dx;
            M[3] += wgt * dQ * 2.0 * fabs(a.dx * a.dy);
            M[4] += wgt * dQ * a.dy * a.dy;
        }
    }
    free(inc);
    free(alph);
    free(Tb);
    const int64_t n = h->n;
    for (int64_t s = 0; s < count; ++s) {
        const or_splat *S = &F.splats[s];
        if (!S->valid) continue;
        const double *M = m + 11 * s;
        for (int k = 0; k < 11; ++k) {
            if (M[k] == 0.0) continue;
            double col[2][OR_NPARAM];
            unit_param_adjoint(h, v, S, k, col);
            for (int q = 0; q < OR_NPARAM; ++q) {
                budget[(int64_t)q * n + S->node] += M[k] * fabs(col[0][q]);
                if (S->parent >= 0) budget[(int64_t)q * n + S->parent] += M[k] * fabs(col[1][q]);
            }
        }
    }
    free(m);
    lists_free(&L);
    frame_free(&F);
}
