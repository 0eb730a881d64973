// Per-splat forward projection in FP64, shared by the preprocess kernel and
// its backward (which recomputes it instead of storing intermediates).
//
// For a cut node n with parent p and weight t (the parent's weight, Eq.
// (t_interp) read so that t = 1 renders n as its parent):
//   interpolation (Sec. 4.2): mu~ - eye = (mu_n - eye) + t (mu_p - mu_n);
//     s~ = (1-t) s_n + t s_p; q~ = normalise((1-t) q_n + t q_p);
//     SH~ = (1-t) SH_n + t SH_p; |o_n| and |o_p| are kept apart for the
//     opacity transition of Eq. (alphap).
//   projection (Sec. 3): p = R (mu~ - eye); Sigma3 = Rq diag(s~^2) Rq^T;
//     J = d(u, v)/d(p); Sigma2 = (J R) Sigma3 (J R)^T.
//   anti-aliasing (Sec. 5.1, EWA filtering): Sigma2' = Sigma2 + h I with
//     opacity compensation kappa = sqrt(det Sigma2 / det Sigma2').
//   colour: max(0, SH~ . Y(dir) + 1/2), dir = normalise(mu~ - eye), Y the
//     real orthonormal SH basis of degree 3.
#pragma once

#include "hgs_internal.h"

namespace hgs {

// Real orthonormal SH basis, degree <= 3, index l*l + l + m, at a unit vector.
__device__ __forceinline__ void sh_eval(double x, double y, double z, double Y[16])
{
    const double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814;
    Y[1] = 0.4886025119029199 * y;
    Y[2] = 0.4886025119029199 * z;
    Y[3] = 0.4886025119029199 * x;
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = 1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (3.0 * zz - 1.0);
    Y[7] = 1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (xx - yy);
    Y[9] = 0.5900435899266435 * y * (3.0 * xx - yy);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = 0.4570457994644658 * y * (5.0 * zz - 1.0);
    Y[12] = 0.3731763325901154 * z * (5.0 * zz - 3.0);
    Y[13] = 0.4570457994644658 * x * (5.0 * zz - 1.0);
    Y[14] = 1.445305721320277 * z * (xx - yy);
    Y[15] = 0.5900435899266435 * x * (xx - 3.0 * yy);
}

// sum_k B[k] * grad Y_k(x, y, z): the gradient of the basis polynomials
// contracted with per-function weights.
__device__ __forceinline__ void sh_grad_dot(double x, double y, double z, const double B[16], double g[3])
{
    const double xx = x * x, yy = y * y, zz = z * z;
    const double c1 = 0.4886025119029199, c2 = 1.0925484305920792, c20 = 0.31539156525252005;
    const double c22 = 0.5462742152960396, c9 = 0.5900435899266435, c10 = 2.890611442640554;
    const double c11 = 0.4570457994644658, c12 = 0.3731763325901154, c14 = 1.445305721320277;
    g[0] = c1 * B[3] + c2 * (y * B[4] + z * B[7]) + c22 * 2.0 * x * B[8] + c9 * 6.0 * x * y * B[9] +
           c10 * y * z * B[10] + c11 * (5.0 * zz - 1.0) * B[13] + c14 * 2.0 * x * z * B[14] +
           c9 * (3.0 * xx - 3.0 * yy) * B[15];
    g[1] = c1 * B[1] + c2 * (x * B[4] + z * B[5]) - c22 * 2.0 * y * B[8] + c9 * (3.0 * xx - 3.0 * yy) * B[9] +
           c10 * x * z * B[10] + c11 * (5.0 * zz - 1.0) * B[11] - c14 * 2.0 * y * z * B[14] -
           c9 * 6.0 * x * y * B[15];
    g[2] = c1 * B[2] + c2 * (y * B[5] + x * B[7]) + c20 * 6.0 * z * B[6] + c10 * x * y * B[10] +
           c11 * 10.0 * y * z * B[11] + c12 * (15.0 * zz - 3.0) * B[12] + c11 * 10.0 * x * z * B[13] +
           c14 * (xx - yy) * B[14];
}

// Basis function k (compile-time after unrolling) and its polynomial gradient.
__device__ __forceinline__ void sh_term(int k, double x, double y, double z, double &Y, double g[3])
{
    const double xx = x * x, yy = y * y, zz = z * z;
    g[0] = g[1] = g[2] = 0.0;
    switch (k) {
    case 0: Y = 0.28209479177387814; break;
    case 1: Y = 0.4886025119029199 * y; g[1] = 0.4886025119029199; break;
    case 2: Y = 0.4886025119029199 * z; g[2] = 0.4886025119029199; break;
    case 3: Y = 0.4886025119029199 * x; g[0] = 0.4886025119029199; break;
    case 4: Y = 1.0925484305920792 * x * y; g[0] = 1.0925484305920792 * y; g[1] = 1.0925484305920792 * x; break;
    case 5: Y = 1.0925484305920792 * y * z; g[1] = 1.0925484305920792 * z; g[2] = 1.0925484305920792 * y; break;
    case 6: Y = 0.31539156525252005 * (3.0 * zz - 1.0); g[2] = 0.31539156525252005 * 6.0 * z; break;
    case 7: Y = 1.0925484305920792 * x * z; g[0] = 1.0925484305920792 * z; g[2] = 1.0925484305920792 * x; break;
    case 8:
        Y = 0.5462742152960396 * (xx - yy);
        g[0] = 0.5462742152960396 * 2.0 * x;
        g[1] = -0.5462742152960396 * 2.0 * y;
        break;
    case 9:
        Y = 0.5900435899266435 * y * (3.0 * xx - yy);
        g[0] = 0.5900435899266435 * 6.0 * x * y;
        g[1] = 0.5900435899266435 * (3.0 * xx - 3.0 * yy);
        break;
    case 10:
        Y = 2.890611442640554 * x * y * z;
        g[0] = 2.890611442640554 * y * z;
        g[1] = 2.890611442640554 * x * z;
        g[2] = 2.890611442640554 * x * y;
        break;
    case 11:
        Y = 0.4570457994644658 * y * (5.0 * zz - 1.0);
        g[1] = 0.4570457994644658 * (5.0 * zz - 1.0);
        g[2] = 0.4570457994644658 * 10.0 * y * z;
        break;
    case 12:
        Y = 0.3731763325901154 * z * (5.0 * zz - 3.0);
        g[2] = 0.3731763325901154 * (15.0 * zz - 3.0);
        break;
    case 13:
        Y = 0.4570457994644658 * x * (5.0 * zz - 1.0);
        g[0] = 0.4570457994644658 * (5.0 * zz - 1.0);
        g[2] = 0.4570457994644658 * 10.0 * x * z;
        break;
    case 14:
        Y = 1.445305721320277 * z * (xx - yy);
        g[0] = 1.445305721320277 * 2.0 * x * z;
        g[1] = -1.445305721320277 * 2.0 * y * z;
        g[2] = 1.445305721320277 * (xx - yy);
        break;
    default:
        Y = 0.5900435899266435 * x * (xx - 3.0 * yy);
        g[0] = 0.5900435899266435 * (3.0 * xx - 3.0 * yy);
        g[1] = -0.5900435899266435 * 6.0 * x * y;
        break;
    }
}

__device__ __forceinline__ void quat_rot(const double q[4], double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

struct Proj {
    uint32_t node, par;
    bool has_par;
    int K;
    double t;
    double mu_rel[3], s[3], qraw[4], q[4], qlen;
    double o_n, o_p, on_raw, op_raw;
    double pc[3];
    double Tm[6];
    double cov3[6];  // xx xy xz yy yz zz
    double a, b, c;  // Sigma2
    double D, Dd, kappa, conic[3];
    double u, v;
    double dir[3], rlen;
    double raw[3];
    double dcol[3][3];  // d raw colour / d dir (polynomial gradient, before normalisation)
    double dpn[3];      // (SH_p - SH_n) . Y(dir), per channel
    bool front, ok;
};

// Gathers node and parent, interpolates, projects; computes the colour only
// when with_colour (the backward recomputes it on the fly).
__device__ __forceinline__ void project_splat(const DevHier &h, const DevView &V, uint32_t node, double t_in,
                                              Proj &P, bool with_colour)
{
    const int64_t n = h.n;
    P.node = node;
    const uint32_t pi = h.pinfo[node];
    const uint32_t par = pi & ~kLeafBit;
    P.has_par = par != kRootParent;
    P.t = P.has_par ? t_in : 0.0;
    const bool use_par = P.has_par && P.t > 0.0;
    P.par = P.has_par ? par : node;
    P.K = P.has_par ? h.child_count[par] : 1;
    const uint32_t src = use_par ? par : node;
    const double t = P.t, w0 = 1.0 - t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double mn = h.mean[k * n + node];
        const double mp = use_par ? (double)h.mean[k * n + src] : mn;
        P.mu_rel[k] = (mn - (double)V.eye[k]) + t * (mp - mn);
        const double sn = h.scale[k * n + node];
        const double sp = use_par ? (double)h.scale[k * n + src] : sn;
        P.s[k] = w0 * sn + t * sp;
    }
    double ql = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double qn = h.rot[k * n + node];
        const double qp = use_par ? (double)h.rot[k * n + src] : qn;
        P.qraw[k] = w0 * qn + t * qp;
        ql += P.qraw[k] * P.qraw[k];
    }
    P.qlen = sqrt(ql);
#pragma unroll
    for (int k = 0; k < 4; ++k) P.q[k] = P.qraw[k] / P.qlen;
    P.on_raw = h.opacity[node];
    P.op_raw = P.has_par ? (double)h.opacity[par] : 0.0;
    P.o_n = fabs(P.on_raw);
    P.o_p = use_par ? fabs(P.op_raw) : 0.0;

#pragma unroll
    for (int r = 0; r < 3; ++r)
        P.pc[r] = (double)V.R[3 * r] * P.mu_rel[0] + (double)V.R[3 * r + 1] * P.mu_rel[1] +
                  (double)V.R[3 * r + 2] * P.mu_rel[2];
    P.front = P.pc[2] > (double)V.z_near;
    P.ok = false;
    if (!P.front) return;
    const double x = P.pc[0], y = P.pc[1], z = P.pc[2];
    const double fx = V.fx, fy = V.fy;
    double Rq[9];
    quat_rot(P.q, Rq);
    double M[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * P.s[c];
    P.cov3[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    P.cov3[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    P.cov3[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    P.cov3[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    P.cov3[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    P.cov3[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    const double iz = 1.0 / z;
    const double J00 = fx * iz, J02 = -fx * x * iz * iz, J11 = fy * iz, J12 = -fy * y * iz * iz;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        P.Tm[c] = J00 * (double)V.R[c] + J02 * (double)V.R[6 + c];
        P.Tm[3 + c] = J11 * (double)V.R[3 + c] + J12 * (double)V.R[6 + c];
    }
    const double *S = P.cov3;
    // rows of Tm times Sigma3
    double A0[3], A1[3];
    A0[0] = P.Tm[0] * S[0] + P.Tm[1] * S[1] + P.Tm[2] * S[2];
    A0[1] = P.Tm[0] * S[1] + P.Tm[1] * S[3] + P.Tm[2] * S[4];
    A0[2] = P.Tm[0] * S[2] + P.Tm[1] * S[4] + P.Tm[2] * S[5];
    A1[0] = P.Tm[3] * S[0] + P.Tm[4] * S[1] + P.Tm[5] * S[2];
    A1[1] = P.Tm[3] * S[1] + P.Tm[4] * S[3] + P.Tm[5] * S[4];
    A1[2] = P.Tm[3] * S[2] + P.Tm[4] * S[4] + P.Tm[5] * S[5];
    P.a = A0[0] * P.Tm[0] + A0[1] * P.Tm[1] + A0[2] * P.Tm[2];
    P.b = A0[0] * P.Tm[3] + A0[1] * P.Tm[4] + A0[2] * P.Tm[5];
    P.c = A1[0] * P.Tm[3] + A1[1] * P.Tm[4] + A1[2] * P.Tm[5];
    const double ad = P.a + kDilation, cd = P.c + kDilation;
    P.D = P.a * P.c - P.b * P.b;
    P.Dd = ad * cd - P.b * P.b;
    if (!(P.Dd > 0.0)) return;
    P.kappa = P.D > 0.0 ? sqrt(P.D / P.Dd) : 0.0;
    P.conic[0] = cd / P.Dd;
    P.conic[1] = -P.b / P.Dd;
    P.conic[2] = ad / P.Dd;
    P.u = fx * x * iz + (double)V.cx;
    P.v = fy * y * iz + (double)V.cy;
    P.rlen = sqrt(P.mu_rel[0] * P.mu_rel[0] + P.mu_rel[1] * P.mu_rel[1] + P.mu_rel[2] * P.mu_rel[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) P.dir[k] = P.mu_rel[k] / P.rlen;
    if (with_colour) {
        double acc[3] = {0.5, 0.5, 0.5};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            P.dpn[ch] = 0.0;
            P.dcol[ch][0] = P.dcol[ch][1] = P.dcol[ch][2] = 0.0;
        }
        // SH~ row 3k + c; interpolate while accumulating colour, its gradient
        // in the direction, and the parent - node difference
#pragma unroll 1
        for (int k = 0; k < 16; ++k) {
            double Yk, gk[3];
            sh_term(k, P.dir[0], P.dir[1], P.dir[2], Yk, gk);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const double cn = h.sh[(3 * k + ch) * n + node];
                const double cp = use_par ? (double)h.sh[(3 * k + ch) * n + src] : cn;
                const double sht = w0 * cn + t * cp;
                acc[ch] += sht * Yk;
                P.dpn[ch] += (cp - cn) * Yk;
                P.dcol[ch][0] += sht * gk[0];
                P.dcol[ch][1] += sht * gk[1];
                P.dcol[ch][2] += sht * gk[2];
            }
        }
        P.raw[0] = acc[0];
        P.raw[1] = acc[1];
        P.raw[2] = acc[2];
    }
    P.ok = true;
}

}  // namespace hgs
