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

// FP32 versions for the forward colour (stored in FP32 afterwards).
__device__ __forceinline__ void sh_eval_f(float x, float y, float z, float Y[16])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[0] = 0.28209479177387814f;
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.0f * zz - 1.0f);
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (xx - yy);
    Y[9] = 0.5900435899266435f * y * (3.0f * xx - yy);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = 0.4570457994644658f * y * (5.0f * zz - 1.0f);
    Y[12] = 0.3731763325901154f * z * (5.0f * zz - 3.0f);
    Y[13] = 0.4570457994644658f * x * (5.0f * zz - 1.0f);
    Y[14] = 1.445305721320277f * z * (xx - yy);
    Y[15] = 0.5900435899266435f * x * (xx - 3.0f * yy);
}

__device__ __forceinline__ void sh_grad_dot_f(float x, float y, float z, const float B[16], float g[3])
{
    const float xx = x * x, yy = y * y, zz = z * z;
    const float c1 = 0.4886025119029199f, c2 = 1.0925484305920792f, c20 = 0.31539156525252005f;
    const float c22 = 0.5462742152960396f, c9 = 0.5900435899266435f, c10 = 2.890611442640554f;
    const float c11 = 0.4570457994644658f, c12 = 0.3731763325901154f, c14 = 1.445305721320277f;
    g[0] = c1 * B[3] + c2 * (y * B[4] + z * B[7]) + c22 * 2.0f * x * B[8] + c9 * 6.0f * x * y * B[9] +
           c10 * y * z * B[10] + c11 * (5.0f * zz - 1.0f) * B[13] + c14 * 2.0f * x * z * B[14] +
           c9 * (3.0f * xx - 3.0f * yy) * B[15];
    g[1] = c1 * B[1] + c2 * (x * B[4] + z * B[5]) - c22 * 2.0f * y * B[8] + c9 * (3.0f * xx - 3.0f * yy) * B[9] +
           c10 * x * z * B[10] + c11 * (5.0f * zz - 1.0f) * B[11] - c14 * 2.0f * y * z * B[14] -
           c9 * 6.0f * x * y * B[15];
    g[2] = c1 * B[2] + c2 * (y * B[5] + x * B[7]) + c20 * 6.0f * z * B[6] + c10 * x * y * B[10] +
           c11 * 10.0f * y * z * B[11] + c12 * (15.0f * zz - 3.0f) * B[12] + c11 * 10.0f * x * z * B[13] +
           c14 * (xx - yy) * B[14];
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
    size_t pn, pp;  // parameter indices of node and parent (cache slots out of core)
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
    bool use_par;
    bool front, ok;
};

// Gathers node and parent, interpolates and projects (geometry only; the
// colour is splat_colour's).
__device__ __forceinline__ void project_splat(const DevHier &h, const DevView &V, uint32_t node, double t_in,
                                              Proj &P)
{
    P.node = node;
    const uint32_t pi = h.pinfo[node];
    const uint32_t par = pi & ~kLeafBit;
    P.has_par = par != kRootParent;
    P.t = P.has_par ? t_in : 0.0;
    const bool use_par = P.has_par && P.t > 0.0;
    P.use_par = use_par;
    P.par = P.has_par ? par : node;
    P.K = P.has_par ? h.child_count[par] : 1;
    const uint32_t src = use_par ? par : node;  // the node itself when t = 0: same values
    // parameter records: by node id, or by cache slot out of core (a node or
    // parent that is not resident leaves the splat out)
    P.pn = param_index(h, node);
    P.pp = P.has_par ? param_index(h, par) : P.pn;
    P.front = false;
    P.ok = false;
    if (h.slot && ((int64_t)P.pn < 0 || (int64_t)P.pp < 0)) return;
    const size_t in = P.pn, is = use_par ? P.pp : P.pn;
    const double t = P.t, w0 = 1.0 - t;
    // node-major records: one vector load per attribute
    const float3 mn3 = *reinterpret_cast<const float3 *>(h.mean + 3 * in);
    const float3 mp3 = *reinterpret_cast<const float3 *>(h.mean + 3 * is);
    const float3 sn3 = *reinterpret_cast<const float3 *>(h.scale + 3 * in);
    const float3 sp3 = *reinterpret_cast<const float3 *>(h.scale + 3 * is);
    const float4 qn4 = *reinterpret_cast<const float4 *>(h.rot + 4 * in);
    const float4 qp4 = *reinterpret_cast<const float4 *>(h.rot + 4 * is);
    const float mn[3] = {mn3.x, mn3.y, mn3.z}, mp[3] = {mp3.x, mp3.y, mp3.z};
    const float sn[3] = {sn3.x, sn3.y, sn3.z}, sp[3] = {sp3.x, sp3.y, sp3.z};
    const float qn[4] = {qn4.x, qn4.y, qn4.z, qn4.w}, qp[4] = {qp4.x, qp4.y, qp4.z, qp4.w};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P.mu_rel[k] = ((double)mn[k] - (double)V.eye[k]) + t * ((double)mp[k] - (double)mn[k]);
        P.s[k] = w0 * (double)sn[k] + t * (double)sp[k];
    }
    double ql = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        P.qraw[k] = w0 * (double)qn[k] + t * (double)qp[k];
        ql += P.qraw[k] * P.qraw[k];
    }
    P.qlen = sqrt(ql);
#pragma unroll
    for (int k = 0; k < 4; ++k) P.q[k] = P.qraw[k] / P.qlen;
    P.on_raw = h.opacity[in];
    P.op_raw = P.has_par ? (double)h.opacity[P.pp] : 0.0;
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
    P.ok = true;
}

// Colour of the interpolated SH (FP32): per channel raw = SH~ . Y(dir) + 1/2,
// dcol = sum_k SH~_k grad Y_k(dir) (the polynomial gradient, before the
// normalisation of dir) and dpn = (SH_p - SH_n) . Y(dir), the derivative of
// raw in t.
__device__ __forceinline__ void splat_colour(const DevHier &h, const Proj &P, float raw[3], float dcol[3][3],
                                             float dpn[3])
{
    const float x = (float)P.dir[0], y = (float)P.dir[1], z = (float)P.dir[2];
    const float t = (float)P.t, w0 = 1.0f - t;
    // 48 coefficients per node, 192 B: twelve 16-byte loads per record
    const float4 *a4 = reinterpret_cast<const float4 *>(h.sh + (size_t)48 * P.pn);
    const float4 *b4 = reinterpret_cast<const float4 *>(h.sh + (size_t)48 * (P.use_par ? P.pp : P.pn));
    float Y[16];
    sh_eval_f(x, y, z, Y);
    float sht[48];
    float acc[3] = {0.5f, 0.5f, 0.5f}, dp[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q4 = 0; q4 < 12; ++q4) {
        const float4 cn4 = a4[q4], cp4 = b4[q4];
        const float cn[4] = {cn4.x, cn4.y, cn4.z, cn4.w}, cp[4] = {cp4.x, cp4.y, cp4.z, cp4.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int q = 4 * q4 + e, k = q / 3, ch = q % 3;  // coefficient 3 k + ch
            sht[q] = w0 * cn[e] + t * cp[e];
            acc[ch] += sht[q] * Y[k];
            dp[ch] += (cp[e] - cn[e]) * Y[k];
        }
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float c[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) c[k] = sht[3 * k + ch];
        raw[ch] = acc[ch];
        dpn[ch] = dp[ch];
        sh_grad_dot_f(x, y, z, c, dcol[ch]);
    }
}

}  // namespace hgs
