// Optimiser step of the hierarchy optimisation (Sec. 5.1): Adam on the
// interior nodes, leaves unchanged.  HBM-bound: per interior node and
// parameter group the parameter, gradient and both moments are read once
// and written once (the gradient as zero).  The moments are stored by
// interior rank (row q belongs to the q-th interior node in ascending id
// order), so that they stream contiguously; parameter and gradient rows are
// reached through the interior list, in 16-byte vectors where the group's
// row allows it.
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;

// One thread per element of a group with COMP components per node (the
// rows of the moments are contiguous, element e = q COMP + c).
template <int COMP>
__global__ __launch_bounds__(kT) void k_adam_scalar(const int32_t *__restrict__ interior, int64_t n_interior,
                                                    float *__restrict__ p, float *__restrict__ g,
                                                    float *__restrict__ m, float *__restrict__ v, AdamScalars s)
{
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n_interior * COMP) return;
    const int64_t q = e / COMP;
    const int c = (int)(e - q * COMP);
    const int64_t k = (int64_t)interior[q] * COMP + c;
    float pk = p[k], mk = m[e], vk = v[e];
    adam_one(pk, g[k], mk, vk, s);
    p[k] = pk;
    g[k] = 0.0f;
    m[e] = mk;
    v[e] = vk;
}

// One thread per 4 consecutive components of a group with COMP (a multiple
// of 4) components per node: 16-byte loads and stores of every array.
template <int COMP>
__global__ __launch_bounds__(kT) void k_adam_vec4(const int32_t *__restrict__ interior, int64_t n_interior,
                                                  float4 *__restrict__ p, float4 *__restrict__ g,
                                                  float4 *__restrict__ m, float4 *__restrict__ v, AdamScalars s)
{
    static_assert(COMP % 4 == 0, "vector rows");
    constexpr int R = COMP / 4;
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n_interior * R) return;
    const int64_t q = e / R;
    const int c = (int)(e - q * R);
    const int64_t k = (int64_t)interior[q] * R + c;
    float4 pk = p[k], mk = m[e], vk = v[e];
    const float4 gk = g[k];
    adam_one(pk.x, gk.x, mk.x, vk.x, s);
    adam_one(pk.y, gk.y, mk.y, vk.y, s);
    adam_one(pk.z, gk.z, mk.z, vk.z, s);
    adam_one(pk.w, gk.w, mk.w, vk.w, s);
    p[k] = pk;
    g[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    m[e] = mk;
    v[e] = vk;
}

template <int COMP>
void launch_adam_t(const int32_t *interior, int64_t n_interior, float *p, float *g, float *m, float *v,
                   const AdamScalars &s, hipStream_t st)
{
    if (n_interior <= 0) return;
    if constexpr (COMP % 4 == 0) {
        const int64_t n = n_interior * (COMP / 4);
        hipLaunchKernelGGL((k_adam_vec4<COMP>), dim3((uint32_t)((n + kT - 1) / kT)), dim3(kT), 0, st, interior,
                           n_interior, reinterpret_cast<float4 *>(p), reinterpret_cast<float4 *>(g),
                           reinterpret_cast<float4 *>(m), reinterpret_cast<float4 *>(v), s);
    } else {
        const int64_t n = n_interior * COMP;
        hipLaunchKernelGGL((k_adam_scalar<COMP>), dim3((uint32_t)((n + kT - 1) / kT)), dim3(kT), 0, st, interior,
                           n_interior, p, g, m, v, s);
    }
}

}  // namespace

void launch_adam(int group, const int32_t *interior, int64_t n_interior, float *p, float *g, float *m, float *v,
                 const AdamScalars &s, hipStream_t st)
{
    switch (group) {
    case 0:
    case 1: launch_adam_t<3>(interior, n_interior, p, g, m, v, s, st); break;  // mean, scale
    case 2: launch_adam_t<4>(interior, n_interior, p, g, m, v, s, st); break;  // rotation
    case 3: launch_adam_t<1>(interior, n_interior, p, g, m, v, s, st); break;  // opacity
    default: launch_adam_t<48>(interior, n_interior, p, g, m, v, s, st); break;  // SH
    }
}

}  // namespace hgs
