// Optimiser step of the hierarchy optimisation (Sec. 5.1): Adam on the
// interior nodes, leaves unchanged.  HBM-bound: per interior node and
// parameter group the parameter, gradient and both moments are read once
// and written once (the gradient as zero).
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;

// One thread per (interior node, run of CH consecutive components) of a
// group with COMP components per node.
template <int COMP, int CH>
__global__ __launch_bounds__(kT) void k_adam(const int32_t *__restrict__ interior, int64_t n_interior,
                                             float *__restrict__ p, float *__restrict__ g, float *__restrict__ m,
                                             float *__restrict__ v, AdamScalars s)
{
    static_assert(COMP % CH == 0, "runs tile the group");
    constexpr int RUNS = COMP / CH;
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= n_interior * RUNS) return;
    const int64_t q = e / RUNS;
    const int r = (int)(e - q * RUNS);
    const int64_t k0 = (int64_t)interior[q] * COMP + r * CH;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int64_t k = k0 + c;
        const float gk = g[k];
        const float mk = s.beta1 * m[k] + (1.0f - s.beta1) * gk;
        const float vk = s.beta2 * v[k] + (1.0f - s.beta2) * gk * gk;
        m[k] = mk;
        v[k] = vk;
        p[k] -= s.lr * (mk * s.bc1) / (sqrtf(vk * s.bc2) + s.eps);
        g[k] = 0.0f;
    }
}

template <int COMP, int CH>
void launch_adam_t(const int32_t *interior, int64_t n_interior, float *p, float *g, float *m, float *v,
                   const AdamScalars &s, hipStream_t st)
{
    const int64_t n = n_interior * (COMP / CH);
    if (n <= 0) return;
    hipLaunchKernelGGL((k_adam<COMP, CH>), dim3((uint32_t)((n + kT - 1) / kT)), dim3(kT), 0, st, interior, n_interior,
                       p, g, m, v, s);
}

}  // namespace

void launch_adam(int group, const int32_t *interior, int64_t n_interior, float *p, float *g, float *m, float *v,
                 const AdamScalars &s, hipStream_t st)
{
    switch (group) {
    case 0:
    case 1: launch_adam_t<3, 3>(interior, n_interior, p, g, m, v, s, st); break;  // mean, scale
    case 2: launch_adam_t<4, 4>(interior, n_interior, p, g, m, v, s, st); break;  // rotation
    case 3: launch_adam_t<1, 1>(interior, n_interior, p, g, m, v, s, st); break;  // opacity
    default: launch_adam_t<48, 4>(interior, n_interior, p, g, m, v, s, st); break;  // SH
    }
}

}  // namespace hgs
