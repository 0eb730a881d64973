// Loss of the hierarchy optimisation (Sec. 5.1 optimises the hierarchy's
// interior nodes against the training images; the loss used here is the
// L1 distance, the image term of 3D Gaussian Splatting's loss): for the
// views of one render,
//   loss = (1 / M) sum over views, pixels and channels |C - C*|,
//   dL/dC = sign(C - C*) / M  (sign(0) = 0),
// with M the number of image values.  HBM-bound: per pixel it reads the
// image and the target and writes the cotangent (36 B).  The sum runs in
// FP64 over fixed per-block partials and one final block, so that it does
// not depend on scheduling.
#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int view_of_pixel(const DevView *views, int nv, uint32_t g)
{
    int lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_base <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kT) void k_l1(const DevView *__restrict__ views, int nv, uint32_t n_pix, double inv_m,
                                           double *__restrict__ partial)
{
    __shared__ double s_w[kT / 64];
    double acc = 0.0;
    for (uint32_t g = blockIdx.x * kT + threadIdx.x; g < n_pix; g += gridDim.x * kT) {
        const DevView &V = views[view_of_pixel(views, nv, g)];
        const size_t p = (size_t)(g - V.pix_base) * 3;
        float *dl = const_cast<float *>(V.dL);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float d = V.out_rgb[p + c] - V.target[p + c];
            acc += fabs((double)d);
            dl[p + c] = d > 0.0f ? (float)inv_m : (d < 0.0f ? -(float)inv_m : 0.0f);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kT / 64; ++w) t += s_w[w];
        partial[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kT) void k_l1_final(const double *__restrict__ partial, int n, double inv_m,
                                                 double *__restrict__ loss)
{
    __shared__ double s_w[kT / 64];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kT) acc += partial[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kT / 64; ++w) t += s_w[w];
        *loss = t * inv_m;
    }
}

}  // namespace

void launch_l1(const DevView *views, int nv, uint32_t n_pix, double *partial, double *loss, hipStream_t st)
{
    const uint64_t m = (uint64_t)n_pix * 3;
    const double inv_m = m ? 1.0 / (double)m : 0.0;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(((uint64_t)n_pix + kT - 1) / kT, kL1Blocks);
    if (blocks == 0) return;
    hipLaunchKernelGGL(k_l1, dim3(blocks), dim3(kT), 0, st, views, nv, n_pix, inv_m, partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kT), 0, st, partial, (int)blocks, inv_m, loss);
}

}  // namespace hgs
