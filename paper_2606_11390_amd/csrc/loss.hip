// L2 image loss and its gradient (gfx950).
//
// Paper Section 4: after rasterising a camera the image-space loss is
// evaluated per camera.  loss = mean((img - target)^2) over every packed image
// element; d_img = 2 (img - target) / n.  The sum is reduced in a fixed order
// (per-block partials in double, then one block) so the loss is deterministic.
#include "gs_device.h"

namespace gs {
namespace {

constexpr int L_THREADS = 256;

__global__ __launch_bounds__(L_THREADS) void k_l2_partial(const float* __restrict__ img,
                                                          const float* __restrict__ tgt,
                                                          long long n, float scale,
                                                          float* __restrict__ dimg,
                                                          double* __restrict__ part)
{
    __shared__ double s_w[L_THREADS / GS_WAVE];
    const long long stride = (long long)gridDim.x * L_THREADS;
    float acc = 0.0f;
    for (long long i = (long long)blockIdx.x * L_THREADS + threadIdx.x; i < n; i += stride) {
        const float d = img[i] - tgt[i];
        nt_store(scale * d, &dimg[i]);
        acc = __builtin_fmaf(d, d, acc);
    }
    const float ws = wave_sum(acc);
    if (__lane_id() == 0) s_w[threadIdx.x / GS_WAVE] = (double)ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < L_THREADS / GS_WAVE; i++) s += s_w[i];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(L_THREADS) void k_l2_final(const double* __restrict__ part, int nb,
                                                        double inv_n, float* __restrict__ loss)
{
    __shared__ double s[L_THREADS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += L_THREADS) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = L_THREADS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(s[0] * inv_n);
}

int loss_blocks(long long n)
{
    long long nb = (n + L_THREADS * 16 - 1) / (L_THREADS * 16);
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    return (int)nb;
}

}  // namespace

size_t loss_workspace_size(long long n) { return sizeof(double) * (size_t)loss_blocks(n); }

hipError_t launch_loss_l2(const float* img, const float* tgt, long long n, float* loss, float* dimg,
                          void* ws, hipStream_t st)
{
    const int nb = loss_blocks(n);
    hipLaunchKernelGGL(k_l2_partial, dim3(nb), dim3(L_THREADS), 0, st, img, tgt, n,
                       n > 0 ? (float)(2.0 / (double)n) : 0.0f, dimg, (double*)ws);
    hipLaunchKernelGGL(k_l2_final, dim3(1), dim3(L_THREADS), 0, st, (const double*)ws, nb,
                       n > 0 ? 1.0 / (double)n : 0.0, loss);
    return hipGetLastError();
}

}  // namespace gs
