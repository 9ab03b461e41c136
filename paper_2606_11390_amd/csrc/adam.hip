// Fused Adam over the Gaussian parameter tensors (gfx950).
//
// Paper Section 3.2 describes the multi-GPU fused Adam of its backend
// (vectorised loads and stores, transcendentals computed once); the update
// itself is Adam (Kingma and Ba 2015) with bias correction:
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   p <- p - lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
// One launch updates up to GS_ADAM_MAX_TENSORS tensors: the grid walks their
// concatenated 16-byte chunks (one HBM read of p, g, m, v and one write of p,
// m, v per element: 28 bytes, the algorithmic minimum).  The step count t is
// read from device memory and advanced by a one-thread kernel afterwards, so
// a captured graph replays successive steps correctly.
#include "gs_device.h"

namespace gs {
namespace {

struct AdamList {
    float* p[GS_ADAM_MAX_TENSORS];
    const float* g[GS_ADAM_MAX_TENSORS];
    float* m[GS_ADAM_MAX_TENSORS];
    float* v[GS_ADAM_MAX_TENSORS];
    long long n[GS_ADAM_MAX_TENSORS];
    long long chunk_off[GS_ADAM_MAX_TENSORS + 1];   // prefix of ceil(n / 4)
    float lr[GS_ADAM_MAX_TENSORS];
    int count;
};

__device__ __forceinline__ void adam1(float& p, float g, float& m, float& v, float b1, float b2, float step,
                                      float rbc2, float eps)
{
    m = __builtin_fmaf(b1, m, (1.0f - b1) * g);
    v = __builtin_fmaf(b2, v, (1.0f - b2) * g * g);
    p -= step * m / (sqrtf(v) * rbc2 + eps);
}

__global__ __launch_bounds__(256) void k_adam(AdamList L, float b1, float b2, float eps,
                                              const int* __restrict__ step_dev)
{
    const long long total = L.chunk_off[L.count];
    const long long stride = (long long)gridDim.x * blockDim.x;
    const float t = (float)(*step_dev + 1);
    // 1 - b^t = -expm1(t log1p(b - 1)): b - 1 is exact for b in [0.5, 1], and
    // the form keeps full relative precision for b close to 1 (b2 = 0.999)
    const float bc1 = -expm1f(t * log1pf(b1 - 1.0f));
    const float rbc2 = 1.0f / sqrtf(-expm1f(t * log1pf(b2 - 1.0f)));
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < total; c += stride) {
        int k = 0;
        while (k + 1 < L.count && L.chunk_off[k + 1] <= c) k++;
        const long long i = 4 * (c - L.chunk_off[k]);
        const float step = L.lr[k] / bc1;
        if (i + 4 <= L.n[k]) {
            float4 p = *reinterpret_cast<float4*>(L.p[k] + i);
            const float4 g = *reinterpret_cast<const float4*>(L.g[k] + i);
            float4 m = *reinterpret_cast<float4*>(L.m[k] + i);
            float4 v = *reinterpret_cast<float4*>(L.v[k] + i);
            adam1(p.x, g.x, m.x, v.x, b1, b2, step, rbc2, eps);
            adam1(p.y, g.y, m.y, v.y, b1, b2, step, rbc2, eps);
            adam1(p.z, g.z, m.z, v.z, b1, b2, step, rbc2, eps);
            adam1(p.w, g.w, m.w, v.w, b1, b2, step, rbc2, eps);
            *reinterpret_cast<float4*>(L.p[k] + i) = p;
            *reinterpret_cast<float4*>(L.m[k] + i) = m;
            *reinterpret_cast<float4*>(L.v[k] + i) = v;
        } else {
            for (long long e = i; e < L.n[k]; e++) {
                float p = L.p[k][e], m = L.m[k][e], v = L.v[k][e];
                adam1(p, L.g[k][e], m, v, b1, b2, step, rbc2, eps);
                L.p[k][e] = p;
                L.m[k][e] = m;
                L.v[k][e] = v;
            }
        }
    }
}

__global__ void k_step_advance(int* step_dev) { step_dev[0] += 1; }

}  // namespace

hipError_t launch_adam(int n_tensors, float* const* params, const float* const* grads, float* const* exp_avg,
                       float* const* exp_avg_sq, const int64_t* numel, const float* lrs, float beta1,
                       float beta2, float eps, int* step_dev, hipStream_t st)
{
    AdamList L;
    L.count = n_tensors;
    L.chunk_off[0] = 0;
    for (int k = 0; k < n_tensors; k++) {
        L.p[k] = params[k];
        L.g[k] = grads[k];
        L.m[k] = exp_avg[k];
        L.v[k] = exp_avg_sq[k];
        L.n[k] = numel[k];
        L.lr[k] = lrs[k];
        L.chunk_off[k + 1] = L.chunk_off[k] + (numel[k] + 3) / 4;
    }
    const long long total = L.chunk_off[n_tensors];
    if (total > 0) {
        long long blocks = (total + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, st, L, beta1, beta2, eps, step_dev);
    }
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, st, step_dev);
    return hipGetLastError();
}

}  // namespace gs
