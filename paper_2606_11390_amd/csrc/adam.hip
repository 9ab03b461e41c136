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
// a captured graph replays successive steps correctly.  The same element
// update (adam_elem) is applied inside the projection backward by
// gs_project_bwd_adam, which then needs no gradient tensors.
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

// chunks a thread handles per loop step (all their loads in flight at once)
constexpr int ADAM_UNROLL = 4;
typedef float af4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void adam4(af4& p, af4 g, af4& m, af4& v, float b1, float b2, float step, float rbc2,
                                      float eps)
{
    float pp[4] = {p.x, p.y, p.z, p.w}, mm[4] = {m.x, m.y, m.z, m.w}, vv[4] = {v.x, v.y, v.z, v.w};
    const float gg[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
    for (int e = 0; e < 4; e++) adam_elem(pp[e], gg[e], mm[e], vv[e], b1, b2, step, rbc2, eps);
    p = af4{pp[0], pp[1], pp[2], pp[3]};
    m = af4{mm[0], mm[1], mm[2], mm[3]};
    v = af4{vv[0], vv[1], vv[2], vv[3]};
}

__device__ __forceinline__ int tensor_of(const AdamList& L, long long c)
{
    int k = 0;
    while (k + 1 < L.count && L.chunk_off[k + 1] <= c) k++;
    return k;
}

__global__ __launch_bounds__(256) void k_adam(AdamList L, float b1, float b2, float eps,
                                              const int* __restrict__ step_dev)
{
    const long long total = L.chunk_off[L.count];
    const long long stride = (long long)gridDim.x * blockDim.x;
    const AdamCoef ac = adam_coef(*step_dev, b1, b2);
    const float rbc2 = ac.rbc2;
    // every element is read and written once per step: streaming
    // (non-temporal) accesses; ADAM_UNROLL chunks c, c + stride, ... per
    // thread and step, so that 4 x ADAM_UNROLL 16-byte loads are in flight
    for (long long c0 = (long long)blockIdx.x * blockDim.x + threadIdx.x; c0 < total;
         c0 += ADAM_UNROLL * stride) {
        af4 p[ADAM_UNROLL], g[ADAM_UNROLL], m[ADAM_UNROLL], v[ADAM_UNROLL];
        int kk[ADAM_UNROLL];
        long long ii[ADAM_UNROLL];
        bool full[ADAM_UNROLL];
#pragma unroll
        for (int u = 0; u < ADAM_UNROLL; u++) {
            const long long c = c0 + u * stride;
            const int k = c < total ? tensor_of(L, c) : 0;
            const long long i = 4 * (c - L.chunk_off[k]);
            kk[u] = k;
            ii[u] = i;
            full[u] = c < total && i + 4 <= L.n[k];
            if (full[u]) {
                p[u] = __builtin_nontemporal_load(reinterpret_cast<const af4*>(L.p[k] + i));
                g[u] = __builtin_nontemporal_load(reinterpret_cast<const af4*>(L.g[k] + i));
                m[u] = __builtin_nontemporal_load(reinterpret_cast<const af4*>(L.m[k] + i));
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const af4*>(L.v[k] + i));
            }
        }
#pragma unroll
        for (int u = 0; u < ADAM_UNROLL; u++) {
            const long long c = c0 + u * stride;
            if (c >= total) continue;
            const int k = kk[u];
            const long long i = ii[u];
            const float step = L.lr[k] * ac.step_scale;
            if (full[u]) {
                adam4(p[u], g[u], m[u], v[u], b1, b2, step, rbc2, eps);
                __builtin_nontemporal_store(p[u], reinterpret_cast<af4*>(L.p[k] + i));
                __builtin_nontemporal_store(m[u], reinterpret_cast<af4*>(L.m[k] + i));
                __builtin_nontemporal_store(v[u], reinterpret_cast<af4*>(L.v[k] + i));
            } else {
                // the ragged tail of a tensor, element by element
                for (long long e = i; e < L.n[k]; e++) {
                    float pe = L.p[k][e], me = L.m[k][e], ve = L.v[k][e];
                    adam_elem(pe, L.g[k][e], me, ve, b1, b2, step, rbc2, eps);
                    L.p[k][e] = pe;
                    L.m[k][e] = me;
                    L.v[k][e] = ve;
                }
            }
        }
    }
}

__global__ void k_step_advance(int* step_dev) { step_dev[0] += 1; }

}  // namespace

hipError_t launch_step_advance(int* step_dev, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, st, step_dev);
    return hipGetLastError();
}

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
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_step_advance(step_dev, st);
}

}  // namespace gs
