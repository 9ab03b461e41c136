// Fused Adam over the Gaussian parameter tensors (gfx950).
//
// Paper Section 3.2 describes the multi-GPU fused Adam of its backend
// (vectorised loads and stores, transcendentals computed once); the update
// itself is Adam (Kingma and Ba 2015) with bias correction:
//   m <- b1 m + (1 - b1) g,  v <- b2 v + (1 - b2) g^2,
//   p <- p - lr / (1 - b1^t) * m / (sqrt(v) / sqrt(1 - b2^t) + eps).
// One launch updates up to GS_ADAM_MAX_TENSORS tensors, each by its own range
// of blocks (one HBM read of p, g, m, v and one write of p, m, v per element:
// 28 bytes, the algorithmic minimum).  The step count t is
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
    int block_off[GS_ADAM_MAX_TENSORS + 1];   // the blocks of tensor k: [block_off[k], block_off[k + 1])
    float lr[GS_ADAM_MAX_TENSORS];
    int count;
};

// 16-byte chunks a thread handles per loop step (all their loads in flight at once)
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

// Each block updates one tensor (the tensor is uniform per block, so its
// pointers are scalar kernel-argument loads): a grid-stride walk over the
// tensor's whole 16-byte chunks by the tensor's blocks, ADAM_UNROLL chunks
// per thread and step whose loads are unconditional (clamped to the last
// whole chunk) and all in flight together; the n mod 4 trailing elements
// are updated one by one by the tensor's first block.
__global__ __launch_bounds__(256) void k_adam(AdamList L, float b1, float b2, float eps,
                                              const int* __restrict__ step_dev)
{
    int k = 0;
    while (k + 1 < L.count && L.block_off[k + 1] <= (int)blockIdx.x) k++;
    k = __builtin_amdgcn_readfirstlane(k);
    const AdamCoef ac = adam_coef(*step_dev, b1, b2);
    const float rbc2 = ac.rbc2;
    const float step = L.lr[k] * ac.step_scale;
    float* const P = L.p[k];
    const float* const G = L.g[k];
    float* const M = L.m[k];
    float* const V = L.v[k];
    const long long n = L.n[k];
    const long long whole = n / 4;
    const int b = (int)blockIdx.x - L.block_off[k];
    const long long stride = (long long)(L.block_off[k + 1] - L.block_off[k]) * blockDim.x;
    af4* const P4 = reinterpret_cast<af4*>(P);
    const af4* const G4 = reinterpret_cast<const af4*>(G);
    af4* const M4 = reinterpret_cast<af4*>(M);
    af4* const V4 = reinterpret_cast<af4*>(V);
    // every element is read and written once per step: streaming
    // (non-temporal) accesses
    for (long long c0 = (long long)b * blockDim.x + threadIdx.x; c0 < whole; c0 += ADAM_UNROLL * stride) {
        af4 p[ADAM_UNROLL], g[ADAM_UNROLL], m[ADAM_UNROLL], v[ADAM_UNROLL];
#pragma unroll
        for (int u = 0; u < ADAM_UNROLL; u++) {
            const long long c = min(c0 + u * stride, whole - 1);
            p[u] = __builtin_nontemporal_load(P4 + c);
            g[u] = __builtin_nontemporal_load(G4 + c);
            m[u] = __builtin_nontemporal_load(M4 + c);
            v[u] = __builtin_nontemporal_load(V4 + c);
        }
#pragma unroll
        for (int u = 0; u < ADAM_UNROLL; u++) {
            const long long c = c0 + u * stride;
            if (c >= whole) continue;
            adam4(p[u], g[u], m[u], v[u], b1, b2, step, rbc2, eps);
            __builtin_nontemporal_store(p[u], P4 + c);
            __builtin_nontemporal_store(m[u], M4 + c);
            __builtin_nontemporal_store(v[u], V4 + c);
        }
    }
    if (b == 0 && (long long)threadIdx.x < n - 4 * whole) {
        const long long e = 4 * whole + threadIdx.x;
        float pe = P[e], me = M[e], ve = V[e];
        adam_elem(pe, G[e], me, ve, b1, b2, step, rbc2, eps);
        P[e] = pe;
        M[e] = me;
        V[e] = ve;
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
    long long total = 0;
    for (int k = 0; k < n_tensors; k++) {
        L.p[k] = params[k];
        L.g[k] = grads[k];
        L.m[k] = exp_avg[k];
        L.v[k] = exp_avg_sq[k];
        L.n[k] = numel[k];
        L.lr[k] = lrs[k];
        total += (numel[k] + 3) / 4;
    }
    // up to ADAM_MAX_BLOCKS blocks of 256 threads, shared out in proportion
    // to the tensors' chunk counts (at least one per tensor)
    constexpr long long ADAM_MAX_BLOCKS = 8192;
    const long long want = min(ADAM_MAX_BLOCKS, max(1ll, (total + 255) / 256));
    L.block_off[0] = 0;
    for (int k = 0; k < n_tensors; k++) {
        const long long chunks = (numel[k] + 3) / 4;
        const long long nb = max(1ll, min((chunks + 255) / 256, (want * chunks + total - 1) / max(total, 1ll)));
        L.block_off[k + 1] = L.block_off[k] + (int)nb;
    }
    if (total > 0)
        hipLaunchKernelGGL(k_adam, dim3((unsigned)L.block_off[n_tensors]), dim3(256), 0, st, L, beta1, beta2, eps,
                           step_dev);
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_step_advance(step_dev, st);
}

}  // namespace gs
